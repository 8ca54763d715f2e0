// Exported C ABI: argument validation, context and workspace management, and
// the synchronous calls that report device-side status through firal_info.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "common.h"

namespace firal {

static thread_local char g_last_error[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
}

int relax_step_launch(Ctx* x, double* w, double b, double lambda, double beta0, uint64_t seed,
                      int t, int s, double tol, int max_iter, uint32_t flags, double* g_out,
                      hipStream_t st);
int objective_launch(Ctx* x, const double* z, double lambda, const void* V, int s, double tol,
                     int max_iter, uint32_t flags, double* g, hipStream_t st);

#define FIRAL_REQ(cond, ...)                                                    \
  do {                                                                          \
    if (!(cond)) {                                                              \
      ::firal::set_error(__VA_ARGS__);                                          \
      return FIRAL_EINVAL;                                                      \
    }                                                                           \
  } while (0)

typedef std::vector<std::pair<hipEvent_t, hipEvent_t>> EventPairs;

static void drop_events(Ctx* x) {
  if (!x->prof_events) return;
  EventPairs* ev = (EventPairs*)x->prof_events;
  for (auto& e : *ev) {
    if (e.first) (void)hipEventDestroy(e.first);
    if (e.second) (void)hipEventDestroy(e.second);
  }
  delete ev;
  x->prof_events = nullptr;
}

int prof_pair(Ctx* x, int kernel, hipEvent_t* e0, hipEvent_t* e1) {
  *e0 = *e1 = nullptr;
  if (!x->profiling || kernel != x->prof_kernel) return FIRAL_OK;
  EventPairs* ev = (EventPairs*)x->prof_events;
  ev->push_back({nullptr, nullptr});
  FIRAL_HIP(hipEventCreate(&ev->back().first));
  FIRAL_HIP(hipEventCreate(&ev->back().second));
  *e0 = ev->back().first;
  *e1 = ev->back().second;
  return FIRAL_OK;
}

static void free_ctx(Ctx* x) {
  drop_events(x);
  void* bufs[] = {x->G, x->gpart, x->part, x->fused_part, x->Xhi, x->Xlo, x->XThi, x->XTlo,
                  x->XTf, x->HTf, x->VTf, x->ntpart, x->P, x->Pinv, x->syrk_part, x->syrk_tiles, x->V, x->W1, x->Y,
                  x->W2, x->cx, x->cgd, x->cr, x->cz, x->cp, x->cq, x->mean, x->omega, x->gbuf, x->ebuf,
                  x->colpart, x->rho, x->bnorm, x->alpha, x->beta, x->relres, x->done,
                  x->redpart, x->status, x->t_dev};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (x->status_host) (void)hipHostFree(x->status_host);
  if (x->chk_word) (void)hipHostFree(x->chk_word);
  delete x;
}

static int dmalloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes ? bytes : 16);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    set_error("hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    return FIRAL_ENOMEM;
  }
  return FIRAL_OK;
}

static int check_common(firal_ctx ctx, int32_t s) {
  FIRAL_REQ(ctx != nullptr, "null context");
  FIRAL_REQ(s >= 1 && s <= C(ctx)->s_max, "s = %d outside [1, s_max = %d]", s, C(ctx)->s_max);
  return FIRAL_OK;
}

static int finish_sync(Ctx* x, hipStream_t st) {
  FIRAL_HIP(hipMemcpyAsync(x->status_host, x->status, sizeof(Status), hipMemcpyDeviceToHost, st));
  FIRAL_HIP(hipStreamSynchronize(st));
  return FIRAL_OK;
}

}  // namespace firal

using namespace firal;

extern "C" {

const char* firal_strerror(int code) {
  switch (code) {
    case FIRAL_OK: return "success";
    case FIRAL_WARN_NOT_CONVERGED: return "PCG did not converge within max_iter";
    case FIRAL_EINVAL: return "invalid argument";
    case FIRAL_EHIP: return "HIP runtime failure or no usable device";
    case FIRAL_ENOMEM: return "device allocation failed";
    case FIRAL_ENOTSUP: return "not supported";
    case FIRAL_EBREAKDOWN: return "PCG breakdown: operator not positive definite on a column";
    case FIRAL_ENOTSPD: return "preconditioner block not positive definite";
    default: return "unknown return code";
  }
}

const char* firal_last_error(void) { return g_last_error; }

int firal_profile_begin(firal_ctx ctx, int32_t kernel) {
  FIRAL_REQ(ctx != nullptr, "null context");
  FIRAL_REQ(kernel >= FIRAL_PROF_PRODUCT && kernel <= FIRAL_PROF_ROUND_SCORE,
            "unknown kernel %d", kernel);
  Ctx* x = C(ctx);
  drop_events(x);
  x->prof_events = new EventPairs();
  x->prof_kernel = kernel;
  x->profiling = 1;
  return FIRAL_OK;
}

int firal_profile_end(firal_ctx ctx, double* total_ms, int64_t* launches) {
  FIRAL_REQ(ctx != nullptr, "null context");
  Ctx* x = C(ctx);
  FIRAL_REQ(x->profiling && x->prof_events, "profiling was not begun");
  x->profiling = 0;
  FIRAL_HIP(hipDeviceSynchronize());
  EventPairs* ev = (EventPairs*)x->prof_events;
  double sum = 0.0;
  int64_t n = 0;
  for (auto& e : *ev) {
    if (!e.first || !e.second) continue;
    float ms = 0.f;
    FIRAL_HIP(hipEventElapsedTime(&ms, e.first, e.second));
    sum += ms;
    ++n;
  }
  drop_events(x);
  if (total_ms) *total_ms = sum;
  if (launches) *launches = n;
  return FIRAL_OK;
}

int firal_create(firal_ctx* out, int64_t n_pool, int64_t n_lab, int32_t d, int32_t c,
                 int32_t s_max, int32_t prec, const void* X, const void* H, void* stream) {
  FIRAL_REQ(out != nullptr, "null output pointer");
  *out = nullptr;
  FIRAL_REQ(n_pool >= 1, "n_pool = %lld < 1", (long long)n_pool);
  FIRAL_REQ(n_lab >= 0, "n_lab = %lld < 0", (long long)n_lab);
  FIRAL_REQ(d >= 1 && d <= 4096, "d = %d outside [1, 4096]", d);
  FIRAL_REQ(c >= 2 && c <= 65536, "c = %d outside [2, 65536]", c);
  FIRAL_REQ(s_max >= 1 && s_max <= 4096, "s_max = %d outside [1, 4096]", s_max);
  FIRAL_REQ(prec == FIRAL_F64 || prec == FIRAL_F32 || prec == FIRAL_BF16X3, "unknown precision %d",
            prec);
  FIRAL_REQ(X != nullptr && H != nullptr, "null X or H");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    set_error("no HIP device available (%s)", e != hipSuccess ? hipGetErrorString(e) : "0 devices");
    return FIRAL_EHIP;
  }
  Ctx* x = new (std::nothrow) Ctx();
  if (!x) {
    set_error("host allocation failed");
    return FIRAL_ENOMEM;
  }
  std::memset(x, 0, sizeof(Ctx));
  x->n_pool = n_pool;
  x->n_lab = n_lab;
  x->N = n_pool + n_lab;
  x->d = d;
  x->c = c;
  x->s_max = s_max;
  x->prec = prec;
  x->esize = prec == FIRAL_F64 ? 8 : 4;
  x->X = X;
  x->H = H;
  if (hipGetDevice(&x->device) != hipSuccess ||
      hipDeviceGetAttribute(&x->n_cu, hipDeviceAttributeMultiprocessorCount, x->device) !=
          hipSuccess) {
    delete x;
    set_error("hipGetDevice / hipDeviceGetAttribute failed");
    return FIRAL_EHIP;
  }
  const int64_t blk = (int64_t)d * s_max * c;        // elements per block
  const int64_t sc = (int64_t)s_max * c;
  // row-chunked intermediate: one (rows x s*c) buffer within ~2 GiB
  const int64_t budget = (int64_t)2 << 30;
  int64_t rows = budget / (sc * (int64_t)x->esize);
  rows = std::max<int64_t>(128, std::min<int64_t>(rows, x->N));
  if (const char* env = getenv("FIRAL_CHUNK_ROWS")) {   // smaller chunks, for tests of the chunked path
    const long long v = atoll(env);
    if (v >= 1 && v < rows) rows = v;
  }
  // bf16x3: chunks start on multiples of 32 rows (the X^T planes are read 8 rows at a time);
  // the wide FP32 path reads its transposed operands 4 rows at a time from 32-row stages
  const char* nt_env = getenv("FIRAL_NT");
  x->use_nt = nt_applies(x) && !(nt_env && atoi(nt_env) == 0);
  if (prec == FIRAL_BF16X3 || x->use_nt) rows = std::max<int64_t>(32, rows - rows % 32);
  x->chunk_rows = rows;
  const int64_t tiles = tiled_out_tiles(prec, d, sc);
  x->max_splits = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(4096, tiles), 64));

  std::vector<int32_t> syrk_tiles;
  // the preconditioner's Gram kernel.  Its bf16x3 form (an opt-in of BF16X3 contexts) leaves
  // ~1e-5 relative error in the blocks: no change to a solve run to a tolerance, but PCG iterates
  // taken at a fixed iteration count move with it
  x->gram_form = gram_form_for(prec, d, c, X);
  syrk_plan(prec, d, c, x->gram_form, x->n_cu, &syrk_tiles, &x->syrk_splits);
  x->syrk_ntiles = (int)(syrk_tiles.size() / 2);
  x->col_parts = (int)std::max<int64_t>(1, std::min<int64_t>(d, cdiv(256, s_max)));
  x->red_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(n_pool, 256), 1024));

  const char* unf = getenv("FIRAL_UNFUSED");
  x->force_tiled = x->force_multik = unf && atoi(unf) != 0;
  // fused tile width in 16-column blocks per wave: FP32 1 (the next row chunk fetched ahead),
  // bf16x3 2 (its X planes are read once per chunk instead of once per column tile); the
  // faster of the two measured at configuration 2 for each
  const char* ncb = getenv("FIRAL_FUSED_MAX_NCB");
  x->fused_max_ncb = ncb ? (atoi(ncb) == 2 ? 2 : 1) : (prec == FIRAL_BF16X3 ? 2 : 1);
  // BF16X3 PCG: switch to FP32 products below this relative residual (0 = never).  With the
  // residual kept in the projected space the split products converge like FP32 ones, so
  // the switch is off unless asked for.
  const char* sw = getenv("FIRAL_BF3_SWITCH");
  x->bf3_switch = sw ? atof(sw) : 0.0;
  const char* wgs = getenv("FIRAL_FUSED_WGS");
  x->fused_wgs = wgs ? std::min(std::max(atoi(wgs), 1), kFusedMaxWgs) : 256;
  x->fused_part_elems = 0;
  const int ncb_set = x->fused_max_ncb, wgs_set = x->fused_wgs;
  for (int ncb_try = 1; ncb_try <= 2; ++ncb_try) {   // room for every tile shape the tuner tries
    for (int wgs_try : {wgs_set, kFusedMaxWgs}) {
      x->fused_max_ncb = ncb_try;
      x->fused_wgs = wgs_try;
      for (int s = 1; s <= s_max; ++s) {
        for (int precise = 0; precise < 2; ++precise) {
          FusedPlan fp;
          if (fused_plan(x, s, x->N, &fp, precise != 0))
            x->fused_part_elems = std::max(x->fused_part_elems, fp.part_elems);
        }
      }
    }
  }
  x->fused_max_ncb = ncb_set;
  x->fused_wgs = wgs_set;

  const size_t es = x->esize;
  int rc = FIRAL_OK;
#define ALLOC(ptr, bytes)                                          \
  if (rc == FIRAL_OK) rc = dmalloc((void**)&(ptr), (size_t)(bytes))
  ALLOC(x->G, rows * sc * es);
  ALLOC(x->gpart, std::min<int64_t>(rows, n_pool) * tiled_col_tiles(prec, c, s_max) * 8);
  ALLOC(x->part, (int64_t)x->max_splits * blk * es);
  ALLOC(x->fused_part, x->fused_part_elems * 4);
  ALLOC(x->P, (int64_t)c * d * d * 8);
  ALLOC(x->Pinv, (int64_t)c * d * d * 8);
  ALLOC(x->syrk_part, (int64_t)x->syrk_splits * c * d * d * es);
  ALLOC(x->syrk_tiles, syrk_tiles.size() * sizeof(int32_t));
  if (x->use_nt) {
    x->ldn = nt_ld(x->N);
    const int64_t ldg = nt_ld(rows), nw = nt_windows(c);
    if (prec == FIRAL_F32) ALLOC(x->XTf, x->ldn * d * 4);
    ALLOC(x->HTf, x->ldn * c * 4);
    if (prec != FIRAL_BF16X3) ALLOC(x->VTf, blk * 4);
    ALLOC(x->ntpart, ((int64_t)s_max * nw * ldg + (int64_t)s_max * ldg) * 4);
  }
  if (prec == FIRAL_BF16X3) {
    // hi/lo planes of V^T for two probe blocks (the gradient's U and W; products use the first)
    ALLOC(x->VTf, blk * 8);
    x->ldt = cdiv(x->N, 8) * 8;
    ALLOC(x->Xhi, x->N * d * 2);
    ALLOC(x->Xlo, x->N * d * 2);
    ALLOC(x->XThi, x->ldt * d * 2);
    ALLOC(x->XTlo, x->ldt * d * 2);
  }
  ALLOC(x->V, blk * es);
  ALLOC(x->W1, blk * es);
  ALLOC(x->Y, blk * es);
  ALLOC(x->W2, blk * es);
  ALLOC(x->cx, blk * es);
  if (col_cg_scratch(d, c, s_max) > 0) ALLOC(x->cgd, col_cg_scratch(d, c, s_max) * 8);
  ALLOC(x->cr, blk * es);
  ALLOC(x->cz, blk * es);
  ALLOC(x->cp, blk * es);
  ALLOC(x->cq, blk * es);
  ALLOC(x->mean, (int64_t)d * s_max * 8);
  ALLOC(x->omega, x->N * 8);
  ALLOC(x->gbuf, n_pool * 8);
  ALLOC(x->ebuf, n_pool * 8);
  ALLOC(x->colpart, (int64_t)4 * s_max * x->col_parts * 8);
  ALLOC(x->rho, s_max * 8);
  ALLOC(x->bnorm, s_max * 8);
  ALLOC(x->alpha, s_max * 8);
  ALLOC(x->beta, s_max * 8);
  ALLOC(x->relres, s_max * 8);
  ALLOC(x->done, 2 * s_max * 4);   // two flag buffers (column-local CG)
  ALLOC(x->redpart, (3 * (int64_t)x->red_blocks + 1) * 8);
  ALLOC(x->status, sizeof(Status));
  ALLOC(x->t_dev, sizeof(int32_t));
#undef ALLOC
  if (rc == FIRAL_OK) {
    hipError_t he = hipHostMalloc((void**)&x->status_host, sizeof(Status), hipHostMallocDefault);
    if (he != hipSuccess) {
      set_error("hipHostMalloc failed: %s", hipGetErrorString(he));
      rc = FIRAL_ENOMEM;
    }
    // check-point words written by the PCG kernels and polled by the host (zero: no tag)
    if (rc == FIRAL_OK &&
        (hipHostMalloc((void**)&x->chk_word, 2 * (size_t)s_max * sizeof(uint32_t),
                       hipHostMallocCoherent) != hipSuccess ||
         hipHostGetDevicePointer((void**)&x->chk_word_dev, x->chk_word, 0) != hipSuccess)) {
      (void)hipGetLastError();
      set_error("pinned check-point words could not be allocated or mapped");
      rc = FIRAL_ENOMEM;
    }
    if (rc == FIRAL_OK) std::memset(x->chk_word, 0, 2 * (size_t)s_max * sizeof(uint32_t));
  }
  if (rc == FIRAL_OK) {
    hipStream_t st = (hipStream_t)stream;
    if (hipMemsetAsync(x->status, 0, sizeof(Status), st) != hipSuccess ||
        hipMemcpyAsync(x->syrk_tiles, syrk_tiles.data(), syrk_tiles.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        (prec == FIRAL_BF16X3 && split_x_launch(x, st) != FIRAL_OK) ||
        (x->use_nt && nt_prepare_ctx(x, st) != FIRAL_OK) ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("status initialisation failed");
      rc = FIRAL_EHIP;
    }
  }
  if (rc != FIRAL_OK) {
    free_ctx(x);
    return rc;
  }
  *out = reinterpret_cast<firal_ctx>(x);
  return FIRAL_OK;
}

int firal_destroy(firal_ctx ctx) {
  if (!ctx) return FIRAL_OK;
  (void)hipDeviceSynchronize();
  free_ctx(C(ctx));
  return FIRAL_OK;
}

int firal_hvp(firal_ctx ctx, const double* omega, int64_t n_rows, double shift, const void* B,
              void* out, int32_t s, void* stream) {
  FIRAL_CHECK(check_common(ctx, s));
  Ctx* x = C(ctx);
  FIRAL_REQ(B != nullptr && out != nullptr, "null B or out");
  FIRAL_REQ(B != out, "out must not alias B");
  FIRAL_REQ(n_rows >= 0 && n_rows <= x->N, "n_rows = %lld outside [0, %lld]", (long long)n_rows,
            (long long)x->N);
  return hvp_launch(x, omega, n_rows, shift, B, out, s, skip_none(), (hipStream_t)stream);
}

int firal_build_precond(firal_ctx ctx, const double* omega, double shift, double* L, double* Pinv,
                        firal_info* info, void* stream) {
  FIRAL_REQ(ctx != nullptr, "null context");
  Ctx* x = C(ctx);
  hipStream_t st = (hipStream_t)stream;
  FIRAL_CHECK(precond_launch(x, omega, shift, st, L != nullptr));
  const size_t bytes = (size_t)x->c * x->d * x->d * 8;
  if (L) FIRAL_HIP(hipMemcpyAsync(L, x->P, bytes, hipMemcpyDeviceToDevice, st));
  if (Pinv) FIRAL_HIP(hipMemcpyAsync(Pinv, x->Pinv, bytes, hipMemcpyDeviceToDevice, st));
  FIRAL_CHECK(finish_sync(x, st));
  const int bad = x->status_host->bad_block == INT_MAX ? -1 : x->status_host->bad_block;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->bad_block = bad;
  }
  if (bad >= 0) {
    set_error("preconditioner block %d is not positive definite", bad);
    return FIRAL_ENOTSPD;
  }
  return FIRAL_OK;
}

__global__ void k_pcg_reset(Status* st) {
  st->converged = 1;
  st->breakdown = 0;
  st->bad_block = INT_MAX;
}

int firal_pcg_solve(firal_ctx ctx, const double* omega, double shift, const double* Pinv,
                    const void* B, void* Xsol, int32_t s, double tol, int32_t max_iter,
                    uint32_t flags, firal_info* info, void* stream) {
  FIRAL_CHECK(check_common(ctx, s));
  Ctx* x = C(ctx);
  FIRAL_REQ(Pinv != nullptr && B != nullptr && Xsol != nullptr, "null Pinv, B or Xsol");
  FIRAL_REQ(tol >= 0.0, "tol < 0");
  FIRAL_REQ(max_iter >= 0, "max_iter < 0");
  FIRAL_REQ((flags & ~FIRAL_PCG_PROJECT) == 0, "unknown flags 0x%x", flags);
  hipStream_t st = (hipStream_t)stream;
  k_pcg_reset<<<1, 1, 0, st>>>(x->status);
  FIRAL_LAUNCHED();
  FIRAL_CHECK(pcg_launch(x, omega, shift, Pinv, B, Xsol, s, tol, max_iter, flags, 0, st));
  FIRAL_CHECK(finish_sync(x, st));
  const Status& h = *x->status_host;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->cg_iters[0] = h.cg_iters[0];
    info->converged = h.converged;
    info->bad_block = -1;
    info->relres_max = h.relres_max;
  }
  if (h.breakdown) {
    set_error("PCG breakdown (p^T q <= 0)");
    return FIRAL_EBREAKDOWN;
  }
  return h.converged ? FIRAL_OK : FIRAL_WARN_NOT_CONVERGED;
}

int firal_grad_z(firal_ctx ctx, const void* U, const void* W, int32_t s, double* g, void* stream) {
  FIRAL_CHECK(check_common(ctx, s));
  FIRAL_REQ(U != nullptr && W != nullptr && g != nullptr, "null U, W or g");
  return grad_launch(C(ctx), U, W, s, g, (hipStream_t)stream);
}

int firal_probes(firal_ctx ctx, uint64_t seed, int32_t t, int32_t s, void* V, void* stream) {
  FIRAL_CHECK(check_common(ctx, s));
  FIRAL_REQ(V != nullptr, "null V");
  FIRAL_REQ(t >= 1, "t = %d < 1", t);
  return probes_launch(C(ctx), seed, t, s, V, (hipStream_t)stream);
}

int firal_sampled_objective(firal_ctx ctx, const double* z, double lambda, const void* V,
                            int32_t s, double tol, int32_t max_iter, uint32_t flags, double* f,
                            double* g, firal_info* info, void* stream) {
  FIRAL_CHECK(check_common(ctx, s));
  Ctx* x = C(ctx);
  FIRAL_REQ(z != nullptr && V != nullptr && f != nullptr, "null z, V or f");
  FIRAL_REQ(lambda >= 0.0, "lambda < 0");
  FIRAL_REQ(tol >= 0.0, "tol < 0");
  FIRAL_REQ(max_iter >= 0, "max_iter < 0");
  FIRAL_REQ((flags & ~FIRAL_PCG_PROJECT) == 0, "unknown flags 0x%x", flags);
  hipStream_t st = (hipStream_t)stream;
  FIRAL_CHECK(objective_launch(x, z, lambda, V, s, tol, max_iter, flags, g, st));
  FIRAL_CHECK(finish_sync(x, st));
  const Status& h = *x->status_host;
  const int bad = h.bad_block == INT_MAX ? -1 : h.bad_block;
  *f = h.f_hat;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->cg_iters[0] = h.cg_iters[0];
    info->cg_iters[1] = h.cg_iters[1];
    info->converged = h.converged;
    info->bad_block = bad;
    info->relres_max = h.relres_max;
    info->f_hat = h.f_hat;
  }
  if (bad >= 0) {
    set_error("preconditioner block %d is not positive definite", bad);
    return FIRAL_ENOTSPD;
  }
  if (h.breakdown) {
    set_error("PCG breakdown (p^T q <= 0)");
    return FIRAL_EBREAKDOWN;
  }
  return h.converged ? FIRAL_OK : FIRAL_WARN_NOT_CONVERGED;
}

// The status of the Relax iteration that finish_sync has just read back, as firal_info and a
// return code (ENOTSPD, EBREAKDOWN, WARN_NOT_CONVERGED or OK).
static int step_result(Ctx* x, firal_info* info) {
  const Status& h = *x->status_host;
  const int bad = h.bad_block == INT_MAX ? -1 : h.bad_block;
  if (info) {
    info->cg_iters[0] = h.cg_iters[0];
    info->cg_iters[1] = h.cg_iters[1];
    info->converged = h.converged;
    info->bad_block = bad;
    info->relres_max = h.relres_max;
    info->f_hat = h.f_hat;
    info->g_absmax = h.g_absmax;
    info->beta = h.beta;
  }
  if (bad >= 0) {
    set_error("preconditioner block %d is not positive definite", bad);
    return FIRAL_ENOTSPD;
  }
  if (h.breakdown) {
    set_error("PCG breakdown (p^T q <= 0)");
    return FIRAL_EBREAKDOWN;
  }
  return h.converged ? FIRAL_OK : FIRAL_WARN_NOT_CONVERGED;
}

static int check_step_args(firal_ctx ctx, double b, double lambda, int32_t s, double tol,
                           int32_t max_iter, uint32_t flags) {
  FIRAL_CHECK(check_common(ctx, s));
  FIRAL_REQ(b > 0.0, "b must be > 0");
  FIRAL_REQ(lambda >= 0.0, "lambda < 0");
  FIRAL_REQ(tol >= 0.0, "tol < 0");
  FIRAL_REQ(max_iter >= 0, "max_iter < 0");
  FIRAL_REQ((flags & ~FIRAL_PCG_PROJECT) == 0, "unknown flags 0x%x", flags);
  return FIRAL_OK;
}

double firal_default_beta0(int64_t n, int32_t T) {
  if (n < 1) return 0.0;
  return std::sqrt(2.0 * std::log((double)n) / (double)std::max<int32_t>(T, 1));
}

int firal_relax_step(firal_ctx ctx, double* w, double b, double lambda, double beta0,
                     uint64_t seed, int32_t t, int32_t s, double tol, int32_t max_iter,
                     uint32_t flags, double* g_out, firal_info* info, void* stream) {
  FIRAL_CHECK(check_step_args(ctx, b, lambda, s, tol, max_iter, flags));
  Ctx* x = C(ctx);
  FIRAL_REQ(w != nullptr, "null w");
  FIRAL_REQ(beta0 >= 0.0, "beta0 < 0");
  FIRAL_REQ(t >= 1, "t = %d < 1", t);
  hipStream_t st = (hipStream_t)stream;
  FIRAL_CHECK(relax_step_launch(x, w, b, lambda, beta0, seed, t, s, tol, max_iter, flags, g_out, st));
  FIRAL_CHECK(finish_sync(x, st));
  return step_result(x, info);
}

int firal_relax_solve(firal_ctx ctx, double b, double lambda, double beta0, uint64_t seed,
                      int32_t T, int32_t s, double tol, int32_t max_iter, uint32_t flags,
                      double stop_rel, double* z, double* f_hist, int32_t* cg_hist,
                      int32_t* iters, firal_info* info, void* stream) {
  FIRAL_CHECK(check_step_args(ctx, b, lambda, s, tol, max_iter, flags));
  Ctx* x = C(ctx);
  FIRAL_REQ(z != nullptr, "null z");
  FIRAL_REQ(T >= 1, "T = %d < 1", T);
  FIRAL_REQ(stop_rel >= 0.0, "stop_rel < 0");
  FIRAL_REQ(!(beta0 != beta0), "beta0 is NaN");
  if (beta0 < 0.0) beta0 = firal_default_beta0(x->n_pool, T);
  if (iters) *iters = 0;
  hipStream_t st = (hipStream_t)stream;
  // z holds the simplex weights w while the iterations run (w^0 = 1/n), then b w
  FIRAL_CHECK(fill_scale_launch(z, x->n_pool, 1.0 / (double)x->n_pool, false, st));
  int rc_all = FIRAL_OK;
  double f_prev = 0.0;
  firal_info last;
  std::memset(&last, 0, sizeof(last));
  int conv_all = 1;
  for (int32_t t = 1; t <= T; ++t) {
    FIRAL_CHECK(relax_step_launch(x, z, b, lambda, beta0, seed, t, s, tol, max_iter, flags,
                                  nullptr, st));
    FIRAL_CHECK(finish_sync(x, st));
    const int rc = step_result(x, &last);
    if (rc < 0) {   // the failed iteration left w unchanged
      if (info) *info = last;
      FIRAL_CHECK(fill_scale_launch(z, x->n_pool, b, true, st));
      FIRAL_HIP(hipStreamSynchronize(st));
      return rc;
    }
    if (rc == FIRAL_WARN_NOT_CONVERGED) rc_all = rc;
    conv_all &= last.converged;
    if (f_hist) f_hist[t - 1] = last.f_hat;
    if (cg_hist) {
      cg_hist[2 * (t - 1)] = last.cg_iters[0];
      cg_hist[2 * (t - 1) + 1] = last.cg_iters[1];
    }
    if (iters) *iters = t;
    const bool stop = stop_rel > 0.0 && t >= 2 &&
                      std::fabs(last.f_hat - f_prev) <= stop_rel * std::fabs(f_prev);
    f_prev = last.f_hat;
    if (stop) break;
  }
  FIRAL_CHECK(fill_scale_launch(z, x->n_pool, b, true, st));
  FIRAL_HIP(hipStreamSynchronize(st));
  if (info) {
    *info = last;
    info->converged = conv_all;
  }
  return rc_all;
}

}  // extern "C"
