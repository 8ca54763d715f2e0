// Many independent Relax problems (uneven n, d, c) advanced together, and the tuner that picks
// each problem's kernel variants.
//
// A batch captures one Relax iteration (Algorithm 2) of every problem into a single HIP graph:
// problem i is enqueued on a stream of its own that forks from and joins back into the
// capture stream, so the graph holds one independent branch per problem and the runtime runs
// the branches side by side, filling the GPU with problems too small to fill it alone.  Each
// branch is the library's ordinary step in its capture-safe form: no host reads (PCG runs a
// fixed number of iterations whose kernels return at once after convergence), no memset
// nodes, and the iteration index t read from and advanced in device memory, so one graph
// replayed T times runs iterations t0 .. t0 + T - 1 of every problem.
//
// The tuner times, on the problem itself, the candidate product tilings (the fused single pass
// with one or two 16-column blocks per wave and 256, 512 or 1024 workgroups, i.e. rows per
// workgroup, wherever its plan fits; or the row-tiled kernels) and PCG step forms
// (column-local or separate kernels), keeps the fastest of each, and remembers the choice per
// bucket (precision, d, c, s, n rounded to a power of two) for the process.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.h"

namespace firal {

int pcg_launch(Ctx* x, const double* omega, double shift, const double* Pinv, const void* B,
               void* Xsol, int s, double tol, int max_iter, uint32_t flags, int slot,
               hipStream_t st);

namespace {

typedef std::tuple<int, int, int, int, int> TuneKey;   // prec, d, c, s, log2 N bucket

std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;   // choice bits: 1 = row-tiled product, 2 = separate-kernel
                                 // PCG, 4 = fused product with two column blocks per wave,
                                 // bits 3-4 = fused workgroup target (256 << code)

TuneKey tune_key(const Ctx* x, int s) {
  const int nb = (int)std::ceil(std::log2((double)std::max<int64_t>(x->N, 1)));
  return TuneKey(x->prec, x->d, x->c, s, nb);
}

void apply_choice(Ctx* x, int choice) {
  x->force_tiled = (choice & 1) != 0;
  x->force_multik = (choice & 2) != 0;
  x->fused_max_ncb = (choice & 4) ? 2 : 1;
  x->fused_wgs = 256 << ((choice >> 3) & 3);
}

// Milliseconds per call of fn (after one untimed call), events on st.
template <typename F>
int time_ms(F fn, int reps, hipStream_t st, double* ms) {
  hipEvent_t e0, e1;
  FIRAL_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("hipEventCreate failed");
    return FIRAL_EHIP;
  }
  int rc = fn();
  if (rc >= 0) rc = hipEventRecord(e0, st) == hipSuccess ? FIRAL_OK : FIRAL_EHIP;
  for (int i = 0; i < reps && rc >= 0; ++i) rc = fn();
  if (rc >= 0) rc = hipEventRecord(e1, st) == hipSuccess ? FIRAL_OK : FIRAL_EHIP;
  if (rc >= 0) rc = hipEventSynchronize(e1) == hipSuccess ? FIRAL_OK : FIRAL_EHIP;
  float t = 0.f;
  if (rc >= 0) rc = hipEventElapsedTime(&t, e0, e1) == hipSuccess ? FIRAL_OK : FIRAL_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == FIRAL_EHIP) set_error("event timing failed");
  *ms = t / std::max(reps, 1);
  return rc;
}

}  // namespace

// Time the variants on this context (its V, W1, Y, P and Pinv buffers are overwritten) and set
// its choice; a bucket already tuned in this process is applied without timing.
int autotune(Ctx* x, int s, hipStream_t st, int* choice_out) {
  const TuneKey key = tune_key(x, s);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      apply_choice(x, it->second);
      if (choice_out) *choice_out = it->second;
      return FIRAL_OK;
    }
  }
  FIRAL_CHECK(probes_launch(x, 1, 1, s, x->V, st));
  // product: the default path (the fused kernel's first tiling where its plan fits, else the
  // wide or row-tiled kernels the context chose), the other fused tilings whose plans fit
  // (distinct plans only: the row ranges are capped by the row chunks), then the row-tiled
  // kernels
  std::vector<int> cands{0};
  std::vector<std::pair<int, int>> plans;   // (column blocks per wave, row ranges)
  for (int ncb_bit = 0; ncb_bit <= 4; ncb_bit += 4)
    for (int code = 0; (256 << code) <= kFusedMaxWgs; ++code) {
      const int bits = ncb_bit | (code << 3);
      apply_choice(x, bits);
      FusedPlan fp;
      if (!fused_plan(x, s, x->N, &fp, false) || fp.part_elems > x->fused_part_elems) continue;
      const std::pair<int, int> key(fp.ncb, fp.n_splits);
      if (std::find(plans.begin(), plans.end(), key) != plans.end()) continue;
      plans.push_back(key);
      if (bits != 0) cands.push_back(bits);
    }
  cands.push_back(1);
  double best = 0.0;
  int prod = cands[0];
  for (size_t v = 0; v < cands.size(); ++v) {
    apply_choice(x, cands[v]);
    double t = 0.0;
    FIRAL_CHECK(time_ms([&] { return hvp_launch(x, nullptr, x->N, 1e-3, x->V, x->W1, s,
                                                skip_none(), st); },
                        3, st, &t));
    if (v == 0 || t < best) {
      best = t;
      prod = cands[v];
    }
  }
  apply_choice(x, prod);
  // PCG step: column-local against separate kernels, 4 fixed iterations each
  FIRAL_CHECK(precond_launch(x, nullptr, 1e-3, st));
  double t_cg[2] = {0.0, 0.0};
  for (int v = 0; v < 2; ++v) {
    apply_choice(x, prod | (v << 1));
    FIRAL_CHECK(time_ms([&] { return pcg_launch(x, nullptr, 1e-3, x->Pinv, x->V, x->W1, s, 0.0,
                                                4, FIRAL_PCG_PROJECT, 0, st); },
                        2, st, &t_cg[v]));
  }
  const int multik = t_cg[1] < t_cg[0] ? 1 : 0;
  const int choice = prod | (multik << 1);
  apply_choice(x, choice);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = choice;
  }
  if (choice_out) *choice_out = choice;
  return FIRAL_OK;
}

struct Batch {
  int n = 0;
  int device = 0;
  std::vector<firal_batch_problem> probs;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> joins;
  hipStream_t cap = nullptr;
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void free_batch(Batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipEvent_t e : b->joins)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipStream_t s : b->streams)
    if (s) (void)hipStreamDestroy(s);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

}  // namespace firal

using namespace firal;

extern "C" int firal_autotune(firal_ctx ctx, int32_t s, int32_t* choice, void* stream) {
  if (!ctx) {
    set_error("firal_autotune: null context");
    return FIRAL_EINVAL;
  }
  Ctx* x = C(ctx);
  if (s < 1 || s > x->s_max) {
    set_error("firal_autotune: s = %d outside [1, %d]", s, x->s_max);
    return FIRAL_EINVAL;
  }
  int ch = 0;
  FIRAL_CHECK(autotune(x, s, (hipStream_t)stream, &ch));
  FIRAL_HIP(hipStreamSynchronize((hipStream_t)stream));
  if (choice) *choice = ch;
  return FIRAL_OK;
}

extern "C" int firal_batch_create(firal_batch* out, int32_t n, const firal_batch_problem* probs,
                                  void* stream) {
  if (!out || !probs || n < 1) {
    set_error("firal_batch_create: null argument or n < 1");
    return FIRAL_EINVAL;
  }
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    const firal_batch_problem& p = probs[i];
    if (!p.ctx || !p.w || p.s < 1 || p.s > C(p.ctx)->s_max || p.t0 < 1 || p.max_iter < 0 ||
        !(p.b > 0.0) || !(p.lambda > 0.0)) {
      set_error("firal_batch_create: problem %d: null context or weights, s outside [1, s_max], "
                "t0 < 1, max_iter < 0, or b, lambda not positive", i);
      return FIRAL_EINVAL;
    }
    for (int j = 0; j < i; ++j)
      if (probs[j].ctx == p.ctx) {
        set_error("firal_batch_create: problems %d and %d share a context", j, i);
        return FIRAL_EINVAL;
      }
  }
  hipStream_t st = (hipStream_t)stream;
  Batch* b = new Batch;
  b->n = n;
  b->probs.assign(probs, probs + n);
  (void)hipGetDevice(&b->device);
  int rc = FIRAL_OK;
  // kernel variants per shape bucket (timed once per bucket in this process)
  for (int i = 0; i < n && rc == FIRAL_OK; ++i) rc = autotune(C(probs[i].ctx), probs[i].s, st, nullptr);
  // one eager pass of the capture-safe step per problem (sets every kernel attribute the
  // branch needs before capture), with the weights restored afterwards
  double* wsave = nullptr;
  int64_t wmax = 0;
  for (int i = 0; i < n; ++i) wmax = std::max<int64_t>(wmax, C(probs[i].ctx)->n_pool);
  if (rc == FIRAL_OK && hipMalloc((void**)&wsave, wmax * sizeof(double)) != hipSuccess) {
    set_error("firal_batch_create: hipMalloc failed");
    rc = FIRAL_ENOMEM;
  }
  for (int i = 0; i < n && rc == FIRAL_OK; ++i) {
    const firal_batch_problem& p = probs[i];
    Ctx* x = C(p.ctx);
    const size_t wb = x->n_pool * sizeof(double);
    const int32_t t0 = p.t0;
    if (hipMemcpyAsync(wsave, p.w, wb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(x->t_dev, &t0, sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess) {
      set_error("firal_batch_create: copy failed");
      rc = FIRAL_EHIP;
      break;
    }
    x->async = 1;
    rc = relax_step_launch(x, p.w, p.b, p.lambda, p.beta0, p.seed, p.t0, p.s, p.tol, p.max_iter,
                           p.flags, nullptr, st);
    x->async = 0;
    if (rc == FIRAL_OK &&
        (hipMemcpyAsync(p.w, wsave, wb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
         hipMemcpyAsync(x->t_dev, &t0, sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess ||
         hipStreamSynchronize(st) != hipSuccess)) {
      set_error("firal_batch_create: warm-up failed");
      rc = FIRAL_EHIP;
    }
  }
  if (wsave) (void)hipFree(wsave);
  // streams and events (default priority), then the capture
  if (rc == FIRAL_OK) {
    b->streams.assign(n, nullptr);
    b->joins.assign(n, nullptr);
    bool ok = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < n && ok; ++i)
      ok = hipStreamCreateWithFlags(&b->streams[i], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&b->joins[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      set_error("firal_batch_create: stream or event creation failed");
      rc = FIRAL_EHIP;
    }
  }
  if (rc == FIRAL_OK) {
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed) != hipSuccess ||
        hipEventRecord(b->fork, b->cap) != hipSuccess) {
      set_error("firal_batch_create: capture could not start");
      rc = FIRAL_EHIP;
    }
    for (int i = 0; i < n && rc == FIRAL_OK; ++i) {
      const firal_batch_problem& p = probs[i];
      Ctx* x = C(p.ctx);
      if (hipStreamWaitEvent(b->streams[i], b->fork, 0) != hipSuccess) {
        set_error("firal_batch_create: fork failed");
        rc = FIRAL_EHIP;
        break;
      }
      x->async = 1;
      rc = relax_step_launch(x, p.w, p.b, p.lambda, p.beta0, p.seed, p.t0, p.s, p.tol,
                             p.max_iter, p.flags, nullptr, b->streams[i]);
      x->async = 0;
      if (rc == FIRAL_OK && (hipEventRecord(b->joins[i], b->streams[i]) != hipSuccess ||
                             hipStreamWaitEvent(b->cap, b->joins[i], 0) != hipSuccess)) {
        set_error("firal_batch_create: join failed");
        rc = FIRAL_EHIP;
      }
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->cap, &g);
    b->graph = g;
    if (rc == FIRAL_OK && ec != hipSuccess) {
      set_error("firal_batch_create: capture failed: %s", hipGetErrorString(ec));
      rc = FIRAL_EHIP;
    }
    if (rc == FIRAL_OK && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
      set_error("firal_batch_create: graph instantiation failed");
      rc = FIRAL_EHIP;
    }
  }
  (void)hipGetLastError();
  if (rc != FIRAL_OK) {
    free_batch(b);
    return rc;
  }
  *out = reinterpret_cast<firal_batch>(b);
  return FIRAL_OK;
}

extern "C" int firal_batch_run(firal_batch batch, int32_t iters, void* stream) {
  if (!batch || iters < 0) {
    set_error("firal_batch_run: null batch or iters < 0");
    return FIRAL_EINVAL;
  }
  Batch* b = reinterpret_cast<Batch*>(batch);
  for (int k = 0; k < iters; ++k) FIRAL_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream));
  return FIRAL_OK;
}

extern "C" int firal_batch_info(firal_batch batch, int32_t i, firal_info* info, void* stream) {
  if (!batch || !info) {
    set_error("firal_batch_info: null argument");
    return FIRAL_EINVAL;
  }
  Batch* b = reinterpret_cast<Batch*>(batch);
  if (i < 0 || i >= b->n) {
    set_error("firal_batch_info: problem %d outside [0, %d)", i, b->n);
    return FIRAL_EINVAL;
  }
  Ctx* x = C(b->probs[i].ctx);
  FIRAL_HIP(hipStreamSynchronize((hipStream_t)stream));
  Status h;
  FIRAL_HIP(hipMemcpy(&h, x->status, sizeof(Status), hipMemcpyDeviceToHost));
  info->cg_iters[0] = h.cg_iters[0];
  info->cg_iters[1] = h.cg_iters[1];
  info->converged = h.converged;
  info->bad_block = h.bad_block == INT32_MAX ? -1 : h.bad_block;
  info->relres_max = h.relres_max;
  info->f_hat = h.f_hat;
  info->g_absmax = h.g_absmax;
  info->beta = h.beta;
  if (h.bad_block != INT32_MAX) return FIRAL_ENOTSPD;
  if (h.breakdown) return FIRAL_EBREAKDOWN;
  return h.converged ? FIRAL_OK : FIRAL_WARN_NOT_CONVERGED;
}

extern "C" int firal_batch_next_t(firal_batch batch, int32_t i, int32_t* t) {
  if (!batch || !t) {
    set_error("firal_batch_next_t: null argument");
    return FIRAL_EINVAL;
  }
  Batch* b = reinterpret_cast<Batch*>(batch);
  if (i < 0 || i >= b->n) {
    set_error("firal_batch_next_t: problem %d outside [0, %d)", i, b->n);
    return FIRAL_EINVAL;
  }
  FIRAL_HIP(hipDeviceSynchronize());
  FIRAL_HIP(hipMemcpy(t, C(b->probs[i].ctx)->t_dev, sizeof(int32_t), hipMemcpyDeviceToHost));
  return FIRAL_OK;
}

extern "C" int firal_batch_destroy(firal_batch batch) {
  if (!batch) return FIRAL_OK;
  (void)hipDeviceSynchronize();
  free_batch(reinterpret_cast<Batch*>(batch));
  return FIRAL_OK;
}
