// Internal declarations of the gfx950 Relax library: context layout, MFMA
// wrappers, reductions and the host-side launchers shared between sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <atomic>
#include <vector>

#include "firal.h"

namespace firal {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);

#define FIRAL_HIP(x)                                                            \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      (void)hipGetLastError(); /* do not leave the error for a later check */   \
      ::firal::set_error("%s failed: %s", #x, hipGetErrorString(e_));           \
      return FIRAL_EHIP;                                                        \
    }                                                                           \
  } while (0)

#define FIRAL_LAUNCHED()                                                        \
  do {                                                                          \
    hipError_t e_ = hipGetLastError();                                          \
    if (e_ != hipSuccess) {                                                     \
      ::firal::set_error("kernel launch failed at %s:%d: %s", __FILE__, __LINE__, \
                         hipGetErrorString(e_));                                \
      return FIRAL_EHIP;                                                        \
    }                                                                           \
  } while (0)

#define FIRAL_CHECK(x)                                                          \
  do {                                                                          \
    int rc_ = (x);                                                              \
    if (rc_ < 0) return rc_;                                                    \
  } while (0)

// ------------------------------------------------------- device status
// One per context, in device memory.  Written only by the library's kernels.
struct Status {
  int32_t all_done;     // PCG loop: nothing left to do (all columns converged, or an error)
  int32_t iters;        // PCG iterations performed by the current solve
  int32_t breakdown;    // PCG: p^T q <= 0 on an active column
  int32_t bad_block;    // Cholesky: smallest failing class index, INT32_MAX when none
  int32_t cg_iters[2];  // iterations of the two solves of a Relax iteration
  int32_t converged;    // 1 while every finished solve converged
  int32_t pad;
  double relres_max;
  double f_hat;
  double g_absmax;
  double beta;
};

// ------------------------------------------------------------- context
struct Ctx {
  int64_t n_pool, n_lab, N;
  int d, c, s_max;
  int prec;             // firal_prec
  size_t esize;         // bytes per element of X, H and blocks
  const void* X;
  const void* H;
  int device;
  int n_cu;             // compute units of the device

  // hvp / grad row-chunk intermediates
  int64_t chunk_rows;   // rows per chunk of the (rows x s*c) intermediate
  void* G;              // chunk_rows * s_max * c elements
  double* gpart;        // column tiles * chunk_rows: per-tile row dot products (gradient)
  int max_splits;       // split-K partial buffers for the X^T G contraction
  void* part;           // max_splits * d * s_max * c elements

  // fused FP32 product: per-row-range partials of the output block
  void* fused_part;
  int64_t fused_part_elems;
  int fused_max_ncb;    // fused product: column blocks per wave, 2 (wide tiles) or 1 (two
                        // workgroups' registers per CU, next chunk fetched ahead)
  int gram_form;        // preconditioner Gram kernel (kGramClassic, kGramWide, kGramWideBf3)
  int fused_wgs;        // fused product: workgroups a launch aims for (row ranges x column
                        // tiles; 0 = 256); firal_autotune chooses it
  int force_tiled;      // product and FP32 gradient: the row-tiled kernels even where the
                        // fused ones fit
  int force_multik;     // PCG: separate kernels even where the column-local step fits
                        // (FIRAL_UNFUSED=1 sets both; firal_autotune chooses them)
  int async;            // enqueue without host reads (graph capture): fixed-trip PCG whose
                        // kernels return once every column has converged
  int32_t* t_dev;       // device Relax-iteration counter of captured steps
  double bf3_switch;    // BF16X3 PCG: FP32 products once max_j ||r_j||/||b_j|| < bf3_switch

  // bf16x3 contexts: hi/lo bf16 planes of X (N x d) and of X^T (d x ldt, ldt = N rounded up
  // to a multiple of 8, padding zero), made once at creation
  void* Xhi;
  void* Xlo;
  void* XThi;
  void* XTlo;
  int64_t ldt;

  // wide FP32 path (gemm_nt.hip; d > 128, d % 4 == 0, c > 128): X^T (d x ldn) and H^T
  // (c x ldn) in FP32, ldn = N rounded up to a multiple of 4 (padding zero), made at creation;
  // the transposed probe block (s_max c x d); per chunk alpha partials, alpha and omega
  int use_nt;
  int64_t ldn;
  void* XTf;
  void* HTf;
  void* VTf;
  void* ntpart;

  // preconditioner
  double* P;            // c * d * d: blocks, factorised in place
  double* Pinv;         // c * d * d
  void* syrk_part;      // syrk_splits * c * d * d elements (lower triangles written)
  int syrk_splits;
  int32_t* syrk_tiles;  // (a-block, b-block) of each pair tile of the Gram GEMM
  int syrk_ntiles;

  // Relax / PCG blocks (d * s_max * c elements each)
  void *V, *W1, *Y, *W2;
  void *cx, *cr, *cz, *cp, *cq;
  double* mean;         // d * s_max: class means for the projection
  double* omega;        // N
  double* gbuf;         // n_pool: gradient
  double* ebuf;         // n_pool: exponents of the mirror step

  // per-column scalars and reduction partials
  int col_parts;        // partial sums per column
  double* colpart;      // 4 * s_max * col_parts
  double* cgd;          // column-local CG: rd and zd, 2 * d * c * s_max (null when unused)
  double* rho;          // s_max
  double* bnorm;        // s_max
  double* alpha;        // s_max
  double* beta;         // s_max
  double* relres;       // s_max
  int32_t* done;        // s_max
  int red_blocks;       // blocks of the n_pool reductions
  double* redpart;      // 3 * red_blocks

  Status* status;       // device
  Status* status_host;  // pinned host mirror
  uint32_t chk_tag;     // tag of the last column-local PCG iteration enqueued
  uint32_t* chk_word;   // pinned coherent host memory [2][s_max], one word per column:
                        //   (tag << 2) | (relres < bf3_switch) << 1 | column stopped
  uint32_t* chk_word_dev;  // its device address

  // firal_profile_begin/end: event pairs around each launch of one kernel (prof_kernel, a
  // FIRAL_PROF_* value)
  int profiling;
  int prof_kernel;
  void* prof_events;    // std::vector<std::pair<hipEvent_t, hipEvent_t>>*
};

// when profiling `kernel` (a FIRAL_PROF_* value), a new event pair for one launch through
// hipExtLaunchKernel, which records the kernel's own start and end in it (null events
// otherwise: a plain launch)
int prof_pair(Ctx* x, int kernel, hipEvent_t* e0, hipEvent_t* e1);

inline Ctx* C(firal_ctx p) { return reinterpret_cast<Ctx*>(p); }

// ------------------------------------------------------------ constants
constexpr int kBlock = 256;
// largest workgroup target of the fused product (its partial-sum buffer is sized for it)
constexpr int kFusedMaxWgs = 1024;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// One-time set-up per device: kernel attributes (the dynamic LDS limit above 64 KiB) apply to the
// device current when they are set, so a process driving contexts on several devices sets them
// on each.  done() and set() refer to the current device (0 .. 63; any other device is never
// marked done, so its set-up simply repeats).
class DeviceOnce {
 public:
  bool done() const {
    const int dev = current();
    return dev >= 0 && dev < 64 && ((bits_.load() >> dev) & 1u) != 0;
  }
  void set() {
    const int dev = current();
    if (dev >= 0 && dev < 64) bits_.fetch_or(uint64_t(1) << dev);
  }

 private:
  static int current() {
    int dev = -1;
    return hipGetDevice(&dev) == hipSuccess ? dev : -1;
  }
  std::atomic<uint64_t> bits_{0};
};

// ------------------------------------------------------------- MFMA
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA: lane l supplies A[l%16][l/16] and B[l/16][l%16] and receives
// D[row(l/16, v)][l%16], v = 0..3, where row(q, v) = 4q + v for FP32 and q + 4v for
// FP64 (the two instructions place their four results differently).
template <typename T> struct Mfma16;
template <> struct Mfma16<float> {
  typedef f32x4 acc;
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }
  static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma16<double> {
  typedef f64x4 acc;
  static __device__ __forceinline__ int row(int q, int v) { return q + 4 * v; }
  static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// bf16x3 products: x y ~ xh yh + xh yl + xl yh with xh = bf16(x) (round to nearest even) and
// xl = bf16(x - xh), each on the 16x16x32 bf16 MFMA with FP32 accumulation.  Lane l supplies
// A[l%16][8(l/16) + u] and B[8(l/16) + u][l%16], u = 0..7, and receives D as the FP32
// 16x16x4 instruction does (row 4(l/16) + v).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split8(const float* v, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const __bf16 h = (__bf16)v[u];
    hi[u] = h;
    lo[u] = (__bf16)(v[u] - (float)h);
  }
}

__device__ __forceinline__ f32x4 mfma3(const bf16x8& ah, const bf16x8& al, const bf16x8& bh,
                                       const bf16x8& bl, f32x4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
  return acc;
}

// ------------------------------------------------------- reductions
// v + (v moved across lanes by one DPP pattern): both 32-bit halves move with the same
// control; lanes the row/bank masks leave unwritten, or whose source lies outside the row
// (bound_ctrl), add 0.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ double dpp_add(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, BANK_MASK, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, BANK_MASK, true);
  return v + __hiloint2double(hi, lo);
}
// Sum over the 64 lanes of a wave in a fixed order, returned in every lane: pairs and quads
// by quad permutes, the 16-lane rows by right shifts of 4 and 8, then row 1 collects row 0
// and row 3 row 2 (row broadcast of lane 15), and row 3 collects rows 0-1 (broadcast of
// lane 31). The total lands in lane 63, which a readlane hands to all lanes.
__device__ __forceinline__ double wave_sum(double v) {
  v = dpp_add<0xB1, 0xF, 0xF>(v);    // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xF, 0xF>(v);    // quad_perm [2,3,0,1]
  v = dpp_add<0x114, 0xF, 0xE>(v);   // row_shr:4, lanes 4-15 of each row
  v = dpp_add<0x118, 0xF, 0xC>(v);   // row_shr:8, lanes 8-15 of each row
  v = dpp_add<0x142, 0xA, 0xF>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xC, 0xF>(v);   // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}
// Block-wide sum/max in a fixed order; result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[NT / 64];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) r += red[i];
  __syncthreads();
  return r;
}
template <int NT>
__device__ __forceinline__ double block_max(double v) {
  __shared__ double red[NT / 64];
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  double r = -INFINITY;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

// ---------------------------------------------------------- skip rule
// Kernels of a PCG loop return at once when there is nothing left to do, so the host can
// queue iterations ahead of its convergence test.  `flag`: skip when *flag != 0;
// `flags`: skip when flags[0..n) are all nonzero (the per-column convergence flags of the
// previous iteration).  skip_now must be reached by every thread of the block.
struct Skip {
  const int32_t* flag;
  const int32_t* flags;
  int n;
};
__host__ __device__ inline Skip skip_none() { return Skip{nullptr, nullptr, 0}; }
__host__ __device__ inline Skip skip_flag(const int32_t* f) { return Skip{f, nullptr, 0}; }
__host__ __device__ inline Skip skip_all(const int32_t* f, int n) { return Skip{nullptr, f, n}; }
__device__ __forceinline__ bool skip_now(const Skip& k) {
  if (k.flag) return *k.flag != 0;
  if (k.flags) {
    int ok = 1;
    for (int j = threadIdx.x; j < k.n; j += blockDim.x) ok &= k.flags[j] != 0;
    return __syncthreads_and(ok) != 0;
  }
  return false;
}

// Tile plan of the fused FP32 product (hvp_fused.hip).
struct FusedPlan {
  void* kernel;
  int bf3;              // bf16x3 products
  int D16, ncb, probes_per_tile, n_ctiles, n_splits;
  int64_t rows_per_split;
  int XS, XT, GT, CP;
  size_t lds_bytes;
  int64_t part_elems;   // n_splits * d * s * c
};
bool fused_plan(const Ctx* x, int s, int64_t n_rows, FusedPlan* p, bool precise = false);
template <typename T>
int reduce_parts_launch(const T* part, int64_t n, int P, double shift, const T* B, T* out,
                        Skip skip, hipStream_t st);
// hi/lo bf16 planes of V^T, (s c) x d, for a probe block B (d x s c, row-major), split once
int nt3_split_vt(const float* B, int d, int SC, __bf16* VTh, __bf16* VTl, hipStream_t st);
int hvp_fused_launch(Ctx* x, const FusedPlan& p, const double* omega, int64_t n_rows, double shift,
                     const float* B, float* out, int s, Skip skip, hipStream_t st);

// ------------------------------------------------- host-side launchers
// All enqueue on `st`; `skip` (see Skip) makes every kernel of the call return at once.
// precise: in a BF16X3 context, take the FP32 products for this call (mixed-precision PCG)
int hvp_launch(Ctx* x, const double* omega, int64_t n_rows, double shift, const void* B,
               void* out, int s, Skip skip, hipStream_t st, bool precise = false);
// Gram blocks, then P^-1 into x->Pinv; the factor L goes to x->P only when want_l (for d <= 256
// x->P otherwise keeps the Gram blocks)
int precond_launch(Ctx* x, const double* omega, double shift, hipStream_t st, bool want_l = false);
// Preconditioner Gram kernels: the classic tiling (classes and pairs split between the waves),
// or, for FP32 storage with c > 64, d a multiple of 4 and X 16-byte aligned, the waves along the
// pairs (FIRAL_GRAM_WIDE=0 in the environment keeps the classic one), in a BF16X3 context as
// bf16x3 products when FIRAL_BF3_GRAM=1 (FP32 otherwise).  Chosen once, at context creation.
constexpr int kGramClassic = 0, kGramWide = 1, kGramWideBf3 = 2;
int gram_form_for(int prec, int d, int c, const void* X);
void syrk_plan(int prec, int d, int c, int form, int n_cu, std::vector<int32_t>* tiles,
               int* splits);
// FP64 weighted Gram blocks sum_r omega_r h_rk (1 - h_rk) x_r x_r^T + shift I over rows [0, N)
// of X and H (storage FP32 unless prec is FIRAL_F64; omega null: weight 1) into out
// (c x d x d); tiles/S from syrk_plan(FIRAL_F64, ...), part holds S x c x d x d doubles.
int gram64_launch(int prec, const void* X, const void* H, const double* omega, int64_t N, int d,
                  int c, const int32_t* tiles, int ntiles, int S, double shift, double* part,
                  double* out, hipStream_t st);
// Cholesky of c SPD blocks: the lower factor replaces P (upper part zeroed) when want_l (always
// for d > 256); the blocks' inverses go to Pinv (for d > 256 only when want_inv).  *bad
// (preset to INT32_MAX) receives the smallest failing block.
int chol_blocks_launch(double* P, double* Pinv, int d, int c, int32_t* bad, bool want_inv,
                       bool want_l, hipStream_t st);
// doubles of column-local CG scratch for d, c, s_max; 0 when that path does not fit
int64_t col_cg_scratch(int d, int c, int s_max);
int pcg_launch(Ctx* x, const double* omega, double shift, const double* Pinv, const void* B,
               void* Xsol, int s, double tol, int max_iter, uint32_t flags, int slot,
               hipStream_t st);
int grad_launch(Ctx* x, const void* U, const void* W, int s, double* g, hipStream_t st);
// wide FP32 path (gemm_nt.hip)
bool nt_applies(const Ctx* x);
int64_t nt_ld(int64_t rows);
int nt_windows(int c);
int nt_prepare_ctx(Ctx* x, hipStream_t st);
int hvp_nt_launch(Ctx* x, const double* omega, int64_t n_rows, double shift, const float* B,
                  float* out, int s, Skip skip, hipStream_t st);
// general (any d, c) product through the row-tiled kernels of tiled.hip
int hvp_tiled_launch(Ctx* x, const double* omega, int64_t n_rows, double shift, const void* B,
                     void* out, int s, Skip skip, hipStream_t st, bool precise);
// buffer sizing of the row-tiled kernels
int64_t tiled_col_tiles(int prec, int c, int s);
// Fused FP32 gradient pass (d <= 128) into x->gpart: per pool row, one partial per tile of
// probes; *n_tiles = 0 when the shape is not covered (nothing launched)
int grad_fused_launch(Ctx* x, const float* U, const float* W, int s, hipStream_t st,
                      int* n_tiles);
int split_x_launch(Ctx* x, hipStream_t st);
int64_t tiled_out_tiles(int prec, int d, int64_t sc);
int probes_launch(Ctx* x, uint64_t seed, int t, int s, void* V, hipStream_t st,
                  const int32_t* t_dev = nullptr);
int relax_step_launch(Ctx* x, double* w, double b, double lambda, double beta0, uint64_t seed,
                      int t, int s, double tol, int max_iter, uint32_t flags, double* g_out,
                      hipStream_t st);
// w = v everywhere (scale false) or w *= v (scale true), n FP64 entries
int fill_scale_launch(double* w, int64_t n, double v, bool scale, hipStream_t st);
int coldot_launch(Ctx* x, const void* A, const void* B, int s, double* part, Skip skip,
                  hipStream_t st);

}  // namespace firal
