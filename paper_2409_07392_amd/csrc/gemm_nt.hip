// FP32 Hessian product of Lemma 1 for wide problems (d > 128, c > 128, d a multiple of 4):
// both contractions as GEMMs whose operands are stored with the contraction index contiguous,
// so every operand moves as 16-byte vectors from HBM to LDS and from LDS to the MFMA inputs.
//
// Per chunk of R rows (rows r0 .. r0 + R):
//   k_nt_xv     G = X V^T[n][.] (X row-major; V^T: the probe block transposed once per call),
//               stored transposed and scaled by the row weights, E^T[n][r] = omega_r G[r][n]; its
//               epilogue also forms, per row and tile, beta_part[p][w][r] = sum over the tile's
//               columns of E h (the tiles of probe p are its column windows w: c > 128, so a
//               tile never mixes probes)
//   k_nt_alpha  beta[p][r] = sum_w beta_part[p][w][r] (FP64, fixed order) = omega_r alpha_rp
//   k_nt_xtg    part[sp][a][n] (+)= sum_r X^T[a][r] G'^T[n][r] over the split's rows, with the
//               row step of Lemma 1, G' = omega (G - alpha) h = (E - beta) h, applied while E^T
//               is staged (X^T and H^T: transposed FP32 copies made at context creation)
// and the split sums are reduced in a fixed order (hvp.hip).
//
// MFMA: v_mfma_f32_16x16x4f32.  Within a 16-deep k group the four instructions q = 0..3 take
// k = 4 g + q from lane group g = lane / 16, so a lane's four k values are contiguous and one
// 128-bit LDS read feeds four instructions; the result lane (g, l % 16) holds rows 4 g .. 4 g + 3
// of column l % 16, contiguous in a transposed store.
#include <algorithm>

#include <hip/hip_ext.h>

#include "common.h"

namespace firal {

namespace {

constexpr int kNtBM = 128, kNtBN = 128;   // workgroup tile (rows x columns of the output)
constexpr int kNtKS = 32;                 // k per pipeline stage of the bf16x3 kernels and the
                                          // row granule of the row splits
constexpr int kNtWG = 256;                // four waves, 2 x 2, each 64 x 64
// FP32 stage depths and workgroups per CU: the first contraction runs 16-deep stages at three
// workgroups per CU (measured 4.0 ms a launch against 4.25 ms with 32-deep stages at two); the
// second, whose staging also applies beta and h, runs faster with 32-deep stages at two
// (4.69 ms against 5.05 ms with 16-deep stages at three).
constexpr int kNtKsXv = 16, kNtMinbXv = 3;
constexpr int kNtKsXtg = 32, kNtMinbXtg = 2;

typedef float f4 __attribute__((ext_vector_type(4)));

// Workgroup b of n runs on XCD b % 8; give each XCD a contiguous range of logical tiles.
__device__ __forceinline__ int64_t nt_lid(int64_t b, int64_t n) {
  const int64_t q = n >> 3, r = n & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// FP32 stages of KS = 16 or 32 k: LDS rows KS + 4 floats apart (16-byte reads of a fragment
// spread over all banks); two buffers of 128 + 128 rows.
template <int KS> constexpr int nt_sk() { return KS + 4; }
template <int KS> constexpr size_t nt_lds_bytes() {
  return (size_t)2 * (kNtBM + kNtBN) * nt_sk<KS>() * 4;
}

// One KS-deep stage of a wave's 4 x 4 blocks of 16 x 16 from LDS tiles a[m][k], b[n][k].
template <int KS>
__device__ __forceinline__ void nt_stage(const float* __restrict__ a, const float* __restrict__ b,
                                         int wm, int wn, int li, int g, f32x4 (&acc)[4][4]) {
  constexpr int SK = nt_sk<KS>();
#pragma unroll
  for (int kg = 0; kg < KS / 16; ++kg) {
    f4 av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      av[i] = *reinterpret_cast<const f4*>(a + (wm + 16 * i + li) * SK + 16 * kg + 4 * g);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      bv[j] = *reinterpret_cast<const f4*>(b + (wn + 16 * j + li) * SK + 16 * kg + 4 * g);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][q], bv[j][q], acc[i][j], 0, 0, 0);
  }
}

// Tile loads: a 128 x KS tile of a row-major source (leading dimension ld, k contiguous) as
// 16-byte vectors, KS / 8 per thread: vector e = tid + 256 t covers row e / (KS / 4), k 4 (e %
// (KS / 4)).  Rows at or beyond nrow and k at or beyond nk read row 0, k 0 (a valid address)
// and are cleared to zero by nt_store through the returned mask (bit t: vector t in range), so
// that nothing consumes a loaded value before the stage's MFMAs (nk a multiple of 4).
template <int KS>
__device__ __forceinline__ unsigned nt_load(const float* __restrict__ src, int64_t ld,
                                            int64_t row0, int64_t nrow, int64_t k0, int64_t nk,
                                            int tid, f4 (&v)[KS / 8]) {
  constexpr int VR = KS / 4;
  unsigned m = 0;
#pragma unroll
  for (int t = 0; t < KS / 8; ++t) {
    const int e = tid + kNtWG * t, rr = e / VR, kk = 4 * (e % VR);
    const int64_t row = row0 + rr, k = k0 + kk;
    const bool ok = row < nrow && k < nk;
    v[t] = *reinterpret_cast<const f4*>(src + (ok ? row * ld + k : 0));
    m |= (unsigned)ok << t;
  }
  return m;
}
template <int KS>
__device__ __forceinline__ void nt_store(float* __restrict__ dst, int tid, const f4 (&v)[KS / 8],
                                         unsigned m) {
  constexpr int VR = KS / 4;
#pragma unroll
  for (int t = 0; t < KS / 8; ++t) {
    const int e = tid + kNtWG * t, rr = e / VR, kk = 4 * (e % VR);
    *reinterpret_cast<f4*>(dst + rr * nt_sk<KS>() + kk) =
        (m >> t) & 1u ? v[t] : f4{0.f, 0.f, 0.f, 0.f};
  }
}

// Keeps the compiler's scheduler from moving instructions across this point: the next stage's
// loads are issued before the stage's MFMAs and consumed only after them.
__device__ __forceinline__ void nt_order() { __builtin_amdgcn_sched_barrier(0); }

// Epilogue of the first contraction (both forms); OM: omega given (else omega = 1).
template <bool OM>
__device__ __forceinline__ void nt_xv_epilogue(const f32x4 (&acc)[4][4], float* nt_lds, int wave,
                                               int wm, int wn, int li, int g, int tid,
                                               int64_t row0, int64_t R, int width, int col0,
                                               int64_t n0, int p, int w, int nw,
                                               const float* __restrict__ HT, int64_t ldh,
                                               const double* __restrict__ omega,
                                               float* __restrict__ GT, int64_t ldg,
                                               float* __restrict__ apart) {
  // Epilogue.  Lane (g, li) of block (i, j) holds G[r][n] for r = row0 + wm + 16 i + 4 g + v,
  // n = col0 + wn + 16 j + li (v = 0..3).  (1) E^T = (omega G)^T as 16-byte stores of four rows;
  // (2) per row the sum over this wave's columns of E h, then over the 16 lanes of a column
  // group, then over the two waves of a row band through LDS, into beta_part[p][w][r].
  float* red = nt_lds;   // [2][kNtBM]: the main buffers are free after the last barrier
  // two halves of two row blocks each: every load of a half first (omega of the lane's 8 rows,
  // h of its 8 row quads), at addresses clamped into the valid rows and columns, so that their
  // latencies overlap
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
    float om[2][4];
    f4 hq[2][4];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) {
      const int64_t r = row0 + wm + 16 * (2 * hf + ii) + 4 * g;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t rv = r + v < R ? r + v : 0;
        const float o = OM ? (float)omega[rv] : 1.f;
        om[ii][v] = r + v < R ? o : 0.f;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int nl = wn + 16 * j + li;
        const int nc = nl < width ? nl : 0;
        hq[ii][j] =
            *reinterpret_cast<const f4*>(HT + (int64_t)(col0 + nc) * ldh + (r < R ? r : 0));
      }
    }
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) {
      const int i = 2 * hf + ii;
      const int64_t r = row0 + wm + 16 * i + 4 * g;   // first of the lane's four rows
      float t[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int nl = wn + 16 * j + li;              // column within the window
        const f4 e = f4{om[ii][0] * acc[i][j][0], om[ii][1] * acc[i][j][1],
                        om[ii][2] * acc[i][j][2], om[ii][3] * acc[i][j][3]};
        if (nl < width && r < R) {
          const int64_t n = n0 + nl;
          // R is a multiple of 4 except at the end of the rows; guard the last vector.  The
          // stores are non-temporal: E^T is read back by the second kernel from HBM (a chunk's
          // E^T is far larger than L2 and the MALL), and should not evict X, V^T and h from L2
          if (r + 3 < R) {
            __builtin_nontemporal_store(e, reinterpret_cast<f4*>(GT + n * ldg + r));
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (r + v < R) GT[n * ldg + r + v] = e[v];
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) t[v] = fmaf(e[v], hq[ii][j][v], t[v]);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float s = t[v];
        s += __shfl_xor(s, 1, 64);
        s += __shfl_xor(s, 2, 64);
        s += __shfl_xor(s, 4, 64);
        s += __shfl_xor(s, 8, 64);
        t[v] = s;
      }
      if (li == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(wave & 1) * kNtBM + wm + 16 * i + 4 * g + v] = t[v];
      }
    }
  }
  __syncthreads();
  if (tid < kNtBM) {
    const int64_t r = row0 + tid;
    if (r < R) apart[((int64_t)p * nw + w) * ldg + r] = red[tid] + red[kNtBM + tid];
  }
}

// Epilogue of the second contraction (both forms): the split's partial output block.
__device__ __forceinline__ void nt_xtg_epilogue(const f32x4 (&acc)[4][4], float* __restrict__ part,
                                                int sp, int64_t part_stride, int a0, int n0,
                                                int n_end, int wm, int wn, int li, int g, int d,
                                                int SC, int accumulate) {
  float* out = part + (int64_t)sp * part_stride;
  if (accumulate) {
    // the earlier partials of two row blocks at a time are loaded first (clamped addresses) so
    // that the loads overlap, then added and stored
#pragma unroll
    for (int i0 = 0; i0 < 4; i0 += 2) {
      float prev[2][4][4];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int a = a0 + wm + 16 * (i0 + i) + 4 * g + v;
            const int n = n0 + wn + 16 * j + li;
            prev[i][j][v] = out[a < d && n < n_end ? (int64_t)a * SC + n : 0];
          }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int a = a0 + wm + 16 * (i0 + i) + 4 * g + v;
            const int n = n0 + wn + 16 * j + li;
            if (a < d && n < n_end)
              out[(int64_t)a * SC + n] = prev[i][j][v] + acc[i0 + i][j][v];
          }
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = a0 + wm + 16 * i + 4 * g + v;
          const int n = n0 + wn + 16 * j + li;
          if (a < d && n < n_end) out[(int64_t)a * SC + n] = acc[i][j][v];
        }
  }
}

// Kernel 1.  Tiles: row tile rt (kNtBM rows of the chunk) x column tile ct: the column windows
// of kNtBN columns of s probes (nw windows each), tile ct = window (ct / s) of probe (ct % s).
template <int KS, int MINB, bool OM>
__global__ __launch_bounds__(kNtWG, MINB) void k_nt_xv(
    const float* __restrict__ X, int d, int64_t R, const float* __restrict__ VT, int c, int nw,
    int ntc, const float* __restrict__ HT, int64_t ldh, const double* __restrict__ omega,
    float* __restrict__ GT, int64_t ldg, float* __restrict__ apart, Skip skip) {
  if (skip_now(skip)) return;
  extern __shared__ __align__(16) float nt_lds[];
  constexpr int SK = nt_sk<KS>();
  float* As = nt_lds;                          // [2][kNtBM][SK]
  float* Bs = nt_lds + 2 * kNtBM * SK;         // [2][kNtBN][SK]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  // tiles in groups of 8 row tiles: consecutive logical ids take the 8 row tiles of a group for
  // one column tile, then the next column tile, so that 64 workgroups resident on one XCD share
  // 8 tiles of X and 8 of V^T in its L2 (the last group may hold fewer row tiles)
  const int64_t lid = nt_lid(blockIdx.x, gridDim.x);
  const int64_t nrt = (R + kNtBM - 1) / kNtBM;
  const int64_t grp = lid / (8 * (int64_t)ntc);
  const int64_t g0 = grp * 8;
  const int64_t gsz = nrt - g0 < 8 ? nrt - g0 : 8;
  const int64_t in = lid - grp * 8 * (int64_t)ntc;
  const int ct = (int)(in / gsz);
  const int64_t rt = g0 + (in - (int64_t)ct * gsz);
  // column tiles with the probe fastest: consecutive tiles share the window's classes (h)
  const int ns = ntc / nw;
  const int w = ct / ns, p = ct - w * ns;
  const int64_t row0 = rt * kNtBM;
  const int col0 = w * kNtBN;                              // within the probe
  const int width = c - col0 < kNtBN ? c - col0 : kNtBN;  // columns of the window
  const int64_t n0 = (int64_t)p * c + col0;                // first column of V^T
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  f4 ra[KS / 8], rb[KS / 8];
  const int nst = (d + KS - 1) / KS;
  unsigned ma = nt_load<KS>(X, d, row0, R, 0, d, tid, ra);
  unsigned mb = nt_load<KS>(VT + n0 * d, d, 0, width, 0, d, tid, rb);
  nt_store<KS>(As, tid, ra, ma);
  nt_store<KS>(Bs, tid, rb, mb);
  __syncthreads();
  // every pass loads the next stage (past the last stage the loads are masked to zero and their
  // store lands in the buffer no later stage reads)
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    ma = nt_load<KS>(X, d, row0, R, (int64_t)(st + 1) * KS, d, tid, ra);
    mb = nt_load<KS>(VT + n0 * d, d, 0, width, (int64_t)(st + 1) * KS, d, tid, rb);
    nt_order();
    nt_stage<KS>(As + buf * kNtBM * SK, Bs + buf * kNtBN * SK, wm, wn, li, g, acc);
    nt_order();
    nt_store<KS>(As + (buf ^ 1) * kNtBM * SK, tid, ra, ma);
    nt_store<KS>(Bs + (buf ^ 1) * kNtBN * SK, tid, rb, mb);
    __syncthreads();
  }

  nt_xv_epilogue<OM>(acc, nt_lds, wave, wm, wn, li, g, tid, row0, R, width, col0, n0, p, w, nw,
                     HT, ldh, omega, GT, ldg, apart);
}

// beta[p][r] = sum_w beta_part[p][w][r] in FP64, fixed order (= omega_r alpha_rp).
__global__ __launch_bounds__(256) void k_nt_alpha(const float* __restrict__ apart, int nw, int s,
                                                  int64_t R, int64_t ldg,
                                                  float* __restrict__ beta, Skip skip) {
  if (skip_now(skip)) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)s * R) return;
  const int p = (int)(e / R);
  const int64_t r = e - (int64_t)p * R;
  double a = 0.0;
  for (int w = 0; w < nw; ++w) a += (double)apart[((int64_t)p * nw + w) * ldg + r];
  beta[(int64_t)p * ldg + r] = (float)a;
}

// E^T and h of CPT consecutive columns nb .. nb + CPT - 1 of one window (the class of nb is
// k_first) and beta of their probe p, at rows r .. r + 3.  Addresses are clamped into the valid
// columns and rows (r0 is a valid row), so every value is finite; nt_store_g zeroes the rows
// beyond re.
template <int CPT>
__device__ __forceinline__ void nt_load_e(const float* __restrict__ GT, int64_t ldg,
                                          const float* __restrict__ HT, int64_t ldh,
                                          const float* __restrict__ beta, int p, int nb,
                                          int nvalid, int k_first, int64_t r, int64_t re,
                                          int64_t r0, f4 (&gv)[CPT], f4 (&hv)[CPT], f4& bt) {
  const int64_t rr = r < re ? r : r0;
#pragma unroll
  for (int t = 0; t < CPT; ++t) {
    const int tt = t < nvalid ? t : 0;
    gv[t] = *reinterpret_cast<const f4*>(GT + (int64_t)(nb + tt) * ldg + rr);
    hv[t] = *reinterpret_cast<const f4*>(HT + (int64_t)(k_first + tt) * ldh + rr);
  }
  bt = *reinterpret_cast<const f4*>(beta + (int64_t)p * ldg + rr);
}
// G'^T = (E^T - beta) h of the CPT columns (rows jl .. jl + CPT - 1 of the LDS tile b[n][k], row
// stride SK) at k offset rk; rows at or beyond re stage as zero (re is a multiple of 4 except at
// the end of the rows).  Columns beyond the window (t >= nvalid) stage the finite values of the
// clamped loads: they only reach output columns that the epilogue drops.
template <int CPT, int SK>
__device__ __forceinline__ void nt_store_g(float* __restrict__ b, int jl, int rk, int64_t r,
                                           int64_t re, const f4 (&gv)[CPT], const f4 (&hv)[CPT],
                                           const f4& bt) {
  const bool full = r + 3 < re;
#pragma unroll
  for (int t = 0; t < CPT; ++t) {
    f4 x;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float y = (gv[t][v] - bt[v]) * hv[t][v];
      x[v] = full || r + v < re ? y : 0.f;
    }
    *reinterpret_cast<f4*>(b + (jl + t) * SK + rk) = x;
  }
}

// Kernel 2.  Output tiles: a-tile mt (kNtBM values of a) x column tile ct (a column window of one
// probe, as in kernel 1), split sp of the chunk's rows.  B is staged as G'^T[n][r] = (E^T[n][r] - beta[p][r]) h_rk with
// p = n / c, k = n % c.  Thread tid stages columns n0 + 4 (tid / 8) + t, t = 0..3, at rows
// 4 (tid % 8) of the stage: E^T and h are fetched before the stage's products, beta (at most two
// probes among four consecutive columns) after them.
template <int KS, int MINB>
__global__ __launch_bounds__(kNtWG, MINB) void k_nt_xtg(
    const float* __restrict__ XT, int64_t ldx, int d, const float* __restrict__ GT, int64_t ldg,
    int SC, int c, int nw, const float* __restrict__ HT, int64_t ldh,
    const float* __restrict__ beta, int64_t R, int64_t rows_per_split, int nmt, int nct,
    float* __restrict__ part, int64_t part_stride, int accumulate, Skip skip) {
  if (skip_now(skip)) return;
  extern __shared__ __align__(16) float nt_lds[];
  constexpr int SK = nt_sk<KS>();
  constexpr int VR = KS / 4;          // 16-byte row vectors per stage row
  constexpr int CPT = KS / 8;         // columns staged per thread (4 rows each)
  float* As = nt_lds;
  float* Bs = nt_lds + 2 * kNtBM * SK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t lid = nt_lid(blockIdx.x, gridDim.x);
  const int mt = (int)(lid % nmt);
  const int64_t rest = lid / nmt;
  const int ct = (int)(rest % nct);
  const int sp = (int)(rest / nct);
  // column tiles are windows of one probe (probe fastest, as in the first contraction)
  const int ns = nct / nw;
  const int w = ct / ns, p = ct - w * ns;
  const int col0w = w * kNtBN;
  const int width = c - col0w < kNtBN ? c - col0w : kNtBN;
  const int a0 = mt * kNtBM;
  const int n0 = p * c + col0w;
  const int64_t rb = (int64_t)sp * rows_per_split;
  const int64_t re = rb + rows_per_split < R ? rb + rows_per_split : R;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // B staging: columns nb + t (t < CPT, all of probe p) at rows 4 (tid % VR) .. + 3 of the
  // stage; their classes and validity are fixed per thread
  const int jl = CPT * (tid / VR);           // first of the thread's columns in the window
  const int nb = n0 + jl;
  const int rk = 4 * (tid % VR);
  const int nvalid = width - jl < CPT ? (width - jl > 0 ? width - jl : 0) : CPT;
  // with no valid column the loads are made from the window's first column (and zeroed)
  const int nb_c = nvalid > 0 ? nb : n0;
  const int k_first = nvalid > 0 ? col0w + jl : col0w;
  f4 ra[KS / 8], gv[CPT], hv[CPT], bt;
  const int64_t nrows = re > rb ? re - rb : 0;
  const int nst = (int)((nrows + KS - 1) / KS);
  if (nst > 0) {
    const unsigned ma = nt_load<KS>(XT + (int64_t)a0 * ldx, ldx, 0, d - a0, rb, re, tid, ra);
    nt_load_e<CPT>(GT, ldg, HT, ldh, beta, p, nb_c, nvalid, k_first, rb + rk, re, rb, gv, hv, bt);
    nt_store<KS>(As, tid, ra, ma);
    nt_store_g<CPT, SK>(Bs, jl, rk, rb + rk, re, gv, hv, bt);
  }
  __syncthreads();
  // every pass loads the next stage (past the last one the rows are out of range: clamped
  // addresses, staged as zero into the buffer no later stage reads)
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    const int64_t k1 = rb + (int64_t)(st + 1) * KS;
    const unsigned ma = nt_load<KS>(XT + (int64_t)a0 * ldx, ldx, 0, d - a0, k1, re, tid, ra);
    nt_load_e<CPT>(GT, ldg, HT, ldh, beta, p, nb_c, nvalid, k_first, k1 + rk, re, rb, gv, hv,
                   bt);
    nt_order();
    nt_stage<KS>(As + buf * kNtBM * SK, Bs + buf * kNtBN * SK, wm, wn, li, g, acc);
    nt_order();
    nt_store<KS>(As + (buf ^ 1) * kNtBM * SK, tid, ra, ma);
    nt_store_g<CPT, SK>(Bs + (buf ^ 1) * kNtBN * SK, jl, rk, k1 + rk, re, gv, hv, bt);
    __syncthreads();
  }
  nt_xtg_epilogue(acc, part, sp, part_stride, a0, n0, n0 + width, wm, wn, li, g, d, SC,
                  accumulate);
}

// The FP32 second contraction with one workgroup of 4 MT waves over all d <= 128 MT output rows
// (as k_nt3_xtg_m below), 32-deep stages: each E^T tile is loaded and formed into G' once
// instead of once per 128-row tile.  The X^T stage goes straight into LDS
// (global_load_lds_dwordx4) as unpadded rows of 32 floats, eight 16-byte chunks, chunk q of
// row a stored at q ^ (a & 7): one instruction fills 8 rows and each lane fetches the chunk the
// swizzle puts in its slot; a fragment read (16 rows, one chunk) then meets distinct banks.
// B is staged through registers by the first 512 threads, two columns by four rows each.
template <int MT>
__device__ __forceinline__ void nt_load_lds32(const float* __restrict__ src, int64_t ld,
                                              int64_t nrow, int64_t k0, int64_t nk, int wave,
                                              int lane, float* __restrict__ dst) {
#pragma unroll 1
  for (int j = 0; j < 4; ++j) {   // blocks of 8 rows: 4 per wave
    const int blk = wave + 4 * MT * j;
    const int row = 8 * blk + (lane >> 3);
    const int ch = (lane & 7) ^ (row & 7);
    const int64_t k = k0 + 4 * ch;
    const bool ok = row < nrow && k < nk;
    const int64_t o = ok ? row * ld + k : 0;
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src + o),
                                     reinterpret_cast<void*>(dst + 8 * blk * 32), 16, 0, 0);
  }
}

__device__ __forceinline__ void nt_stage_m32(const float* __restrict__ a,
                                             const float* __restrict__ b, int wm, int wn, int li,
                                             int g, f32x4 (&acc)[4][4]) {
  constexpr int SK = nt_sk<32>();
#pragma unroll
  for (int kg = 0; kg < 2; ++kg) {
    f4 av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wm + 16 * i + li;
      av[i] = *reinterpret_cast<const f4*>(a + row * 32 + 4 * ((4 * kg + g) ^ (row & 7)));
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      bv[j] = *reinterpret_cast<const f4*>(b + (wn + 16 * j + li) * SK + 16 * kg + 4 * g);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][q], bv[j][q], acc[i][j], 0, 0, 0);
  }
}

template <int MT>
constexpr size_t ntm_lds_bytes() {
  return (size_t)2 * kNtBM * MT * 32 * 4 + (size_t)2 * kNtBN * nt_sk<32>() * 4;
}

template <int MT>
__global__ __launch_bounds__(256 * MT, 1) void k_nt_xtg_m(
    const float* __restrict__ XT, int64_t ldx, int d, const float* __restrict__ GT, int64_t ldg,
    int SC, int c, int nw, const float* __restrict__ HT, int64_t ldh,
    const float* __restrict__ beta, int64_t R, int64_t rows_per_split, int nct,
    float* __restrict__ part, int64_t part_stride, int accumulate, Skip skip) {
  if (skip_now(skip)) return;
  constexpr int KS = 32, SK = nt_sk<KS>(), TMR = kNtBM * MT;
  constexpr int PA = TMR * 32, PB = kNtBN * SK;   // one buffer of each operand, floats
  extern __shared__ __align__(16) float nt_lds[];
  float* As = nt_lds;              // [2][TMR][32], swizzled
  float* Bs = nt_lds + 2 * PA;     // [2][128][SK]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t lid = nt_lid(blockIdx.x, gridDim.x);
  const int ct = (int)(lid % nct);
  const int sp = (int)(lid / nct);
  const int ns = nct / nw;
  const int w = ct / ns, p = ct - w * ns;
  const int col0w = w * kNtBN;
  const int width = c - col0w < kNtBN ? c - col0w : kNtBN;
  const int n0 = p * c + col0w;
  const int64_t rb = (int64_t)sp * rows_per_split;
  const int64_t re = rb + rows_per_split < R ? rb + rows_per_split : R;
  const int q = wave & 3;
  const int wm = (wave >> 2) * kNtBM + (q >> 1) * 64, wn = (q & 1) * 64;

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const bool bst = tid < 512;                  // this thread stages B (whole waves)
  const int jl = 2 * ((tid & 511) >> 3);
  const int nb = n0 + jl;
  const int rk = 4 * (tid & 7);
  const int nvalid = width - jl < 2 ? (width - jl > 0 ? width - jl : 0) : 2;
  const int nb_c = nvalid > 0 ? nb : n0;
  const int k_first = nvalid > 0 ? col0w + jl : col0w;
  f4 gv[2], hv[2], bt;
  const int64_t nrows = re > rb ? re - rb : 0;
  const int nst = (int)((nrows + KS - 1) / KS);
  constexpr int kWaitVm0 = 0x0F70;   // vmcnt(0), no wait on the other counters
  if (nst > 0) {
    nt_load_lds32<MT>(XT, ldx, d, rb, re, wave, lane, As);
    if (bst) nt_load_e<2>(GT, ldg, HT, ldh, beta, p, nb_c, nvalid, k_first, rb + rk, re, rb, gv, hv, bt);
    if (bst) nt_store_g<2, SK>(Bs, jl, rk, rb + rk, re, gv, hv, bt);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    const int64_t k1 = rb + (int64_t)(st + 1) * KS;
    // the other buffer was last read before the previous barrier
    nt_load_lds32<MT>(XT, ldx, d, k1, re, wave, lane, As + (buf ^ 1) * PA);
    if (bst) nt_load_e<2>(GT, ldg, HT, ldh, beta, p, nb_c, nvalid, k_first, k1 + rk, re, rb, gv, hv, bt);
    nt_order();
    nt_stage_m32(As + buf * PA, Bs + buf * PB, wm, wn, li, g, acc);
    nt_order();
    if (bst) nt_store_g<2, SK>(Bs + (buf ^ 1) * PB, jl, rk, k1 + rk, re, gv, hv, bt);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
  }
  nt_xtg_epilogue(acc, part, sp, part_stride, 0, n0, n0 + width, wm, wn, li, g, d, SC,
                  accumulate);
}

// ------------------------------------------------------------------ bf16x3 form
// The same two contractions with every product taken as hi*hi + hi*lo + lo*hi of bf16 halves
// (hi = bf16(x), lo = bf16(x - hi), round to nearest even) on v_mfma_f32_16x16x32_bf16 with FP32
// accumulation.  A stage holds 32 k of each operand as two bf16 planes [row][32] (64 bytes per
// row, four 16-byte chunks, chunk q of row m stored at chunk q ^ ((m >> 2) & 3) so that the 16
// lanes of a fragment read fall in distinct banks).  Lane (g, li) reads k = 8 g .. 8 g + 7 of
// row li: one 16-byte read per plane and operand feeds the three products of a block.
// Operands: k_nt3_xv takes X from the context's hi/lo planes and V^T from planes made once per
// call; k_nt3_xtg takes X^T from the context's transposed planes and splits G' = (E - beta) h as
// it is staged.  The epilogues are those of the FP32 kernels.
constexpr size_t kNt3Lds = (size_t)2 * 2 * (kNtBM + kNtBN) * 32 * 2;   // 65,536 bytes
constexpr size_t kNt3XvLds = kNt3Lds / 2;   // single-buffered first contraction

__device__ __forceinline__ bf16x8 nt3_zero8() {
  bf16x8 z;
#pragma unroll
  for (int u = 0; u < 8; ++u) z[u] = (__bf16)0.0f;
  return z;
}

__device__ __forceinline__ int nt3_off(int plane, int row, int ch) {   // in bf16 elements
  return (plane * kNtBM + row) * 32 + ((ch ^ ((row >> 2) & 3)) << 3);
}

// One 32-deep stage of a wave's 4 x 4 blocks from hi/lo LDS planes a[2][128][32], b[2][128][32].
__device__ __forceinline__ void nt3_stage(const __bf16* __restrict__ a,
                                          const __bf16* __restrict__ b, int wm, int wn, int li,
                                          int g, f32x4 (&acc)[4][4]) {
  bf16x8 ah[4], al[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = wm + 16 * i + li;
    ah[i] = *reinterpret_cast<const bf16x8*>(a + nt3_off(0, row, g));
    al[i] = *reinterpret_cast<const bf16x8*>(a + nt3_off(1, row, g));
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = wn + 16 * j + li;
    const bf16x8 bh = *reinterpret_cast<const bf16x8*>(b + nt3_off(0, row, g));
    const bf16x8 bl = *reinterpret_cast<const bf16x8*>(b + nt3_off(1, row, g));
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i][j] = mfma3(ah[i], al[i], bh, bl, acc[i][j]);
  }
}

// A 128 x 32 tile of two row-major bf16 planes (leading dimension ld): 512 16-byte chunks per
// plane, two per thread: chunk e = tid + 256 t is row e / 4, k 8 (e % 4).  Rows at or beyond
// nrow and k at or beyond nk read element 0 (a valid address) and are cleared by nt3_store
// through the returned mask (nk a multiple of 8).
__device__ __forceinline__ unsigned nt3_load(const __bf16* __restrict__ hi,
                                             const __bf16* __restrict__ lo, int64_t ld,
                                             int64_t nrow, int64_t k0, int64_t nk, int tid,
                                             bf16x8 (&vh)[2], bf16x8 (&vl)[2]) {
  unsigned m = 0;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int e = tid + kNtWG * t, row = e >> 2, ch = e & 3;
    const int64_t k = k0 + 8 * ch;
    const bool ok = row < nrow && k < nk;
    const int64_t o = ok ? row * ld + k : 0;
    vh[t] = *reinterpret_cast<const bf16x8*>(hi + o);
    vl[t] = *reinterpret_cast<const bf16x8*>(lo + o);
    m |= (unsigned)ok << t;
  }
  return m;
}
__device__ __forceinline__ void nt3_store(__bf16* __restrict__ dst, int tid, const bf16x8 (&vh)[2],
                                          const bf16x8 (&vl)[2], unsigned m) {
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int e = tid + kNtWG * t, row = e >> 2, ch = e & 3;
    const bool ok = (m >> t) & 1u;
    *reinterpret_cast<bf16x8*>(dst + nt3_off(0, row, ch)) = ok ? vh[t] : nt3_zero8();
    *reinterpret_cast<bf16x8*>(dst + nt3_off(1, row, ch)) = ok ? vl[t] : nt3_zero8();
  }
}

template <bool OM>
__global__ __launch_bounds__(kNtWG, 3) void k_nt3_xv(
    const __bf16* __restrict__ Xh, const __bf16* __restrict__ Xl, int d, int64_t R,
    const __bf16* __restrict__ VTh, const __bf16* __restrict__ VTl, int c, int nw, int ntc,
    const float* __restrict__ HT, int64_t ldh, const double* __restrict__ omega,
    float* __restrict__ GT, int64_t ldg, float* __restrict__ apart, Skip skip) {
  if (skip_now(skip)) return;
  extern __shared__ __align__(16) float nt_lds[];
  // one buffer per operand (two planes): 32 KB, three workgroups per CU, whose epilogues (the
  // E^T stores) overlap the others' main loops better than two double-buffered workgroups'
  __bf16* As = reinterpret_cast<__bf16*>(nt_lds);      // [2 planes][128][32]
  __bf16* Bs = As + 2 * kNtBM * 32;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t lid = nt_lid(blockIdx.x, gridDim.x);
  const int64_t nrt = (R + kNtBM - 1) / kNtBM;
  const int64_t grp = lid / (8 * (int64_t)ntc);
  const int64_t g0 = grp * 8;
  const int64_t gsz = nrt - g0 < 8 ? nrt - g0 : 8;
  const int64_t in = lid - grp * 8 * (int64_t)ntc;
  const int ct = (int)(in / gsz);
  const int64_t rt = g0 + (in - (int64_t)ct * gsz);
  // column tiles with the probe fastest: consecutive tiles share the window's classes (h)
  const int ns = ntc / nw;
  const int w = ct / ns, p = ct - w * ns;
  const int64_t row0 = rt * kNtBM;
  const int col0 = w * kNtBN;
  const int width = c - col0 < kNtBN ? c - col0 : kNtBN;
  const int64_t n0 = (int64_t)p * c + col0;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  bf16x8 ah[2], al[2], bh[2], bl[2];
  const __bf16* xh = Xh + row0 * d;
  const __bf16* xl = Xl + row0 * d;
  const __bf16* vh = VTh + n0 * d;
  const __bf16* vl = VTl + n0 * d;
  const int nst = (d + kNtKS - 1) / kNtKS;
  unsigned ma = nt3_load(xh, xl, d, R - row0, 0, d, tid, ah, al);
  unsigned mb = nt3_load(vh, vl, d, width, 0, d, tid, bh, bl);
  nt3_store(As, tid, ah, al, ma);
  nt3_store(Bs, tid, bh, bl, mb);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {   // loads of the next stage on every pass, as in FP32
    ma = nt3_load(xh, xl, d, R - row0, (int64_t)(st + 1) * kNtKS, d, tid, ah, al);
    mb = nt3_load(vh, vl, d, width, (int64_t)(st + 1) * kNtKS, d, tid, bh, bl);
    nt_order();
    nt3_stage(As, Bs, wm, wn, li, g, acc);
    __syncthreads();   // every wave is done with the buffers
    nt3_store(As, tid, ah, al, ma);
    nt3_store(Bs, tid, bh, bl, mb);
    __syncthreads();
  }
  nt_xv_epilogue<OM>(acc, nt_lds, wave, wm, wn, li, g, tid, row0, R, width, col0, n0, p, w, nw,
                     HT, ldh, omega, GT, ldg, apart);
}

// G'^T = (E^T - beta[p]) h of four columns at rows r .. r + 3 (rows at or beyond re as zero;
// columns beyond the window as in nt_store_g), split into hi/lo bf16 and stored into the planes
// of the LDS tile (row 4 (tid / 8) + t, k 4 (tid % 8)).
__device__ __forceinline__ void nt3_store_g(__bf16* __restrict__ b, int tid, int64_t r, int64_t re,
                                            const f4 (&gv)[4], const f4 (&hv)[4], const f4& bt) {
  const bool full = r + 3 < re;
  const int kq = 4 * (tid & 7);              // k offset of the four rows within the stage
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    bf16x4 h4, l4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float y = (gv[t][v] - bt[v]) * hv[t][v];
      const float x = full || r + v < re ? y : 0.f;
      const __bf16 h = (__bf16)x;
      h4[v] = h;
      l4[v] = (__bf16)(x - (float)h);
    }
    const int row = 4 * (tid >> 3) + t;
    *reinterpret_cast<bf16x4*>(b + nt3_off(0, row, kq >> 3) + (kq & 4)) = h4;
    *reinterpret_cast<bf16x4*>(b + nt3_off(1, row, kq >> 3) + (kq & 4)) = l4;
  }
}

__global__ __launch_bounds__(kNtWG, 2) void k_nt3_xtg(
    const __bf16* __restrict__ XTh, const __bf16* __restrict__ XTl, int64_t ldx, int d,
    const float* __restrict__ GT, int64_t ldg, int SC, int c, int nw, const float* __restrict__ HT,
    int64_t ldh, const float* __restrict__ beta, int64_t R, int64_t rows_per_split, int nmt,
    int nct, float* __restrict__ part, int64_t part_stride, int accumulate, Skip skip) {
  if (skip_now(skip)) return;
  extern __shared__ __align__(16) float nt_lds[];
  __bf16* As = reinterpret_cast<__bf16*>(nt_lds);
  __bf16* Bs = As + 2 * 2 * kNtBM * 32;
  constexpr int PL = 2 * kNtBM * 32;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t lid = nt_lid(blockIdx.x, gridDim.x);
  const int mt = (int)(lid % nmt);
  const int64_t rest = lid / nmt;
  const int ct = (int)(rest % nct);
  const int sp = (int)(rest / nct);
  // column tiles are windows of one probe (probe fastest, as in the first contraction)
  const int ns = nct / nw;
  const int w = ct / ns, p = ct - w * ns;
  const int col0w = w * kNtBN;
  const int width = c - col0w < kNtBN ? c - col0w : kNtBN;
  const int a0 = mt * kNtBM;
  const int n0 = p * c + col0w;
  const int64_t rb = (int64_t)sp * rows_per_split;
  const int64_t re = rb + rows_per_split < R ? rb + rows_per_split : R;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int jl = 4 * (tid >> 3);               // first of the thread's columns in the window
  const int nb = n0 + jl;
  const int rk = 4 * (tid & 7);
  const int nvalid = width - jl < 4 ? (width - jl > 0 ? width - jl : 0) : 4;
  // with no valid column the loads are made from the window's first column (and zeroed)
  const int nb_c = nvalid > 0 ? nb : n0;
  const int k_first = nvalid > 0 ? col0w + jl : col0w;
  bf16x8 ah[2], al[2];
  f4 gv[4], hv[4], bt;
  const __bf16* xh = XTh + (int64_t)a0 * ldx;
  const __bf16* xl = XTl + (int64_t)a0 * ldx;
  const int64_t nrows = re > rb ? re - rb : 0;
  const int nst = (int)((nrows + kNtKS - 1) / kNtKS);
  // X^T rows are read 8 at a time: rows beyond re (a multiple of 8 except at the end of the
  // pool) come from the padding or the next rows and meet zero in B
  if (nst > 0) {
    const unsigned ma = nt3_load(xh, xl, ldx, d - a0, rb, re, tid, ah, al);
    nt_load_e<4>(GT, ldg, HT, ldh, beta, p, nb_c, nvalid, k_first, rb + rk, re, rb, gv, hv, bt);
    nt3_store(As, tid, ah, al, ma);
    nt3_store_g(Bs, tid, rb + rk, re, gv, hv, bt);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {   // loads of the next stage on every pass, as in FP32
    const int buf = st & 1;
    const int64_t k1 = rb + (int64_t)(st + 1) * kNtKS;
    const unsigned ma = nt3_load(xh, xl, ldx, d - a0, k1, re, tid, ah, al);
    nt_load_e<4>(GT, ldg, HT, ldh, beta, p, nb_c, nvalid, k_first, k1 + rk, re, rb, gv, hv, bt);
    nt_order();
    nt3_stage(As + buf * PL, Bs + buf * PL, wm, wn, li, g, acc);
    nt_order();
    nt3_store(As + (buf ^ 1) * PL, tid, ah, al, ma);
    nt3_store_g(Bs + (buf ^ 1) * PL, tid, k1 + rk, re, gv, hv, bt);
    __syncthreads();
  }
  nt_xtg_epilogue(acc, part, sp, part_stride, a0, n0, n0 + width, wm, wn, li, g, d, SC,
                  accumulate);
}

// The bf16x3 second contraction with one workgroup over all d <= 128 MT output rows: MT row
// tiles of 128, four waves each (waves 4 m .. 4 m + 3 on row tile m, in the 2 x 2 arrangement
// of the kernel above), so that each E^T tile is loaded, turned into G' and split into bf16
// halves once instead of once per row tile.  X^T planes [2][128 MT][32] per buffer; B as above,
// staged by the first 512 threads, two columns by four rows each (MT = 3: waves 8-11 stage X^T
// only).  One workgroup per CU (128 KB of LDS at MT = 3).
template <int PR>
__device__ __forceinline__ int nt3_offp(int plane, int row, int ch) {   // plane of PR rows
  return (plane * PR + row) * 32 + ((ch ^ ((row >> 2) & 3)) << 3);
}

template <int PA>
__device__ __forceinline__ void nt3_stage_p(const __bf16* __restrict__ a,
                                            const __bf16* __restrict__ b, int wm, int wn, int li,
                                            int g, f32x4 (&acc)[4][4]) {
  bf16x8 ah[4], al[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = wm + 16 * i + li;
    ah[i] = *reinterpret_cast<const bf16x8*>(a + nt3_offp<PA>(0, row, g));
    al[i] = *reinterpret_cast<const bf16x8*>(a + nt3_offp<PA>(1, row, g));
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = wn + 16 * j + li;
    const bf16x8 bh = *reinterpret_cast<const bf16x8*>(b + nt3_off(0, row, g));
    const bf16x8 bl = *reinterpret_cast<const bf16x8*>(b + nt3_off(1, row, g));
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i][j] = mfma3(ah[i], al[i], bh, bl, acc[i][j]);
  }
}

// X^T rows 0 .. 128 MT - 1, 32 k of two planes: 512 MT 16-byte chunks per plane, two per
// thread; rows at or beyond nrow and k at or beyond nk read element 0 and are cleared at the
// store through the returned mask.
template <int MT>
__device__ __forceinline__ unsigned nt3_load_m(const __bf16* __restrict__ hi,
                                               const __bf16* __restrict__ lo, int64_t ld,
                                               int64_t nrow, int64_t k0, int64_t nk, int tid,
                                               bf16x8 (&vh)[2], bf16x8 (&vl)[2]) {
  unsigned m = 0;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int e = tid + 256 * MT * t, row = e >> 2, ch = e & 3;
    const int64_t k = k0 + 8 * ch;
    const bool ok = row < nrow && k < nk;
    const int64_t o = ok ? row * ld + k : 0;
    vh[t] = *reinterpret_cast<const bf16x8*>(hi + o);
    vl[t] = *reinterpret_cast<const bf16x8*>(lo + o);
    m |= (unsigned)ok << t;
  }
  return m;
}
template <int MT>
__device__ __forceinline__ void nt3_store_m(__bf16* __restrict__ dst, int tid,
                                            const bf16x8 (&vh)[2], const bf16x8 (&vl)[2],
                                            unsigned m) {
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int e = tid + 256 * MT * t, row = e >> 2, ch = e & 3;
    const bool ok = (m >> t) & 1u;
    *reinterpret_cast<bf16x8*>(dst + nt3_offp<kNtBM * MT>(0, row, ch)) = ok ? vh[t] : nt3_zero8();
    *reinterpret_cast<bf16x8*>(dst + nt3_offp<kNtBM * MT>(1, row, ch)) = ok ? vl[t] : nt3_zero8();
  }
}

// G'^T = (E^T - beta[p]) h of CPT columns jl .. jl + CPT - 1 at rows r .. r + 3 (k offset rk of
// the stage), split into hi/lo bf16 planes of the LDS tile; rows at or beyond re as zero.
template <int CPT>
__device__ __forceinline__ void nt3_store_gc(__bf16* __restrict__ b, int jl, int rk, int64_t r,
                                             int64_t re, const f4 (&gv)[CPT], const f4 (&hv)[CPT],
                                             const f4& bt) {
  const bool full = r + 3 < re;
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int t = 0; t < CPT; ++t) {
    bf16x4 h4, l4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float y = (gv[t][v] - bt[v]) * hv[t][v];
      const float x = full || r + v < re ? y : 0.f;
      const __bf16 h = (__bf16)x;
      h4[v] = h;
      l4[v] = (__bf16)(x - (float)h);
    }
    const int row = jl + t;
    *reinterpret_cast<bf16x4*>(b + nt3_off(0, row, rk >> 3) + (rk & 4)) = h4;
    *reinterpret_cast<bf16x4*>(b + nt3_off(1, row, rk >> 3) + (rk & 4)) = l4;
  }
}

// The X^T stage of k_nt3_xtg_m loaded straight into LDS (global_load_lds_dwordx4: lane L of a
// wave writes the 16 bytes at the instruction's LDS base + 16 L).  One instruction fills 16
// rows of one plane; lane L's slot is row 16 blk + L / 4, physical chunk L % 4, which under the
// swizzle of nt3_offp holds logical chunk (L % 4) ^ ((row / 4) % 4), so the lane fetches that
// chunk.  Rows at or beyond nrow and k at or beyond nk fetch element 0 of the plane: such rows
// of A only meet output rows the epilogue drops or rows of B staged as zero.  Wave w fills
// blocks w and w + 4 MT of each plane.
template <int MT>
__device__ __forceinline__ void nt3_load_lds(const __bf16* __restrict__ hi,
                                             const __bf16* __restrict__ lo, int64_t ld,
                                             int64_t nrow, int64_t k0, int64_t nk, int wave,
                                             int lane, __bf16* __restrict__ dst) {
  constexpr int TMR = kNtBM * MT;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int blk = wave + 4 * MT * j;
    const int row = 16 * blk + (lane >> 2);
    const int ch = (lane & 3) ^ ((row >> 2) & 3);
    const int64_t k = k0 + 8 * ch;
    const bool ok = row < nrow && k < nk;
    const int64_t o = ok ? row * ld + k : 0;
#pragma unroll
    for (int pl = 0; pl < 2; ++pl) {
      const __bf16* src = (pl == 0 ? hi : lo) + o;
      __bf16* base = dst + (pl * TMR + 16 * blk) * 32;   // 16 rows of 32 bf16: 1 KB
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src),
                                       reinterpret_cast<void*>(base), 16, 0, 0);
    }
  }
}

template <int MT>
constexpr size_t nt3m_lds_bytes() { return (size_t)2 * 2 * (kNtBM * MT + kNtBN) * 32 * 2; }

template <int MT>
__global__ __launch_bounds__(256 * MT, 1) void k_nt3_xtg_m(
    const __bf16* __restrict__ XTh, const __bf16* __restrict__ XTl, int64_t ldx, int d,
    const float* __restrict__ GT, int64_t ldg, int SC, int c, int nw, const float* __restrict__ HT,
    int64_t ldh, const float* __restrict__ beta, int64_t R, int64_t rows_per_split, int nct,
    float* __restrict__ part, int64_t part_stride, int accumulate, Skip skip) {
  if (skip_now(skip)) return;
  constexpr int TMR = kNtBM * MT;
  constexpr int PLA = 2 * TMR * 32, PLB = 2 * kNtBN * 32;   // one buffer's two planes
  extern __shared__ __align__(16) float nt_lds[];
  __bf16* As = reinterpret_cast<__bf16*>(nt_lds);   // [2 bufs][2 planes][TMR][32]
  __bf16* Bs = As + 2 * PLA;                         // [2 bufs][2 planes][128][32]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t lid = nt_lid(blockIdx.x, gridDim.x);
  const int ct = (int)(lid % nct);
  const int sp = (int)(lid / nct);
  const int ns = nct / nw;
  const int w = ct / ns, p = ct - w * ns;
  const int col0w = w * kNtBN;
  const int width = c - col0w < kNtBN ? c - col0w : kNtBN;
  const int n0 = p * c + col0w;
  const int64_t rb = (int64_t)sp * rows_per_split;
  const int64_t re = rb + rows_per_split < R ? rb + rows_per_split : R;
  const int q = wave & 3;
  const int wm = (wave >> 2) * kNtBM + (q >> 1) * 64, wn = (q & 1) * 64;

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const bool bst = tid < 512;                  // this thread stages B (whole waves)
  const int jl = 2 * ((tid & 511) >> 3);       // its first column in the window
  const int nb = n0 + jl;
  const int rk = 4 * (tid & 7);
  const int nvalid = width - jl < 2 ? (width - jl > 0 ? width - jl : 0) : 2;
  const int nb_c = nvalid > 0 ? nb : n0;
  const int k_first = nvalid > 0 ? col0w + jl : col0w;
  f4 gv[2], hv[2], bt;
  const int64_t nrows = re > rb ? re - rb : 0;
  const int nst = (int)((nrows + kNtKS - 1) / kNtKS);
  // vmcnt(0), no wait on the other counters: the direct-to-LDS loads of X^T have landed
  constexpr int kWaitVm0 = 0x0F70;
  if (nst > 0) {
    nt3_load_lds<MT>(XTh, XTl, ldx, d, rb, re, wave, lane, As);
    if (bst) nt_load_e<2>(GT, ldg, HT, ldh, beta, p, nb_c, nvalid, k_first, rb + rk, re, rb, gv, hv, bt);
    if (bst) nt3_store_gc<2>(Bs, jl, rk, rb + rk, re, gv, hv, bt);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    const int64_t k1 = rb + (int64_t)(st + 1) * kNtKS;
    // the other buffer was last read before the previous barrier
    nt3_load_lds<MT>(XTh, XTl, ldx, d, k1, re, wave, lane, As + (buf ^ 1) * PLA);
    if (bst) nt_load_e<2>(GT, ldg, HT, ldh, beta, p, nb_c, nvalid, k_first, k1 + rk, re, rb, gv, hv, bt);
    nt_order();
    nt3_stage_p<TMR>(As + buf * PLA, Bs + buf * PLB, wm, wn, li, g, acc);
    nt_order();
    if (bst) nt3_store_gc<2>(Bs + (buf ^ 1) * PLB, jl, rk, k1 + rk, re, gv, hv, bt);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
  }
  nt_xtg_epilogue(acc, part, sp, part_stride, 0, n0, n0 + width, wm, wn, li, g, d, SC,
                  accumulate);
}

// hi/lo bf16 planes of the transpose of an rows x cols row-major FP32 source: dst[j][i] for the
// cols x rows destination (leading dimension rows).
__global__ __launch_bounds__(256) void k_nt3_transpose_split(const float* __restrict__ src,
                                                             int64_t rows, int64_t cols,
                                                             __bf16* __restrict__ dh,
                                                             __bf16* __restrict__ dl) {
  __shared__ float tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int q = ty; q < 32; q += 8) {
    const int64_t i = i0 + q, j = j0 + tx;
    tile[q][tx] = (i < rows && j < cols) ? src[i * cols + j] : 0.f;
  }
  __syncthreads();
  for (int q = ty; q < 32; q += 8) {
    const int64_t j = j0 + q, i = i0 + tx;
    if (j < cols && i < rows) {
      const float v = tile[tx][q];
      const __bf16 h = (__bf16)v;
      dh[j * rows + i] = h;
      dl[j * rows + i] = (__bf16)(v - (float)h);
    }
  }
}

// dst[j][i] = src[i][j] for an rows x cols row-major source (leading dimension lds) into a
// destination with leading dimension ldd; entries of dst beyond rows (up to ldd) are zeroed.
__global__ __launch_bounds__(256) void k_nt_transpose(const float* __restrict__ src, int64_t rows,
                                                      int64_t cols, int64_t lds,
                                                      float* __restrict__ dst, int64_t ldd) {
  __shared__ float tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int q = ty; q < 32; q += 8) {
    const int64_t i = i0 + q, j = j0 + tx;
    tile[q][tx] = (i < rows && j < cols) ? src[i * lds + j] : 0.f;
  }
  __syncthreads();
  for (int q = ty; q < 32; q += 8) {
    const int64_t j = j0 + q, i = i0 + tx;
    if (j < cols && i < ldd) dst[j * ldd + i] = tile[tx][q];
  }
}

int nt_transpose(const float* src, int64_t rows, int64_t cols, int64_t lds, float* dst,
                 int64_t ldd, hipStream_t st) {
  dim3 grid((unsigned)cdiv(ldd, 32), (unsigned)cdiv(cols, 32));
  k_nt_transpose<<<grid, 256, 0, st>>>(src, rows, cols, lds, dst, ldd);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

DeviceOnce g_nt_attr;

}  // namespace

int nt3_split_vt(const float* B, int d, int SC, __bf16* VTh, __bf16* VTl, hipStream_t st) {
  dim3 grid((unsigned)cdiv(d, 32), (unsigned)cdiv(SC, 32));
  k_nt3_transpose_split<<<grid, 256, 0, st>>>(B, d, SC, VTh, VTl);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

// The wide path covers FP32 contexts with d % 4 == 0 and bf16x3 contexts with d % 8 == 0, both
// with d > 128 and c > 128; its transposed FP32 copies of H (and for FP32 of X; bf16x3 contexts
// read the transposed hi/lo planes of X) are made at creation when this holds.
bool nt_applies(const Ctx* x) {
  const bool form = (x->prec == FIRAL_F32 && x->d % 4 == 0) ||
                    (x->prec == FIRAL_BF16X3 && x->d % 8 == 0);
  return form && x->d > 128 && x->c > kNtBN;
}

int64_t nt_ld(int64_t rows) { return cdiv(rows, 4) * 4; }

// Column windows per probe of the wide path.
int nt_windows(int c) { return (int)cdiv(c, kNtBN); }

int nt_prepare_ctx(Ctx* x, hipStream_t st) {
  if (x->prec == FIRAL_F32)
    FIRAL_CHECK(nt_transpose((const float*)x->X, x->N, x->d, x->d, (float*)x->XTf, x->ldn, st));
  FIRAL_CHECK(nt_transpose((const float*)x->H, x->N, x->c, x->c, (float*)x->HTf, x->ldn, st));
  return FIRAL_OK;
}

int hvp_nt_launch(Ctx* x, const double* omega, int64_t n_rows, double shift, const float* B,
                  float* out, int s, Skip skip, hipStream_t st) {
  const int d = x->d, c = x->c, SC = s * c, nw = nt_windows(c);
  if (!g_nt_attr.done()) {
    for (const void* f : {(const void*)k_nt_xv<kNtKsXv, kNtMinbXv, true>,
                          (const void*)k_nt_xv<kNtKsXv, kNtMinbXv, false>})
      FIRAL_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)nt_lds_bytes<kNtKsXv>()));
    FIRAL_HIP(hipFuncSetAttribute((const void*)k_nt_xtg<kNtKsXtg, kNtMinbXtg>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)nt_lds_bytes<kNtKsXtg>()));
    for (const void* f : {(const void*)k_nt3_xv<true>, (const void*)k_nt3_xv<false>})
      FIRAL_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)kNt3XvLds));
    FIRAL_HIP(hipFuncSetAttribute((const void*)k_nt3_xtg,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kNt3Lds));
    FIRAL_HIP(hipFuncSetAttribute((const void*)k_nt3_xtg_m<2>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)nt3m_lds_bytes<2>()));
    FIRAL_HIP(hipFuncSetAttribute((const void*)k_nt_xtg_m<2>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)ntm_lds_bytes<2>()));
    FIRAL_HIP(hipFuncSetAttribute((const void*)k_nt_xtg_m<3>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)ntm_lds_bytes<3>()));
    FIRAL_HIP(hipFuncSetAttribute((const void*)k_nt3_xtg_m<3>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)nt3m_lds_bytes<3>()));
    g_nt_attr.set();
  }
  const bool bf3 = x->prec == FIRAL_BF16X3;
  // V^T: the probe block d x (s c) transposed to (s c) x d (bf16x3: its hi/lo planes)
  float* VT = (float*)x->VTf;
  __bf16* VTh = (__bf16*)x->VTf;
  __bf16* VTl = VTh + (int64_t)SC * d;
  if (bf3) {
    FIRAL_CHECK(nt3_split_vt(B, d, SC, VTh, VTl, st));
  } else {
    FIRAL_CHECK(nt_transpose(B, d, SC, SC, VT, d, st));
  }
  // buffers: E^T [s c][ldg], beta_part [s][nw][ldg], beta [s][ldg]
  const int64_t ldg = nt_ld(x->chunk_rows);
  float* GT = (float*)x->G;
  float* apart = (float*)x->ntpart;
  float* beta = apart + (int64_t)s * nw * ldg;
  float* part = (float*)x->part;
  const int64_t n_out = (int64_t)d * SC;
  const int nmt = (int)cdiv(d, kNtBM), nct = s * nw;   // column windows of every probe
  // d <= 384: one workgroup per column tile covers every output row
  const int mt_all = nmt == 2 || nmt == 3 ? nmt : 0;
  const int64_t tiles = mt_all ? (int64_t)nct : (int64_t)nmt * nct;
  const int64_t cap = (int64_t)x->max_splits * x->s_max / s;
  // split count: the second contraction runs two workgroups per CU, so a grid of tiles * S
  // workgroups takes ceil(tiles * S / slots) rounds of R / S rows each; take the S with the least
  // time in rounds (the smallest such S: fewest partial sums), with at least 8 stages per split
  const int64_t slots = (int64_t)(mt_all ? 1 : 2) * std::max(1, x->n_cu);
  const int64_t s_hi = std::max<int64_t>(1, std::min<int64_t>({cap, 256, cdiv(x->chunk_rows, 8 * kNtKS)}));
  int S = 1;
  for (int64_t t = 2; t <= s_hi; ++t)   // rounds / S, compared as cross products
    if (cdiv(tiles * t, slots) * S < cdiv(tiles * S, slots) * t) S = (int)t;
  const int ntc = s * nw;
  for (int64_t r0 = 0; r0 < n_rows; r0 += x->chunk_rows) {
    const int64_t R = std::min<int64_t>(x->chunk_rows, n_rows - r0);
    hipEvent_t e0, e1;
    FIRAL_CHECK(prof_pair(x, FIRAL_PROF_PRODUCT, &e0, &e1));
    const dim3 grid1((unsigned)(cdiv(R, kNtBM) * ntc));
    const double* om = omega ? omega + r0 : nullptr;
    if (bf3)
      hipExtLaunchKernelGGL(omega ? k_nt3_xv<true> : k_nt3_xv<false>, grid1, dim3(kNtWG),
                            (uint32_t)kNt3XvLds, st, e0, e1, 0u, (const __bf16*)x->Xhi + r0 * d,
                            (const __bf16*)x->Xlo + r0 * d, d, R, (const __bf16*)VTh,
                            (const __bf16*)VTl, c, nw, ntc, (const float*)x->HTf + r0, x->ldn, om,
                            GT, ldg, apart, skip);
    else
      hipExtLaunchKernelGGL(omega ? k_nt_xv<kNtKsXv, kNtMinbXv, true>
                                  : k_nt_xv<kNtKsXv, kNtMinbXv, false>,
                            grid1, dim3(kNtWG), (uint32_t)nt_lds_bytes<kNtKsXv>(), st, e0, e1, 0u,
                            (const float*)x->X + r0 * d, d, R, (const float*)VT, c, nw, ntc,
                            (const float*)x->HTf + r0, x->ldn, om, GT, ldg, apart, skip);
    FIRAL_LAUNCHED();
    k_nt_alpha<<<(unsigned)cdiv((int64_t)s * R, 256), 256, 0, st>>>(apart, nw, s, R, ldg, beta,
                                                                     skip);
    FIRAL_LAUNCHED();
    // splits start on multiples of 32 rows (the stage depth)
    const int64_t rps = cdiv(cdiv(R, S), kNtKS) * kNtKS;
    FIRAL_CHECK(prof_pair(x, FIRAL_PROF_PRODUCT_T, &e0, &e1));
    const dim3 grid2((unsigned)(tiles * S));
    if (!bf3 && mt_all == 3)
      hipExtLaunchKernelGGL(k_nt_xtg_m<3>, grid2, dim3(3 * kNtWG), (uint32_t)ntm_lds_bytes<3>(),
                            st, e0, e1, 0u, (const float*)x->XTf + r0, x->ldn, d,
                            (const float*)GT, ldg, SC, c, nw, (const float*)x->HTf + r0, x->ldn,
                            (const float*)beta, R, rps, nct, part, n_out, (int)(r0 > 0), skip);
    else if (!bf3 && mt_all == 2)
      hipExtLaunchKernelGGL(k_nt_xtg_m<2>, grid2, dim3(2 * kNtWG), (uint32_t)ntm_lds_bytes<2>(),
                            st, e0, e1, 0u, (const float*)x->XTf + r0, x->ldn, d,
                            (const float*)GT, ldg, SC, c, nw, (const float*)x->HTf + r0, x->ldn,
                            (const float*)beta, R, rps, nct, part, n_out, (int)(r0 > 0), skip);
    else if (mt_all == 3)
      hipExtLaunchKernelGGL(k_nt3_xtg_m<3>, grid2, dim3(3 * kNtWG), (uint32_t)nt3m_lds_bytes<3>(),
                            st, e0, e1, 0u, (const __bf16*)x->XThi + r0,
                            (const __bf16*)x->XTlo + r0, x->ldt, d, (const float*)GT, ldg, SC, c,
                            nw, (const float*)x->HTf + r0, x->ldn, (const float*)beta, R, rps, nct,
                            part, n_out, (int)(r0 > 0), skip);
    else if (mt_all == 2)
      hipExtLaunchKernelGGL(k_nt3_xtg_m<2>, grid2, dim3(2 * kNtWG), (uint32_t)nt3m_lds_bytes<2>(),
                            st, e0, e1, 0u, (const __bf16*)x->XThi + r0,
                            (const __bf16*)x->XTlo + r0, x->ldt, d, (const float*)GT, ldg, SC, c,
                            nw, (const float*)x->HTf + r0, x->ldn, (const float*)beta, R, rps, nct,
                            part, n_out, (int)(r0 > 0), skip);
    else if (bf3)
      hipExtLaunchKernelGGL(k_nt3_xtg, grid2, dim3(kNtWG), (uint32_t)kNt3Lds, st, e0, e1, 0u,
                            (const __bf16*)x->XThi + r0, (const __bf16*)x->XTlo + r0, x->ldt, d,
                            (const float*)GT, ldg, SC, c, nw, (const float*)x->HTf + r0, x->ldn,
                            (const float*)beta, R, rps, nmt, nct, part, n_out, (int)(r0 > 0),
                            skip);
    else
      hipExtLaunchKernelGGL(k_nt_xtg<kNtKsXtg, kNtMinbXtg>, grid2, dim3(kNtWG),
                            (uint32_t)nt_lds_bytes<kNtKsXtg>(), st, e0, e1, 0u,
                            (const float*)x->XTf + r0, x->ldn, d, (const float*)GT, ldg, SC, c, nw,
                            (const float*)x->HTf + r0, x->ldn, (const float*)beta, R, rps, nmt,
                            nct, part, n_out, (int)(r0 > 0), skip);
    FIRAL_LAUNCHED();
  }
  return reduce_parts_launch<float>(part, n_out, n_rows > 0 ? S : 0, shift, B, out, skip, st);
}

}  // namespace firal
