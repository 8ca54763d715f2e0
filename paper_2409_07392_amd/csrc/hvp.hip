// Matrix-free Hessian product of Lemma 1, aggregated over rows:
//   out_j = sum_i omega_i H_i v_j + shift v_j,  H_i = Gamma_i (x) x_i x_i^T.
//
// With the block layout (a, j, k) the per-row steps of the lemma become two
// contractions around a row-local epilogue:
//   G  = X V                   (rows x s*c; gamma_ij = V_j^T x_i for every probe)
//   G' = omega * (G - alpha) * h   per row and probe, alpha_ij = gamma_ij . h_i
//   out = X^T G' + shift V     (sum over rows of vec(x_i gamma_ij^T))
// Rows are processed in chunks so that the intermediate stays bounded; the
// X^T G' contraction is split over rows into partial buffers that a final
// pass sums in a fixed order (no float atomics: results are reproducible).
#include <algorithm>

#include "common.h"

namespace firal {

constexpr int TM = 64, TN = 64, TK = 16;

// G[r, col] = sum_a X[r, a] Bm[a, col], r < R (X is a chunk of rows, leading dim d).
// Workgroup: 64 x 64 output tile, four waves of 32 x 32 (2 x 2 MFMA blocks).
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_xb(const T* __restrict__ X, int d,
                                                 const T* __restrict__ Bm, int SC,
                                                 T* __restrict__ G, int64_t R,
                                                 Skip skip) {
  if (skip_now(skip)) return;
  __shared__ T As[TK][TM + 4];
  __shared__ T Bs[TK][TN + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.y * TM;
  const int col0 = blockIdx.x * TN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  typedef Mfma16<T> M;
  typename M::acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = M::zero();

  for (int k0 = 0; k0 < d; k0 += TK) {
    for (int e = tid; e < TM * TK; e += 256) {
      const int r = e / TK, kk = e % TK;
      const int64_t gr = row0 + r;
      const int gk = k0 + kk;
      As[kk][r] = (gr < R && gk < d) ? X[gr * d + gk] : T(0);
    }
    for (int e = tid; e < TK * TN; e += 256) {
      const int kk = e / TN, cc = e % TN;
      const int gk = k0 + kk, gc = col0 + cc;
      Bs[kk][cc] = (gk < d && gc < SC) ? Bm[(int64_t)gk * SC + gc] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const T a0 = As[kk + lk][wm + li], a1 = As[kk + lk][wm + 16 + li];
      const T b0 = Bs[kk + lk][wn + li], b1 = Bs[kk + lk][wn + 16 + li];
      acc[0][0] = M::run(a0, b0, acc[0][0]);
      acc[0][1] = M::run(a0, b1, acc[0][1]);
      acc[1][0] = M::run(a1, b0, acc[1][0]);
      acc[1][1] = M::run(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = row0 + wm + i * 16 + M::row(lk, v);
        const int col = col0 + wn + j * 16 + li;
        if (r < R && col < SC) G[r * SC + col] = acc[i][j][v];
      }
}

// Row-local steps 2-3 of Lemma 1 with the row weight: for each row r and probe j,
// alpha = sum_k G[r,j,k] h_rk, then G[r,j,k] <- omega_r (G[r,j,k] - alpha) h_rk.
template <typename T>
__global__ __launch_bounds__(256) void k_gamma(T* __restrict__ G, int64_t R, int s, int c,
                                               const T* __restrict__ H,
                                               const double* __restrict__ omega,
                                               Skip skip) {
  if (skip_now(skip)) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= R * s) return;
  const int64_t r = idx / s;
  const int j = (int)(idx % s);
  T* g = G + r * (int64_t)s * c + (int64_t)j * c;
  const T* h = H + r * c;
  T alpha = T(0);
  for (int k = 0; k < c; ++k) alpha += g[k] * h[k];
  const T w = omega ? (T)omega[r] : T(1);
  for (int k = 0; k < c; ++k) g[k] = w * ((g[k] - alpha) * h[k]);
}

// part[split][a, col] (+)= sum over the split's rows r of X[r, a] G[r, col].
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_xtg(const T* __restrict__ X, int d,
                                                  const T* __restrict__ G, int SC, int64_t R,
                                                  int64_t rows_per_split, T* __restrict__ part,
                                                  int64_t part_stride, int accumulate,
                                                  Skip skip) {
  if (skip_now(skip)) return;
  __shared__ T As[TK][TM + 4];
  __shared__ T Bs[TK][TN + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int a0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
  const int64_t rb = (int64_t)blockIdx.z * rows_per_split;
  const int64_t re = rb + rows_per_split < R ? rb + rows_per_split : R;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  typedef Mfma16<T> M;
  typename M::acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = M::zero();

  for (int64_t r0 = rb; r0 < re; r0 += TK) {
    for (int e = tid; e < TK * TM; e += 256) {
      const int kk = e / TM, aa = e % TM;
      const int64_t r = r0 + kk;
      As[kk][aa] = (r < re && a0 + aa < d) ? X[r * d + a0 + aa] : T(0);
    }
    for (int e = tid; e < TK * TN; e += 256) {
      const int kk = e / TN, cc = e % TN;
      const int64_t r = r0 + kk;
      Bs[kk][cc] = (r < re && col0 + cc < SC) ? G[r * SC + col0 + cc] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const T x0 = As[kk + lk][wm + li], x1 = As[kk + lk][wm + 16 + li];
      const T g0 = Bs[kk + lk][wn + li], g1 = Bs[kk + lk][wn + 16 + li];
      acc[0][0] = M::run(x0, g0, acc[0][0]);
      acc[0][1] = M::run(x0, g1, acc[0][1]);
      acc[1][0] = M::run(x1, g0, acc[1][0]);
      acc[1][1] = M::run(x1, g1, acc[1][1]);
    }
    __syncthreads();
  }
  T* out = part + (int64_t)blockIdx.z * part_stride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = a0 + wm + i * 16 + M::row(lk, v);
        const int col = col0 + wn + j * 16 + li;
        if (a < d && col < SC) {
          const int64_t o = (int64_t)a * SC + col;
          out[o] = accumulate ? out[o] + acc[i][j][v] : acc[i][j][v];
        }
      }
}

// out[e] = sum_p part[p][e] + shift * B[e] in FP64 with a fixed summation tree: a block
// covers 32 outputs; its 8 groups of 32 threads each sum every 8th partial, then group 0
// adds the 8 group sums in order.
template <typename T>
__global__ __launch_bounds__(256) void k_reduce_parts(const T* __restrict__ part, int64_t n,
                                                      int P, double shift,
                                                      const T* __restrict__ B,
                                                      T* __restrict__ out,
                                                      Skip skip) {
  if (skip_now(skip)) return;
  __shared__ double red[8][33];
  const int el = threadIdx.x & 31, q = threadIdx.x >> 5;
  const int64_t i = (int64_t)blockIdx.x * 32 + el;
  double acc = 0.0;
  if (i < n) {
    int p = q;
    for (; p + 24 < P; p += 32) {
      const double v0 = (double)part[(int64_t)p * n + i];
      const double v1 = (double)part[(int64_t)(p + 8) * n + i];
      const double v2 = (double)part[(int64_t)(p + 16) * n + i];
      const double v3 = (double)part[(int64_t)(p + 24) * n + i];
      acc += (v0 + v1) + (v2 + v3);
    }
    for (; p < P; p += 8) acc += (double)part[(int64_t)p * n + i];
  }
  red[q][el] = acc;
  __syncthreads();
  if (q == 0 && i < n) {
    double s = 0.0;
#pragma unroll
    for (int g = 0; g < 8; ++g) s += red[g][el];
    out[i] = (T)(s + shift * (double)B[i]);
  }
}

template <typename T>
int reduce_parts_launch(const T* part, int64_t n, int P, double shift, const T* B, T* out,
                        Skip skip, hipStream_t st) {
  k_reduce_parts<T><<<(unsigned)cdiv(n, 32), 256, 0, st>>>(part, n, P, shift, B, out, skip);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}
template int reduce_parts_launch<float>(const float*, int64_t, int, double, const float*, float*,
                                        Skip, hipStream_t);

template <typename T>
static int launch_gemm_xb(const T* X, int d, const T* Bm, int SC, T* G, int64_t R,
                          Skip skip, hipStream_t st) {
  dim3 grid((unsigned)cdiv(SC, TN), (unsigned)cdiv(R, TM));
  k_gemm_xb<T><<<grid, 256, 0, st>>>(X, d, Bm, SC, G, R, skip);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

int gemm_xb_launch(Ctx* x, const void* Xrows, const void* Bm, int SC, void* G, int64_t R,
                   Skip skip, hipStream_t st) {
  if (x->prec == FIRAL_F64)
    return launch_gemm_xb<double>((const double*)Xrows, x->d, (const double*)Bm, SC,
                                  (double*)G, R, skip, st);
  return launch_gemm_xb<float>((const float*)Xrows, x->d, (const float*)Bm, SC, (float*)G, R,
                               skip, st);
}

template <typename T>
static int hvp_t(Ctx* x, const double* omega, int64_t n_rows, double shift, const T* B, T* out,
                 int s, Skip skip, hipStream_t st) {
  const int d = x->d, c = x->c;
  const int SC = s * c;
  const T* X = (const T*)x->X;
  const T* H = (const T*)x->H;
  T* G = (T*)x->G;
  T* part = (T*)x->part;
  const int64_t n_out = (int64_t)d * SC;
  const int64_t tiles = cdiv(d, TM) * cdiv(SC, TN);
  const int64_t cap = (int64_t)x->max_splits * x->s_max / s;
  int S = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(cdiv(1024, tiles), cap), 256));
  FIRAL_CHECK(prof_mark(x, st, true));
  for (int64_t r0 = 0; r0 < n_rows; r0 += x->chunk_rows) {
    const int64_t R = std::min<int64_t>(x->chunk_rows, n_rows - r0);
    FIRAL_CHECK(launch_gemm_xb<T>(X + r0 * d, d, B, SC, G, R, skip, st));
    k_gamma<T><<<(unsigned)cdiv(R * s, 256), 256, 0, st>>>(G, R, s, c, H + r0 * c,
                                                            omega ? omega + r0 : nullptr, skip);
    FIRAL_LAUNCHED();
    const int64_t rps = cdiv(R, S);
    dim3 grid((unsigned)cdiv(SC, TN), (unsigned)cdiv(d, TM), (unsigned)S);
    k_gemm_xtg<T><<<grid, 256, 0, st>>>(X + r0 * d, d, G, SC, R, rps, part, n_out, r0 > 0, skip);
    FIRAL_LAUNCHED();
  }
  FIRAL_CHECK(prof_mark(x, st, false));
  return reduce_parts_launch<T>(part, n_out, n_rows > 0 ? S : 0, shift, B, out, skip, st);
}

int hvp_launch(Ctx* x, const double* omega, int64_t n_rows, double shift, const void* B,
               void* out, int s, Skip skip, hipStream_t st, bool precise) {
  FusedPlan plan;
  if (x->prec != FIRAL_F64 && !x->force_unfused && fused_plan(x, s, n_rows, &plan, precise) &&
      plan.part_elems <= x->fused_part_elems)
    return hvp_fused_launch(x, plan, omega, n_rows, shift, (const float*)B, (float*)out, s, skip,
                            st);
  if (x->prec == FIRAL_F64)
    return hvp_t<double>(x, omega, n_rows, shift, (const double*)B, (double*)out, s, skip, st);
  return hvp_t<float>(x, omega, n_rows, shift, (const float*)B, (float*)out, s, skip, st);
}

}  // namespace firal
