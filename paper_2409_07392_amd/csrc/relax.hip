// Rademacher probes, the entropic mirror-descent update, the sampled objective
// and one full iteration of the fast Relax solve (Algorithm 2).  The eq. 11
// per-point gradient contraction is in tiled.hip.
#include <algorithm>
#include <climits>
#include <cmath>

#include "common.h"

namespace firal {

// ------------------------------------------------------------- probes
// SplitMix64 (Steele, Lea & Flood 2014): output m of the stream seeded with `seed` is the
// finaliser applied to seed + (m + 1) * 0x9E3779B97F4A7C15.
__device__ __forceinline__ uint64_t splitmix_final(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ __launch_bounds__(256) void k_probes(T* __restrict__ V, uint64_t seed, int t_host,
                                                const int32_t* __restrict__ t_dev, int d, int s,
                                                int c) {
  const int t = t_dev ? *t_dev : t_host;   // captured steps read the iteration from the device
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t sc = (int64_t)s * c;
  if (idx >= (int64_t)d * sc) return;
  const int a = (int)(idx / sc);
  const int j = (int)((idx / c) % s);
  const int k = (int)(idx % c);
  const uint64_t ctr = ((uint64_t)(t - 1) * (uint64_t)s + (uint64_t)j) * ((uint64_t)d * c) +
                       (uint64_t)k * d + (uint64_t)a;
  const uint64_t z = splitmix_final(seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull);
  V[idx] = (z >> 63) ? T(-1) : T(1);
}

int probes_launch(Ctx* x, uint64_t seed, int t, int s, void* V, hipStream_t st,
                  const int32_t* t_dev) {
  const int64_t n = (int64_t)x->d * s * x->c;
  if (x->prec == FIRAL_F64)
    k_probes<double><<<(unsigned)cdiv(n, 256), 256, 0, st>>>((double*)V, seed, t, t_dev, x->d, s,
                                                             x->c);
  else
    k_probes<float><<<(unsigned)cdiv(n, 256), 256, 0, st>>>((float*)V, seed, t, t_dev, x->d, s,
                                                            x->c);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

// ----------------------------------------------------- mirror descent
// Four passes with per-block partials re-reduced in a fixed order by every block:
//   (1) max|g|   (2) beta = beta0/max|g|, e = log w - beta g, max e
//   (3) u = exp(e - max e), sum u   (4) w = u / sum u
// A failed step (non-SPD block or CG breakdown) leaves w unchanged.

__device__ __forceinline__ bool step_failed(const Status* st) {
  return st->breakdown != 0 || st->bad_block != INT_MAX;
}

// max / sum of nb per-block partials, every block computing the same value: each thread
// takes every 256th partial, then a fixed block tree (one memory round trip, not nb).
__device__ __forceinline__ double reduce_parts_max(const double* part, int nb) {
  double m = -INFINITY;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, part[i]);
  m = block_max<256>(m);
  __shared__ double bc;
  if (threadIdx.x == 0) bc = m;
  __syncthreads();
  return bc;
}
__device__ __forceinline__ double reduce_parts_sum(const double* part, int nb) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[i];
  v = block_sum<256>(v);
  __shared__ double bc;
  if (threadIdx.x == 0) bc = v;
  __syncthreads();
  return bc;
}

__global__ __launch_bounds__(256) void k_md1(const double* __restrict__ g, int64_t n,
                                             double* __restrict__ part) {
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(g[i]));
  m = block_max<256>(m);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void k_md2(const double* __restrict__ w,
                                             const double* __restrict__ g, int64_t n,
                                             double beta0, const double* __restrict__ part_g,
                                             double* __restrict__ e, double* __restrict__ part_e,
                                             Status* st) {
  const double gmax = reduce_parts_max(part_g, gridDim.x);
  const double beta = gmax > 0.0 ? beta0 / gmax : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->g_absmax = gmax;
    st->beta = beta;
  }
  double m = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = log(w[i]) - beta * g[i];
    e[i] = v;
    m = fmax(m, v);
  }
  m = block_max<256>(m);
  if (threadIdx.x == 0) part_e[blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void k_md3(double* __restrict__ e, int64_t n,
                                             const double* __restrict__ part_e,
                                             double* __restrict__ part_s) {
  const double m = reduce_parts_max(part_e, gridDim.x);
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double u = exp(e[i] - m);
    e[i] = u;
    acc += u;
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) part_s[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_md4(double* __restrict__ w, const double* __restrict__ u,
                                             int64_t n, const double* __restrict__ part_s,
                                             const Status* st) {
  if (step_failed(st)) return;
  const double S = reduce_parts_sum(part_s, gridDim.x);
  const double inv = 1.0 / S;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    w[i] = u[i] * inv;
}

// omega = [b w ; 1]
__global__ __launch_bounds__(256) void k_omega(const double* __restrict__ w, double b,
                                               int64_t n_pool, int64_t N,
                                               double* __restrict__ omega) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) omega[i] = i < n_pool ? b * w[i] : 1.0;
}

__global__ __launch_bounds__(256) void k_fhat(const double* part, int s, int P, Status* st) {
  double f = 0.0;
  for (int i = threadIdx.x; i < s * P; i += blockDim.x) f += part[i];
  f = block_sum<256>(f);
  if (threadIdx.x == 0) st->f_hat = f / s;
}

__global__ void k_step_reset(Status* st, double* keep) {
  *keep = 0.0;   // running max of the two solves' residuals
  st->converged = 1;
  st->breakdown = 0;
  st->bad_block = INT_MAX;
  st->cg_iters[0] = 0;
  st->cg_iters[1] = 0;
  st->relres_max = 0.0;
  st->f_hat = 0.0;
  st->g_absmax = 0.0;
  st->beta = 0.0;
}

__global__ void k_advance(int32_t* t) { *t += 1; }

// w_i = v (the first iterate 1/n of Algorithm 2) or w_i *= v (z = b w after the last one)
__global__ __launch_bounds__(256) void k_fill_scale(double* __restrict__ w, int64_t n, double v,
                                                    int scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = scale ? w[i] * v : v;
}

int fill_scale_launch(double* w, int64_t n, double v, bool scale, hipStream_t st) {
  if (n <= 0) return FIRAL_OK;
  k_fill_scale<<<(unsigned)cdiv(n, 256), 256, 0, st>>>(w, n, v, scale ? 1 : 0);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

__global__ void k_relres_merge(Status* st, double* keep) {
  // keeps the max recurrence residual over both solves
  *keep = fmax(*keep, st->relres_max);
  st->relres_max = *keep;
}

int objective_launch(Ctx* x, const double* z, double lambda, const void* V, int s, double tol,
                     int max_iter, uint32_t flags, double* g, hipStream_t st) {
  const int64_t n = x->n_pool, N = x->N;
  double* keep = x->redpart + 3 * x->red_blocks;
  k_step_reset<<<1, 1, 0, st>>>(x->status, keep);
  FIRAL_LAUNCHED();
  k_omega<<<(unsigned)cdiv(N, 256), 256, 0, st>>>(z, 1.0, n, N, x->omega);
  FIRAL_LAUNCHED();
  FIRAL_CHECK(precond_launch(x, x->omega, lambda, st));
  FIRAL_CHECK(pcg_launch(x, x->omega, lambda, x->Pinv, V, x->W1, s, tol, max_iter, flags, 0, st));
  k_relres_merge<<<1, 1, 0, st>>>(x->status, keep);
  FIRAL_LAUNCHED();
  FIRAL_CHECK(hvp_launch(x, nullptr, n, 0.0, V, x->Y, s, skip_none(), st));
  FIRAL_CHECK(coldot_launch(x, x->W1, x->Y, s, x->colpart, skip_none(), st));
  k_fhat<<<1, 256, 0, st>>>(x->colpart, s, x->col_parts, x->status);
  FIRAL_LAUNCHED();
  if (g) {
    FIRAL_CHECK(pcg_launch(x, x->omega, lambda, x->Pinv, x->Y, x->W2, s, tol, max_iter, flags, 1,
                           st));
    k_relres_merge<<<1, 1, 0, st>>>(x->status, keep);
    FIRAL_LAUNCHED();
    FIRAL_CHECK(grad_launch(x, x->W1, x->W2, s, g, st));
  }
  return FIRAL_OK;
}

int relax_step_launch(Ctx* x, double* w, double b, double lambda, double beta0, uint64_t seed,
                      int t, int s, double tol, int max_iter, uint32_t flags, double* g_out,
                      hipStream_t st) {
  const int64_t n = x->n_pool, N = x->N;
  double* keep = x->redpart + 3 * x->red_blocks;   // one spare slot
  k_step_reset<<<1, 1, 0, st>>>(x->status, keep);
  FIRAL_LAUNCHED();
  k_omega<<<(unsigned)cdiv(N, 256), 256, 0, st>>>(w, b, n, N, x->omega);
  FIRAL_LAUNCHED();
  FIRAL_CHECK(probes_launch(x, seed, t, s, x->V, st, x->async ? x->t_dev : nullptr));
  FIRAL_CHECK(precond_launch(x, x->omega, lambda, st));
  FIRAL_CHECK(pcg_launch(x, x->omega, lambda, x->Pinv, x->V, x->W1, s, tol, max_iter, flags, 0, st));
  k_relres_merge<<<1, 1, 0, st>>>(x->status, keep);
  FIRAL_LAUNCHED();
  FIRAL_CHECK(hvp_launch(x, nullptr, n, 0.0, x->W1, x->Y, s, skip_none(), st));
  FIRAL_CHECK(coldot_launch(x, x->V, x->Y, s, x->colpart, skip_none(), st));
  k_fhat<<<1, 256, 0, st>>>(x->colpart, s, x->col_parts, x->status);
  FIRAL_LAUNCHED();
  FIRAL_CHECK(pcg_launch(x, x->omega, lambda, x->Pinv, x->Y, x->W2, s, tol, max_iter, flags, 1, st));
  k_relres_merge<<<1, 1, 0, st>>>(x->status, keep);
  FIRAL_LAUNCHED();
  double* g = g_out ? g_out : x->gbuf;
  FIRAL_CHECK(grad_launch(x, x->V, x->W2, s, g, st));
  const int nb = x->red_blocks;
  double* pg = x->redpart;
  double* pe = x->redpart + nb;
  double* ps = x->redpart + 2 * nb;
  k_md1<<<nb, 256, 0, st>>>(g, n, pg);
  FIRAL_LAUNCHED();
  k_md2<<<nb, 256, 0, st>>>(w, g, n, beta0, pg, x->ebuf, pe, x->status);
  FIRAL_LAUNCHED();
  k_md3<<<nb, 256, 0, st>>>(x->ebuf, n, pe, ps);
  FIRAL_LAUNCHED();
  k_md4<<<nb, 256, 0, st>>>(w, x->ebuf, n, ps, x->status);
  FIRAL_LAUNCHED();
  if (x->async) {
    k_advance<<<1, 1, 0, st>>>(x->t_dev);
    FIRAL_LAUNCHED();
  }
  return FIRAL_OK;
}

}  // namespace firal
