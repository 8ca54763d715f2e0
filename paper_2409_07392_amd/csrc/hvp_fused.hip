// Fused FP32 Hessian product (Lemma 1): one kernel computes, for a tile of
// whole probes and a range of rows, X^T [omega * Gamma(X V)] into a per-range
// partial; a second pass sums the ranges in a fixed order and adds shift*V.
//
// Per workgroup (8 waves) and per chunk of 32 rows:
//   1. the chunk of X is staged in LDS twice (row-major for the first
//      contraction, transposed for the second) with h and omega;
//   2. G = X_chunk V_tile on MFMA 16x16x4; each wave owns up to NCB 16-column
//      blocks of the tile and keeps its slice of V in registers for the whole
//      kernel (V is reused by every chunk);
//   3. G goes to LDS column-major; one thread per (row, probe) forms
//      alpha = G.h and G' = omega (G - alpha) h (steps 2-3 of the lemma);
//   4. Out_tile += X_chunk^T G' on MFMA, accumulated in registers across all
//      chunks of the range.
// The contraction index of every MFMA is permuted within groups of 16 so that
// each lane's four operands are contiguous in LDS (one 128-bit read).
// The same staging serves the bf16x3 form of the product and the fused FP32
// gradient of eq. 11 (k_grad_fused: X U and X W per chunk, then the per-row
// contraction, with no second product).
#include <algorithm>

#include <hip/hip_ext.h>

#include "common.h"

namespace firal {

namespace {

constexpr int kNW = 8;        // waves per workgroup
constexpr int kRC = 32;       // rows per chunk
constexpr int kThreads = kNW * 64;
constexpr int kHP = 2;        // h values per thread fetched ahead (all of h when c <= 32)

struct FusedGeom {
  int XS, XT, GT;             // LDS strides (floats) of Xs[r][a], XsT[a][r], GsT[col][r]
  int DP, CP;                 // padded d and padded tile width
  size_t lds_floats;
};

inline FusedGeom fused_geom(int D16, int C16, int c) {
  FusedGeom g;
  g.DP = 16 * D16;
  g.CP = 16 * C16;
  g.XS = g.DP + 4;
  g.XT = kRC + 4;
  g.GT = kRC + 4;
  g.lds_floats = (size_t)kRC * g.XS + (size_t)g.DP * g.XT + (size_t)g.CP * g.GT +
                 (size_t)kRC * c + kRC;
  return g;
}

}  // namespace

typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// The context's bf16 hi/lo planes of X (row-major) and of X^T (leading dimension ldt), made
// once at creation in BF16X3 contexts; the FP32 kernel ignores them.
struct XPlanes {
  const __bf16* h;
  const __bf16* l;
  const __bf16* th;
  const __bf16* tl;
  int64_t ldt;
};

// Row step of Lemma 1 for one (row, probe) of the LDS tile: g[k * GT], k < c, holds the
// probe's c values of G for the row, h the row's probabilities, w its weight:
// alpha = g . h, then g <- w (g - alpha) h.  Up to 16 classes the row is held in registers
// (one pass over LDS, when the kernel has the registers: REG); beyond, it is streamed twice.
template <bool REG>
__device__ __forceinline__ void gamma_row(float* g, int GT, const float* h, float w, int c) {
  constexpr int kGR = 16;
  if (REG && c <= kGR) {
    float gv[kGR], hv[kGR];
    float alpha = 0.f;
#pragma unroll
    for (int k = 0; k < kGR; ++k) {
      gv[k] = k < c ? g[k * GT] : 0.f;
      hv[k] = k < c ? h[k] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kGR; ++k) alpha += gv[k] * hv[k];
#pragma unroll
    for (int k = 0; k < kGR; ++k)
      if (k < c) g[k * GT] = w * ((gv[k] - alpha) * hv[k]);
    return;
  }
  float alpha = 0.f;
  for (int k0 = 0; k0 < c; k0 += 4) {
    float gv[4], hv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      gv[u] = k0 + u < c ? g[(k0 + u) * GT] : 0.f;
      hv[u] = k0 + u < c ? h[k0 + u] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) alpha += gv[u] * hv[u];
  }
  for (int k0 = 0; k0 < c; k0 += 4) {
    float gv[4], hv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      gv[u] = k0 + u < c ? g[(k0 + u) * GT] : 0.f;
      hv[u] = k0 + u < c ? h[k0 + u] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k0 + u < c) g[(k0 + u) * GT] = w * ((gv[u] - alpha) * hv[u]);
  }
}

template <int D16, int NCB>
__global__ __launch_bounds__(kThreads) void k_hvp_fused(
    const float* __restrict__ X, const float* __restrict__ H, const double* __restrict__ omega,
    int64_t n_rows, int d, int c, int SC, const float* __restrict__ B, int probes_per_tile, int s,
    int n_ctiles, int64_t rows_per_split, int n_splits, int XS, int XT, int GT, int CP,
    float* __restrict__ part, XPlanes xp, Skip skip) {
  if (skip_now(skip)) return;
  // XCD-aware placement: workgroups are dealt round-robin to the 8 XCDs, so the
  // logical id packs the column tiles of one row range onto one XCD (shared L2).
  const int nwg = gridDim.x;
  const int lid = (blockIdx.x & 7) * (nwg >> 3) + (blockIdx.x >> 3);
  if (lid >= n_splits * n_ctiles) return;
  const int ct = lid % n_ctiles;
  const int split = lid / n_ctiles;
  const int j0 = ct * probes_per_tile;
  const int sp = min(probes_per_tile, s - j0);
  const int col0 = j0 * c;
  const int CT = sp * c;
  const int C16 = (CT + 15) >> 4;
  const int64_t rb = (int64_t)split * rows_per_split;
  const int64_t re = rb + rows_per_split < n_rows ? rb + rows_per_split : n_rows;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  constexpr int DP = 16 * D16;

  extern __shared__ float lds[];
  float* Xs = lds;                       // [kRC][XS]
  float* XsT = Xs + kRC * XS;            // [DP][XT]
  float* GsT = XsT + DP * XT;            // [CP][GT]
  float* Hs = GsT + CP * GT;             // [kRC][c]
  float* Om = Hs + kRC * c;              // [kRC]

  // V slice in registers: k index 16g + 4lk + t for "step" 4g + t.
  float breg[NCB][4 * D16];
#pragma unroll
  for (int i = 0; i < NCB; ++i) {
    const int cb = wave + kNW * i;
    const int col = cb * 16 + li;
    const bool ok = cb < C16 && col < CT;
#pragma unroll
    for (int g = 0; g < D16; ++g)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = 16 * g + 4 * lk + t;
        breg[i][4 * g + t] = (ok && k < d) ? B[(int64_t)k * SC + col0 + col] : 0.f;
      }
  }
  f32x4 acc2[NCB][D16];
#pragma unroll
  for (int i = 0; i < NCB; ++i)
#pragma unroll
    for (int ab = 0; ab < D16; ++ab) acc2[i][ab] = f32x4{0.f, 0.f, 0.f, 0.f};

  // 1. the next chunk's X, h and omega are fetched into registers while the current chunk's
  //    products run, then staged in LDS (zero padding outside the chunk and beyond d)
  // with two column blocks per wave the registers are taken by V and the accumulators: the
  // chunk is then read just before it is staged
  constexpr bool kAhead = NCB == 1;
  constexpr int NX = kAhead ? kRC * DP / kThreads : 1;
  const int nh = (kRC * c + kThreads - 1) / kThreads;   // c <= 256: at most 16
  float xr[NX], hr[kHP], omr = 0.f;
  auto fetch_h = [&](int64_t r0) {
    const int R = (int)(re - r0 < kRC ? re - r0 : kRC);
#pragma unroll
    for (int q = 0; q < kHP; ++q) {
      const int e = tid + kThreads * q;
      if (q < nh) hr[q] = (e < kRC * c && e / c < R) ? H[r0 * c + e] : 0.f;
    }
    omr = tid < R ? (omega ? (float)omega[r0 + tid] : 1.f) : 0.f;
  };
  auto fetch = [&](int64_t r0) {
    const int R = (int)(re - r0 < kRC ? re - r0 : kRC);
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int e = tid + kThreads * q, r = e / DP, a = e - r * DP;
      xr[q] = (r < R && a < d) ? X[(r0 + r) * d + a] : 0.f;
    }
    fetch_h(r0);
  };
  if (kAhead && rb < re) fetch(rb);
  for (int64_t r0 = rb; r0 < re; r0 += kRC) {
    if (kAhead) {
#pragma unroll
      for (int q = 0; q < NX; ++q) {
        const int e = tid + kThreads * q, r = e / DP, a = e - r * DP;
        Xs[r * XS + a] = xr[q];
        XsT[a * XT + r] = xr[q];
      }
    } else {
      fetch_h(r0);
      const int R = (int)(re - r0 < kRC ? re - r0 : kRC);
      for (int e = tid; e < kRC * DP; e += kThreads) {
        const int r = e / DP, a = e - r * DP;
        const float v = (r < R && a < d) ? X[(r0 + r) * d + a] : 0.f;
        Xs[r * XS + a] = v;
        XsT[a * XT + r] = v;
      }
    }
#pragma unroll
    for (int q = 0; q < kHP; ++q) {
      const int e = tid + kThreads * q;
      if (q < nh && e < kRC * c) Hs[e] = hr[q];
    }
    for (int q = kHP; q < nh; ++q) {   // beyond c = 32 the rest of h is read directly
      const int e = tid + kThreads * q;
      const int R = (int)(re - r0 < kRC ? re - r0 : kRC);
      if (e < kRC * c) Hs[e] = e / c < R ? H[r0 * c + e] : 0.f;
    }
    if (tid < kRC) Om[tid] = omr;
    __syncthreads();
    if (kAhead && r0 + kRC < re) fetch(r0 + kRC);

    // 2. G = X_chunk V_tile for this wave's column blocks
    f32x4 acc1[NCB][2];
#pragma unroll
    for (int i = 0; i < NCB; ++i) {
      acc1[i][0] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc1[i][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int g = 0; g < D16; ++g) {
      const f32x4v a0 = *(const f32x4v*)(Xs + li * XS + 16 * g + 4 * lk);
      const f32x4v a1 = *(const f32x4v*)(Xs + (16 + li) * XS + 16 * g + 4 * lk);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < NCB; ++i) {
          acc1[i][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[t], breg[i][4 * g + t], acc1[i][0], 0, 0, 0);
          acc1[i][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[t], breg[i][4 * g + t], acc1[i][1], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < NCB; ++i) {
      const int cb = wave + kNW * i;
      if (cb < C16) {
        // lane holds G[rb*16 + 4lk + v][cb*16 + li], v = 0..3: contiguous in the column-major tile
        *(f32x4v*)(GsT + (cb * 16 + li) * GT + 4 * lk) =
            f32x4v{acc1[i][0][0], acc1[i][0][1], acc1[i][0][2], acc1[i][0][3]};
        *(f32x4v*)(GsT + (cb * 16 + li) * GT + 16 + 4 * lk) =
            f32x4v{acc1[i][1][0], acc1[i][1][1], acc1[i][1][2], acc1[i][1][3]};
      }
    }
    __syncthreads();

    // 3. Gamma apply per (row, probe), rows fastest across threads; loads issued in groups
    for (int e = tid; e < kRC * sp; e += kThreads) {
      gamma_row<NCB == 1>(GsT + (e / kRC) * c * GT + e % kRC, GT, Hs + (e % kRC) * c, Om[e % kRC],
                          c);
    }
    __syncthreads();

    // 4. Out += X_chunk^T G'
#pragma unroll
    for (int g2 = 0; g2 < kRC / 16; ++g2) {
      f32x4v bq[NCB];
#pragma unroll
      for (int i = 0; i < NCB; ++i) {
        const int cb = wave + kNW * i;
        bq[i] = cb < C16 ? *(const f32x4v*)(GsT + (cb * 16 + li) * GT + 16 * g2 + 4 * lk)
                         : f32x4v{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int ab = 0; ab < D16; ++ab) {
        const f32x4v aq = *(const f32x4v*)(XsT + (ab * 16 + li) * XT + 16 * g2 + 4 * lk);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < NCB; ++i)
            acc2[i][ab] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[t], bq[i][t], acc2[i][ab], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  float* out = part + (int64_t)split * d * SC;
#pragma unroll
  for (int i = 0; i < NCB; ++i) {
    const int cb = wave + kNW * i;
    const int col = cb * 16 + li;
    if (cb < C16 && col < CT) {
#pragma unroll
      for (int ab = 0; ab < D16; ++ab)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = ab * 16 + 4 * lk + v;
          if (a < d) out[(int64_t)a * SC + col0 + col] = acc2[i][ab][v];
        }
    }
  }
}

// ------------------------------------------------------ fused FP32 gradient (eq. 11)
// One pass over the pool rows for d <= 128: per workgroup a row range and a tile of whole
// probes; per 32-row chunk (staged as in k_hvp_fused, fetched one chunk ahead) B = X W and
// A = X U on MFMA (the W and U slices of one 16-column block per wave in registers), then per
// (row, probe) alpha = b . h and t = a . ((b - alpha) h) = u_j^T H_i w_j in FP64, and per
// row the sum over the tile's probes in probe order into gpart[tile][row] (k_grad_sum adds
// the tiles in order and scales by -1/s).
template <int D16>
__global__ __launch_bounds__(kThreads) void k_grad_fused(
    const float* __restrict__ X, const float* __restrict__ H, int64_t n_rows, int d, int c,
    int SC, const float* __restrict__ U, const float* __restrict__ W, int probes_per_tile, int s,
    int n_ctiles, int64_t rows_per_split, int n_splits, int XS, int GT, int CP,
    double* __restrict__ gpart) {
  const int nwg = gridDim.x;
  const int lid = (blockIdx.x & 7) * (nwg >> 3) + (blockIdx.x >> 3);
  if (lid >= n_splits * n_ctiles) return;
  const int ct = lid % n_ctiles;
  const int split = lid / n_ctiles;
  const int j0 = ct * probes_per_tile;
  const int sp = min(probes_per_tile, s - j0);
  const int col0 = j0 * c;
  const int CT = sp * c;
  const int C16 = (CT + 15) >> 4;
  const int64_t rb = (int64_t)split * rows_per_split;
  const int64_t re = rb + rows_per_split < n_rows ? rb + rows_per_split : n_rows;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  constexpr int DP = 16 * D16;

  extern __shared__ float lds[];
  float* Xs = lds;                          // [kRC][XS]
  float* Bs = Xs + kRC * XS;                // [CP][GT] X W of the chunk, column-major
  float* As = Bs + CP * GT;                 // [CP][GT] X U
  float* Hs = As + CP * GT;                 // [kRC][c]
  double* Ts = (double*)(Hs + ((kRC * c + 1) & ~1));   // [kRC][probes_per_tile]

  // W and U slices of this wave's column block: k index 16g + 4lk + t for step 4g + t
  float bw[4 * D16], bu[4 * D16];
  {
    const int col = wave * 16 + li;
    const bool ok = wave < C16 && col < CT;
#pragma unroll
    for (int g = 0; g < D16; ++g)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = 16 * g + 4 * lk + t;
        const int64_t o = (int64_t)k * SC + col0 + col;
        bw[4 * g + t] = (ok && k < d) ? W[o] : 0.f;
        bu[4 * g + t] = (ok && k < d) ? U[o] : 0.f;
      }
  }
  constexpr int NX = kRC * DP / kThreads;
  const int nh = (kRC * c + kThreads - 1) / kThreads;
  float xr[NX], hr[kHP];
  auto fetch = [&](int64_t r0) {
    const int R = (int)(re - r0 < kRC ? re - r0 : kRC);
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int e = tid + kThreads * q, r = e / DP, a = e - r * DP;
      xr[q] = (r < R && a < d) ? X[(r0 + r) * d + a] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < kHP; ++q) {
      const int e = tid + kThreads * q;
      if (q < nh) hr[q] = (e < kRC * c && e / c < R) ? H[r0 * c + e] : 0.f;
    }
  };
  if (rb < re) fetch(rb);
  for (int64_t r0 = rb; r0 < re; r0 += kRC) {
    const int R = (int)(re - r0 < kRC ? re - r0 : kRC);
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const int e = tid + kThreads * q, r = e / DP, a = e - r * DP;
      Xs[r * XS + a] = xr[q];
    }
#pragma unroll
    for (int q = 0; q < kHP; ++q) {
      const int e = tid + kThreads * q;
      if (q < nh && e < kRC * c) Hs[e] = hr[q];
    }
    for (int q = kHP; q < nh; ++q) {   // beyond c = 32 the rest of h is read directly
      const int e = tid + kThreads * q;
      if (e < kRC * c) Hs[e] = e / c < R ? H[r0 * c + e] : 0.f;
    }
    __syncthreads();
    if (r0 + kRC < re) fetch(r0 + kRC);

    // B = X_chunk W_tile and A = X_chunk U_tile for this wave's column block
    f32x4 ab0 = {0.f, 0.f, 0.f, 0.f}, ab1 = ab0, aa0 = ab0, aa1 = ab0;
#pragma unroll
    for (int g = 0; g < D16; ++g) {
      const f32x4v a0 = *(const f32x4v*)(Xs + li * XS + 16 * g + 4 * lk);
      const f32x4v a1 = *(const f32x4v*)(Xs + (16 + li) * XS + 16 * g + 4 * lk);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        ab0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[t], bw[4 * g + t], ab0, 0, 0, 0);
        ab1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[t], bw[4 * g + t], ab1, 0, 0, 0);
        aa0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[t], bu[4 * g + t], aa0, 0, 0, 0);
        aa1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[t], bu[4 * g + t], aa1, 0, 0, 0);
      }
    }
    if (wave < C16) {
      // lane holds rows 4lk + v (and 16 + 4lk + v) of column wave * 16 + li
      float* bc = Bs + (wave * 16 + li) * GT + 4 * lk;
      float* ac = As + (wave * 16 + li) * GT + 4 * lk;
      *(f32x4v*)bc = f32x4v{ab0[0], ab0[1], ab0[2], ab0[3]};
      *(f32x4v*)(bc + 16) = f32x4v{ab1[0], ab1[1], ab1[2], ab1[3]};
      *(f32x4v*)ac = f32x4v{aa0[0], aa0[1], aa0[2], aa0[3]};
      *(f32x4v*)(ac + 16) = f32x4v{aa1[0], aa1[1], aa1[2], aa1[3]};
    }
    __syncthreads();

    // per (row, probe): u_j^T H_i w_j = a . ((b - alpha) h), alpha = b . h (FP64)
    for (int e = tid; e < kRC * sp; e += kThreads) {
      const int r = e % kRC, j = e / kRC;
      const float* bcol = Bs + j * c * GT + r;
      const float* acol = As + j * c * GT + r;
      const float* hrow = Hs + r * c;
      double al = 0.0;
      for (int k = 0; k < c; ++k) al += (double)bcol[k * GT] * (double)hrow[k];
      double t = 0.0;
      for (int k = 0; k < c; ++k)
        t += (double)acol[k * GT] * (((double)bcol[k * GT] - al) * (double)hrow[k]);
      Ts[r * probes_per_tile + j] = t;
    }
    __syncthreads();
    if (tid < R) {
      double q = 0.0;
      for (int j = 0; j < sp; ++j) q += Ts[tid * probes_per_tile + j];
      gpart[(int64_t)ct * n_rows + r0 + tid] = q;
    }
  }
}

typedef void (*GradFusedKernel)(const float*, const float*, int64_t, int, int, int, const float*,
                                const float*, int, int, int, int64_t, int, int, int, int, double*);

template <int D16>
static GradFusedKernel grad_fused_kernel() {
  return k_grad_fused<D16>;
}

int grad_fused_launch(Ctx* x, const float* U, const float* W, int s, hipStream_t st,
                      int* n_tiles) {
  *n_tiles = 0;
  const int d = x->d, c = x->c;
  const int64_t n = x->n_pool;
  const int D16 = (d + 15) / 16;
  if (x->prec != FIRAL_F32 || D16 > 8 || c > 128 || n <= 0) return FIRAL_OK;
  // tiles of whole probes, at most one 16-column block per wave
  int pp = std::min(s, kNW * 16 / c);
  const int n_ct = (s + pp - 1) / pp;
  pp = (s + n_ct - 1) / n_ct;
  const int C16 = (pp * c + 15) / 16;
  // the per-row tile partials must fit the gradient's partial buffer
  const int64_t cap = std::min<int64_t>(x->chunk_rows, n) * tiled_col_tiles(x->prec, c, x->s_max);
  if (n * n_ct > cap) return FIRAL_OK;
  const int XS = 16 * D16 + 4, GT = kRC + 4, CP = 16 * C16;
  const size_t lds = 4 * ((size_t)kRC * XS + 2 * (size_t)CP * GT + ((kRC * c + 1) & ~1)) +
                     8 * (size_t)kRC * pp;
  if (lds > 64 * 1024) return FIRAL_OK;
  const int64_t chunks = (n + kRC - 1) / kRC;
  int64_t splits = std::max<int64_t>(1, std::min<int64_t>(chunks, 256 / n_ct));
  const int64_t rps = ((n + splits - 1) / splits + kRC - 1) / kRC * kRC;
  splits = (n + rps - 1) / rps;
  GradFusedKernel k = nullptr;
  switch (D16) {
    case 1: k = grad_fused_kernel<1>(); break;
    case 2: k = grad_fused_kernel<2>(); break;
    case 3: k = grad_fused_kernel<3>(); break;
    case 4: k = grad_fused_kernel<4>(); break;
    case 5: k = grad_fused_kernel<5>(); break;
    case 6: k = grad_fused_kernel<6>(); break;
    case 7: k = grad_fused_kernel<7>(); break;
    default: k = grad_fused_kernel<8>(); break;
  }
  const int nwg = (int)((splits * n_ct + 7) / 8 * 8);
  k<<<nwg, kThreads, lds, st>>>((const float*)x->X, (const float*)x->H, n, d, c, s * c, U, W, pp,
                                s, n_ct, rps, (int)splits, XS, GT, CP, x->gpart);
  FIRAL_LAUNCHED();
  *n_tiles = n_ct;
  return FIRAL_OK;
}

// ------------------------------------------------------------- bf16x3 variant
// Same tiling with each FP32 product taken as three bf16 products on the
// 16x16x32 bf16 MFMA (FP32 accumulation): x y ~ xh yh + xh yl + xl yh with
// xh = bf16(x), xl = bf16(x - xh).  X is split once per chunk while it is
// staged (hi and lo planes, both layouts), V once per kernel into registers,
// and G' per use.  The contraction index is again permuted so a lane's eight
// operands are adjacent: k = 32 g + 8 lk + u.

template <int D16, int NCB>
__global__ __launch_bounds__(kThreads) void k_hvp_fused_bf3(
    const float* __restrict__ X, const float* __restrict__ H, const double* __restrict__ omega,
    int64_t n_rows, int d, int c, int SC, const float* __restrict__ B, int probes_per_tile, int s,
    int n_ctiles, int64_t rows_per_split, int n_splits, int XS, int XT, int GT, int CP,
    float* __restrict__ part, XPlanes xp, Skip skip) {
  if (skip_now(skip)) return;
  const int nwg = gridDim.x;
  const int lid = (blockIdx.x & 7) * (nwg >> 3) + (blockIdx.x >> 3);
  if (lid >= n_splits * n_ctiles) return;
  const int ct = lid % n_ctiles;
  const int split = lid / n_ctiles;
  const int j0 = ct * probes_per_tile;
  const int sp = min(probes_per_tile, s - j0);
  const int col0 = j0 * c;
  const int CT = sp * c;
  const int C16 = (CT + 15) >> 4;
  const int64_t rb = (int64_t)split * rows_per_split;
  const int64_t re = rb + rows_per_split < n_rows ? rb + rows_per_split : n_rows;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  constexpr int D32 = (D16 + 1) / 2;
  constexpr int DP = 32 * D32;          // contraction padding of the first product

  extern __shared__ float lds[];
  __bf16* Xh = (__bf16*)lds;             // [kRC][XS]  hi plane, row-major
  __bf16* Xl = Xh + kRC * XS;            // [kRC][XS]  lo plane
  __bf16* XTh = Xl + kRC * XS;           // [DP][XT]   hi plane, transposed
  __bf16* XTl = XTh + DP * XT;           // [DP][XT]
  float* GsT = (float*)(XTl + DP * XT);  // [CP][GT]
  float* Hs = GsT + CP * GT;             // [kRC][c]
  float* Om = Hs + kRC * c;              // [kRC]

  bf16x8 bh[NCB][D32], bl[NCB][D32];
#pragma unroll
  for (int i = 0; i < NCB; ++i) {
    const int cb = wave + kNW * i;
    const int col = cb * 16 + li;
    const bool ok = cb < C16 && col < CT;
#pragma unroll
    for (int g = 0; g < D32; ++g) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = 32 * g + 8 * lk + u;
        v[u] = (ok && k < d) ? B[(int64_t)k * SC + col0 + col] : 0.f;
      }
      split8(v, bh[i][g], bl[i][g]);
    }
  }
  f32x4 acc2[NCB][D16];
#pragma unroll
  for (int i = 0; i < NCB; ++i)
#pragma unroll
    for (int ab = 0; ab < D16; ++ab) acc2[i][ab] = f32x4{0.f, 0.f, 0.f, 0.f};

  // the next chunk is fetched into registers while the current one's products run
  // with two column blocks per wave the registers are taken by V and the accumulators: the
  // chunk is then read just before it is staged
  constexpr bool kAhead = NCB == 1;
  const int nh = (kRC * c + kThreads - 1) / kThreads;   // c <= 256: at most 16
  float hr[kHP], omr = 0.f;
  auto fetch_h = [&](int64_t r0) {
    const int R = (int)(re - r0 < kRC ? re - r0 : kRC);
#pragma unroll
    for (int q = 0; q < kHP; ++q) {
      const int e = tid + kThreads * q;
      if (q < nh) hr[q] = (e < kRC * c && e / c < R) ? H[r0 * c + e] : 0.f;
    }
    omr = tid < R ? (omega ? (float)omega[r0 + tid] : 1.f) : 0.f;
  };
  // X comes from the context's pre-split planes: row-major in 8-byte groups of 4, transposed
  // in 16-byte groups of 8 rows (chunks start on multiples of 32 rows, ldt a multiple of 8)
  constexpr int RG = DP / 4;                                    // 4-element groups per row
  constexpr int NRM = (2 * kRC * RG + kThreads - 1) / kThreads; // row-major groups, both planes
  constexpr int NTR = (2 * DP * 4 + kThreads - 1) / kThreads;   // transposed groups, both planes
  const bool dvec = (d & 3) == 0;
  bf16x4 prm[NRM];
  bf16x8 ptr[NTR];
  auto fetch = [&](int64_t r0) {
    const int R = (int)(re - r0 < kRC ? re - r0 : kRC);
#pragma unroll
    for (int q = 0; q < NRM; ++q) {
      const int e = tid + kThreads * q;
      bf16x4 v;
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = (__bf16)0.0f;
      if (e < 2 * kRC * RG) {
        const int plane = e / (kRC * RG), rem = e - plane * (kRC * RG);
        const int r = rem / RG, a = 4 * (rem - r * RG);
        const __bf16* src = plane ? xp.l : xp.h;
        if (r < R && a < d) {
          const int64_t o = (r0 + r) * d + a;
          if (dvec) {
            v = *reinterpret_cast<const bf16x4*>(src + o);
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (a + u < d) v[u] = src[o + u];
          }
        }
      }
      prm[q] = v;
    }
#pragma unroll
    for (int q = 0; q < NTR; ++q) {
      const int e = tid + kThreads * q;
      bf16x8 v;
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = (__bf16)0.0f;
      if (e < 2 * DP * 4) {
        const int plane = e / (DP * 4), rem = e - plane * (DP * 4);
        const int a = rem >> 2, rg = 8 * (rem & 3);
        if (a < d && rg < R) {
          v = *reinterpret_cast<const bf16x8*>((plane ? xp.tl : xp.th) + a * xp.ldt + r0 + rg);
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (rg + u >= R) v[u] = (__bf16)0.0f;
        }
      }
      ptr[q] = v;
    }
    fetch_h(r0);
  };
  if (kAhead && rb < re) fetch(rb);
  for (int64_t r0 = rb; r0 < re; r0 += kRC) {
    if (!kAhead) fetch(r0);
#pragma unroll
    for (int q = 0; q < NRM; ++q) {
      const int e = tid + kThreads * q;
      if (e < 2 * kRC * RG) {
        const int plane = e / (kRC * RG), rem = e - plane * (kRC * RG);
        const int r = rem / RG, a = 4 * (rem - r * RG);
        *reinterpret_cast<bf16x4*>((plane ? Xl : Xh) + r * XS + a) = prm[q];
      }
    }
#pragma unroll
    for (int q = 0; q < NTR; ++q) {
      const int e = tid + kThreads * q;
      if (e < 2 * DP * 4) {
        const int plane = e / (DP * 4), rem = e - plane * (DP * 4);
        const int a = rem >> 2, rg = 8 * (rem & 3);
        *reinterpret_cast<bf16x8*>((plane ? XTl : XTh) + a * XT + rg) = ptr[q];
      }
    }
#pragma unroll
    for (int q = 0; q < kHP; ++q) {
      const int e = tid + kThreads * q;
      if (q < nh && e < kRC * c) Hs[e] = hr[q];
    }
    for (int q = kHP; q < nh; ++q) {   // beyond c = 32 the rest of h is read directly
      const int e = tid + kThreads * q;
      const int R = (int)(re - r0 < kRC ? re - r0 : kRC);
      if (e < kRC * c) Hs[e] = e / c < R ? H[r0 * c + e] : 0.f;
    }
    if (tid < kRC) Om[tid] = omr;
    __syncthreads();
    if (kAhead && r0 + kRC < re) fetch(r0 + kRC);

    // G = X_chunk V_tile
    f32x4 acc1[NCB][2];
#pragma unroll
    for (int i = 0; i < NCB; ++i) {
      acc1[i][0] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc1[i][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int g = 0; g < D32; ++g) {
      const bf16x8 a0h = *(const bf16x8*)(Xh + li * XS + 32 * g + 8 * lk);
      const bf16x8 a0l = *(const bf16x8*)(Xl + li * XS + 32 * g + 8 * lk);
      const bf16x8 a1h = *(const bf16x8*)(Xh + (16 + li) * XS + 32 * g + 8 * lk);
      const bf16x8 a1l = *(const bf16x8*)(Xl + (16 + li) * XS + 32 * g + 8 * lk);
#pragma unroll
      for (int i = 0; i < NCB; ++i) {
        acc1[i][0] = mfma3(a0h, a0l, bh[i][g], bl[i][g], acc1[i][0]);
        acc1[i][1] = mfma3(a1h, a1l, bh[i][g], bl[i][g], acc1[i][1]);
      }
    }
#pragma unroll
    for (int i = 0; i < NCB; ++i) {
      const int cb = wave + kNW * i;
      if (cb < C16) {
        *(f32x4v*)(GsT + (cb * 16 + li) * GT + 4 * lk) =
            f32x4v{acc1[i][0][0], acc1[i][0][1], acc1[i][0][2], acc1[i][0][3]};
        *(f32x4v*)(GsT + (cb * 16 + li) * GT + 16 + 4 * lk) =
            f32x4v{acc1[i][1][0], acc1[i][1][1], acc1[i][1][2], acc1[i][1][3]};
      }
    }
    __syncthreads();

    // Gamma apply (FP32)
    for (int e = tid; e < kRC * sp; e += kThreads) {
      gamma_row<NCB == 1>(GsT + (e / kRC) * c * GT + e % kRC, GT, Hs + (e % kRC) * c, Om[e % kRC],
                          c);
    }
    __syncthreads();

    // Out += X_chunk^T G' (one group of 32 rows)
    bf16x8 gh[NCB], gl[NCB];
#pragma unroll
    for (int i = 0; i < NCB; ++i) {
      const int cb = wave + kNW * i;
      float v[8];
      if (cb < C16) {
        const f32x4v q0 = *(const f32x4v*)(GsT + (cb * 16 + li) * GT + 8 * lk);
        const f32x4v q1 = *(const f32x4v*)(GsT + (cb * 16 + li) * GT + 8 * lk + 4);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          v[u] = q0[u];
          v[4 + u] = q1[u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = 0.f;
      }
      split8(v, gh[i], gl[i]);
    }
#pragma unroll
    for (int ab = 0; ab < D16; ++ab) {
      const bf16x8 ah = *(const bf16x8*)(XTh + (ab * 16 + li) * XT + 8 * lk);
      const bf16x8 al = *(const bf16x8*)(XTl + (ab * 16 + li) * XT + 8 * lk);
#pragma unroll
      for (int i = 0; i < NCB; ++i) acc2[i][ab] = mfma3(ah, al, gh[i], gl[i], acc2[i][ab]);
    }
    __syncthreads();
  }

  float* out = part + (int64_t)split * d * SC;
#pragma unroll
  for (int i = 0; i < NCB; ++i) {
    const int cb = wave + kNW * i;
    const int col = cb * 16 + li;
    if (cb < C16 && col < CT) {
#pragma unroll
      for (int ab = 0; ab < D16; ++ab)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = ab * 16 + 4 * lk + v;
          if (a < d) out[(int64_t)a * SC + col0 + col] = acc2[i][ab][v];
        }
    }
  }
}

// ---------------------------------------------------------------- dispatch

typedef void (*FusedKernel)(const float*, const float*, const double*, int64_t, int, int, int,
                            const float*, int, int, int, int64_t, int, int, int, int, int, float*,
                            XPlanes, Skip);

template <int D16>
static FusedKernel pick_ncb(int ncb) {
  if (ncb == 1) return k_hvp_fused<D16, 1>;
  if (ncb == 2) return k_hvp_fused<D16, 2>;
  return nullptr;
}

template <int D16>
static FusedKernel pick_bf3_ncb(int ncb) {
  if (ncb == 1) return k_hvp_fused_bf3<D16, 1>;
  if (ncb == 2) return k_hvp_fused_bf3<D16, 2>;
  return nullptr;
}

static FusedKernel pick_bf3(int D16, int ncb) {
  switch (D16) {
    case 1: return pick_bf3_ncb<1>(ncb);
    case 2: return pick_bf3_ncb<2>(ncb);
    case 3: return pick_bf3_ncb<3>(ncb);
    case 4: return pick_bf3_ncb<4>(ncb);
    case 5: return pick_bf3_ncb<5>(ncb);
    case 6: return pick_bf3_ncb<6>(ncb);
    case 7: return pick_bf3_ncb<7>(ncb);
    case 8: return pick_bf3_ncb<8>(ncb);
    default: return nullptr;
  }
}

static FusedKernel pick(int D16, int ncb) {
  switch (D16) {
    case 1: return pick_ncb<1>(ncb);
    case 2: return pick_ncb<2>(ncb);
    case 3: return pick_ncb<3>(ncb);
    case 4: return pick_ncb<4>(ncb);
    case 5: return pick_ncb<5>(ncb);
    case 6: return pick_ncb<6>(ncb);
    case 7: return pick_ncb<7>(ncb);
    case 8: return pick_ncb<8>(ncb);
    default: return nullptr;
  }
}

// Tile plan of the fused product for a call with s probes (FP32 contexts only).
// Returns false when the shape is outside what the fused kernel holds in registers/LDS.
bool fused_plan(const Ctx* x, int s, int64_t n_rows, FusedPlan* p, bool precise) {
  if (x->prec == FIRAL_F64 || n_rows <= 0) return false;
  const int d = x->d, c = x->c;
  const int D16 = (d + 15) / 16;
  const bool bf3 = x->prec == FIRAL_BF16X3 && !precise;
  // above d = 128 the row-tiled kernels are faster (measured at d = 256, c = 100: 2x)
  if (D16 > 8) return false;
  const int max_ncb = x->fused_max_ncb;
  // widest tile of whole probes whose 16-column blocks fit max_ncb per wave
  const int max_cols = max_ncb * kNW * 16;
  int pp = std::min(s, max_cols / c);
  if (pp < 1) return false;
  const int n_ct = (s + pp - 1) / pp;
  pp = (s + n_ct - 1) / n_ct;            // balance the tiles
  const int C16 = (pp * c + 15) / 16;
  const int ncb = (C16 + kNW - 1) / kNW;
  FusedGeom g = fused_geom(D16, C16, c);
  size_t lds_bytes = g.lds_floats * 4;
  if (bf3) {
    // hi/lo bf16 planes of the X chunk in both layouts, then the FP32 G tile, h, omega
    const int DP32 = 32 * ((D16 + 1) / 2);
    g.XS = DP32 + 8;
    g.XT = kRC + 8;
    lds_bytes = (size_t)2 * 2 * kRC * g.XS + (size_t)2 * 2 * DP32 * g.XT +
                4 * ((size_t)g.CP * g.GT + (size_t)kRC * c + kRC);
  }
  if (lds_bytes > 156 * 1024) return false;   // the kernel's own static LDS needs a little
  const int64_t chunks = (n_rows + kRC - 1) / kRC;
  const int target_wgs = x->fused_wgs > 0 ? x->fused_wgs : 256;
  int64_t splits = std::max<int64_t>(1, std::min<int64_t>(chunks, target_wgs / n_ct));
  const int64_t rps = ((n_rows + splits - 1) / splits + kRC - 1) / kRC * kRC;
  splits = (n_rows + rps - 1) / rps;
  p->part_elems = splits * (int64_t)d * s * c;
  p->kernel = bf3 ? (void*)pick_bf3(D16, ncb) : (void*)pick(D16, ncb);
  if (!p->kernel) return false;
  p->bf3 = bf3;
  p->D16 = D16;
  p->ncb = ncb;
  p->probes_per_tile = pp;
  p->n_ctiles = n_ct;
  p->rows_per_split = rps;
  p->n_splits = (int)splits;
  p->XS = g.XS;
  p->XT = g.XT;
  p->GT = g.GT;
  p->CP = g.CP;
  p->lds_bytes = lds_bytes;
  return true;
}

int hvp_fused_launch(Ctx* x, const FusedPlan& p, const double* omega, int64_t n_rows, double shift,
                     const float* B, float* out, int s, Skip skip, hipStream_t st) {
  FusedKernel k = (FusedKernel)p.kernel;
  // largest dynamic LDS size granted per device and instantiation (devices 0 .. 15 remembered;
  // on others the attribute is set on every call)
  static std::atomic<size_t> attr_set[16][2][17][3] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  std::atomic<size_t>* granted =
      dev >= 0 && dev < 16 ? &attr_set[dev][p.bf3][p.D16][p.ncb] : nullptr;
  if (p.lds_bytes > 64 * 1024 && (!granted || granted->load() < p.lds_bytes)) {
    FIRAL_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)p.lds_bytes));
    if (granted) granted->store(p.lds_bytes);
  }
  const int SC = s * x->c;
  const int nwg = (int)(((int64_t)p.n_splits * p.n_ctiles + 7) / 8 * 8);
  float* part = (float*)x->fused_part;
  hipEvent_t e0, e1;   // the kernel's own execution when profiling
  FIRAL_CHECK(prof_pair(x, FIRAL_PROF_PRODUCT, &e0, &e1));
  hipExtLaunchKernelGGL(k, dim3(nwg), dim3(kThreads), (uint32_t)p.lds_bytes, st, e0, e1, 0u,
                        (const float*)x->X, (const float*)x->H, omega, n_rows, x->d, x->c, SC, B,
                        p.probes_per_tile, s, p.n_ctiles, p.rows_per_split, p.n_splits, p.XS, p.XT,
                        p.GT, p.CP, part,
                        XPlanes{(const __bf16*)x->Xhi, (const __bf16*)x->Xlo,
                                (const __bf16*)x->XThi, (const __bf16*)x->XTlo, x->ldt},
                        skip);
  FIRAL_LAUNCHED();
  return reduce_parts_launch<float>(part, (int64_t)x->d * SC, p.n_splits, shift, B, out, skip, st);
}

}  // namespace firal
