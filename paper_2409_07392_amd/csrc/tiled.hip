// Row-tiled MFMA contractions of the general Hessian product (Lemma 1, aggregated over
// rows) and of the per-point gradient contraction (eq. 11), for any d and c.
//
// Product, per chunk of rows:
//   kernel 1   G = X V on a TM x TN tile (pipelined through LDS).  When a tile holds whole
//              probes (c <= TN) its epilogue takes the row-local step of the lemma,
//              alpha_rj = sum_k G[r,j,k] h_rk and G' = omega_r (G - alpha_rj) h_r, and writes
//              G'; for c > TN a probe spans several column windows, so the tile writes raw G
//              and a separate pass (one wave per row and probe) takes the row step in place.
//   kernel 2   part[split] (+)= X^T G' over the split's rows.
// A final fixed-order pass (reduce_parts_launch) sums the splits and adds shift * V.
//
// Gradient, per chunk of pool rows: u_j^T H_i w_j = a^T Gamma_i b with a = U_j^T x_i and
// b = W_j^T x_i, and Gamma_i b is the row step applied to b with unit weight; so the chunk's
// G' = Gamma-step(X W) is formed as in the product, and a second pass of kernel 1 takes the
// row-wise dot product of X U with G' tile by tile (FP64 sums, reduced in a fixed order).
//
// All sums are in a fixed order (no float atomics): results are reproducible run to run.
#include <algorithm>

#include <hip/hip_ext.h>

#include "common.h"

namespace firal {

namespace {

constexpr int kTK = 16;      // k-rows per pipeline stage
constexpr int kMaxPP = 16;   // probes per column tile when tiles hold whole probes

// Workgroup b of n runs on XCD b % 8 (round-robin dispatch); give each XCD a contiguous range
// of logical tiles so that tiles sharing operands share that XCD's L2.
__device__ __forceinline__ int64_t xcd_lid(int64_t b, int64_t n) {
  const int64_t q = n >> 3, r = n & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// Column tiling of a block of s probes with c columns each (SC = s*c flat columns).
struct ColMap {
  int c, s, SC, TN;
  int full;     // 1: each tile holds up to pp whole probes; 0: each probe is cut into nw windows
  int pp, nw, ntiles;
  __device__ __forceinline__ void tile(int t, int& col0, int& width, int& p0, int& np,
                                       int& w) const {
    if (full) {
      p0 = t * pp;
      np = s - p0 < pp ? s - p0 : pp;
      col0 = p0 * c;
      width = np * c;
      w = 0;
    } else {
      p0 = t / nw;
      w = t - p0 * nw;
      np = 1;
      col0 = p0 * c + w * TN;
      width = c - w * TN < TN ? c - w * TN : TN;
    }
  }
};

ColMap make_colmap(int c, int s, int TN) {
  ColMap m;
  m.c = c;
  m.s = s;
  m.SC = s * c;
  m.TN = TN;
  m.full = c <= TN;
  if (m.full) {
    // as few tiles as whole probes allow, the probes spread evenly over them
    m.ntiles = (int)cdiv(s, std::min(TN / c, kMaxPP));
    m.pp = (int)cdiv(s, m.ntiles);
    m.nw = 1;
  } else {
    m.pp = 1;
    m.nw = (int)cdiv(c, TN);
    m.ntiles = s * m.nw;
  }
  return m;
}

enum XvMode { kGamma = 0, kRaw = 1, kDot = 2 };

// Pipeline stage depth and LDS row strides (FP32/FP64): stages of 16 k-rows read four rows
// apart (k = 4q + g); the stride puts the four 16-lane groups of a wave on two disjoint halves
// of the banks.  bf16x3 stages are 32 deep and held as bf16 hi/lo planes, one 32-element row
// per m or n, its four 16-byte chunks swizzled by row so that the eight lanes of a 128-bit
// read hit eight different bank groups.
template <bool BF3> constexpr int stage_k() { return BF3 ? 32 : kTK; }
constexpr int kPad = 4;
__device__ __forceinline__ int swz(int row, int ch) { return ch ^ ((row >> 1) & 3); }
// element offset of (plane, row, chunk) in a [2 planes][rows][32] bf16 buffer
__device__ __forceinline__ int pl_off(int plane, int rows, int row, int ch) {
  return (plane * rows + row) * 32 + swz(row, ch) * 8;
}

template <typename T, int WM, int WN, int MODE, bool BF3>
constexpr size_t xv_lds_bytes() {
  constexpr int TK = stage_k<BF3>();
  constexpr int TM = 32 * WM, TN = 32 * WN, SA = TM + kPad, SB = TN + kPad;
  constexpr size_t main_b = BF3 ? (size_t)(TM + TN) * 2 * 2 * 32 * 2
                                : (size_t)(2 * TK * SA + 2 * TK * SB) * sizeof(T);
  constexpr size_t epi_b = (size_t)(TM * (TN + 1) + (MODE == kGamma ? TM * kMaxPP : 0)) * sizeof(T);
  return main_b > epi_b ? main_b : epi_b;
}

// One pipeline stage (16 k-rows) of a wave's WM x WN blocks from LDS tiles stored k-major
// (a[k][m], b[k][n]): four 16x16x4 steps, lane (li, g) reading k = 4q + g.
template <typename T, int WM, int WN>
__device__ __forceinline__ void mma_stage(const T* __restrict__ a, int SA, const T* __restrict__ b,
                                          int SB, int wm, int wn, int li, int g,
                                          typename Mfma16<T>::acc (&acc)[WM][WN]) {
  typedef Mfma16<T> M;
#pragma unroll
  for (int q = 0; q < kTK / 4; ++q) {
    T av[WM], bv[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i) av[i] = a[(4 * q + g) * SA + wm + 16 * i + li];
#pragma unroll
    for (int j = 0; j < WN; ++j) bv[j] = b[(4 * q + g) * SB + wn + 16 * j + li];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) acc[i][j] = M::run(av[i], bv[j], acc[i][j]);
  }
}

// One 32-deep bf16x3 stage from hi/lo planes: A planes [2][TM][32], B planes [2][TN][32].
template <int TM, int TN, int WM, int WN>
__device__ __forceinline__ void mma_stage3(const __bf16* __restrict__ a, const __bf16* __restrict__ b,
                                           int wm, int wn, int li, int g,
                                           f32x4 (&acc)[WM][WN]) {
  bf16x8 ah[WM], al[WM];
#pragma unroll
  for (int i = 0; i < WM; ++i) {
    const int row = wm + 16 * i + li;
    ah[i] = *reinterpret_cast<const bf16x8*>(a + pl_off(0, TM, row, g));
    al[i] = *reinterpret_cast<const bf16x8*>(a + pl_off(1, TM, row, g));
  }
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int row = wn + 16 * j + li;
    const bf16x8 bh = *reinterpret_cast<const bf16x8*>(b + pl_off(0, TN, row, g));
    const bf16x8 bl = *reinterpret_cast<const bf16x8*>(b + pl_off(1, TN, row, g));
#pragma unroll
    for (int i = 0; i < WM; ++i) acc[i][j] = mfma3(ah[i], al[i], bh, bl, acc[i][j]);
  }
}

__device__ __forceinline__ bf16x8 bf16_zero8() {
  bf16x8 z;
#pragma unroll
  for (int u = 0; u < 8; ++u) z[u] = (__bf16)0.0f;
  return z;
}

// Kernel 1: tile (row tile, column tile) of X_chunk B on four waves in a 2 x 2 arrangement, each
// WM x WN MFMA blocks of 16 x 16, k pipelined through double-buffered LDS.  Epilogue by MODE:
//   kGamma  (tiles of whole probes) alpha = gamma . h per row and probe, then
//           Gout = omega (gamma - alpha) h;
//   kRaw    Gout = gamma;
//   kDot    part[ct][r] = sum over the tile's columns of gamma * Gin (FP64): one tile's share of
//           a row-wise dot product with a matrix of the same shape.
// The epilogue moves the tile through LDS so that every global access is a coalesced row
// segment, and issues all of a wave's loads before it uses any of them.
template <typename T, int WM, int WN, int MODE, bool BF3>
__global__ __launch_bounds__(256, 2) void k_xv(
    const T* __restrict__ X, const __bf16* __restrict__ Xh, const __bf16* __restrict__ Xl, int d,
    int64_t R, const T* __restrict__ B, const __bf16* __restrict__ Vh,
    const __bf16* __restrict__ Vl, const T* __restrict__ H, const double* __restrict__ omega,
    ColMap cm, T* __restrict__ Gout, const T* __restrict__ Gin, double* __restrict__ dpart,
    Skip skip) {
  if (skip_now(skip)) return;
  constexpr int TM = 32 * WM, TN = 32 * WN, SCs = TN + 1;
  constexpr int NU = TN / 64, RPW = TM / 4;   // columns per lane, rows per wave (epilogue)
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t lid = xcd_lid(blockIdx.x, gridDim.x);
  const int64_t rt = lid / cm.ntiles;
  const int ct = (int)(lid - rt * cm.ntiles);
  const int64_t row0 = rt * TM;
  int col0, width, p0, np, w;
  cm.tile(ct, col0, width, p0, np, w);
  const int c = cm.c, SC = cm.SC;
  const int wm = (wave >> 1) * 16 * WM, wn = (wave & 1) * 16 * WN;
  typedef Mfma16<T> M;
  typename M::acc acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = M::zero();

  if constexpr (BF3) {
    // X and B from their pre-split planes (16-byte chunks of 8 k): X's made at context
    // creation, B's (as V^T, (s c) x d) once per call
    static_assert(TM * 4 == 512 && TN * 4 == 512, "two staging tasks per thread and operand");
    __bf16* Ab = reinterpret_cast<__bf16*>(lds_raw);   // [2 bufs][2 planes][TM][32]
    __bf16* Bb = Ab + 2 * 2 * TM * 32;                 // [2 bufs][2 planes][TN][32]
    const bool xvec = (d & 7) == 0;
    bf16x8 pah[2], pal[2], pbh[2], pbl[2];
    auto load = [&](int kt) {
      const int k0 = kt * 32;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int idx = tid + 256 * i, row = idx >> 2, ch = idx & 3;
        const int64_t gr = row0 + row;
        const int k = k0 + 8 * ch;
        pah[i] = bf16_zero8();
        pal[i] = bf16_zero8();
        if (gr < R && k < d) {
          if (xvec) {
            pah[i] = *reinterpret_cast<const bf16x8*>(Xh + gr * d + k);
            pal[i] = *reinterpret_cast<const bf16x8*>(Xl + gr * d + k);
          } else {
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (k + u < d) {
                pah[i][u] = Xh[gr * d + k + u];
                pal[i][u] = Xl[gr * d + k + u];
              }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int n = tid & (TN - 1), ch = (tid / TN) + 2 * i;
        const int k = k0 + 8 * ch;
        pbh[i] = bf16_zero8();
        pbl[i] = bf16_zero8();
        if (n < width && k < d) {
          const int64_t o = (int64_t)(col0 + n) * d + k;
          if (xvec) {
            pbh[i] = *reinterpret_cast<const bf16x8*>(Vh + o);
            pbl[i] = *reinterpret_cast<const bf16x8*>(Vl + o);
          } else {
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (k + u < d) {
                pbh[i][u] = Vh[o + u];
                pbl[i][u] = Vl[o + u];
              }
          }
        }
      }
    };
    auto store = [&](int buf) {
      __bf16* a = Ab + buf * 2 * TM * 32;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int idx = tid + 256 * i, row = idx >> 2, ch = idx & 3;
        *reinterpret_cast<bf16x8*>(a + pl_off(0, TM, row, ch)) = pah[i];
        *reinterpret_cast<bf16x8*>(a + pl_off(1, TM, row, ch)) = pal[i];
      }
      __bf16* b = Bb + buf * 2 * TN * 32;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int n = tid & (TN - 1), ch = (tid / TN) + 2 * i;
        *reinterpret_cast<bf16x8*>(b + pl_off(0, TN, n, ch)) = pbh[i];
        *reinterpret_cast<bf16x8*>(b + pl_off(1, TN, n, ch)) = pbl[i];
      }
    };
    const int nk = (d + 31) / 32;
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) load(kt + 1);
      mma_stage3<TM, TN, WM, WN>(Ab + buf * 2 * TM * 32, Bb + buf * 2 * TN * 32, wm, wn, li, g,
                                 acc);
      if (kt + 1 < nk) store(buf ^ 1);
      __syncthreads();
    }
  } else {
    constexpr int SA = TM + kPad, SB = TN + kPad;
    constexpr int EA = TM * kTK / 256, EB = TN * kTK / 256;
    T* As = reinterpret_cast<T*>(lds_raw);   // [2][kTK][SA]
    T* Bs = As + 2 * kTK * SA;               // [2][kTK][SB]
    T ra[EA], rb[EB];
    auto load = [&](int kt) {
      const int k0 = kt * kTK;
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int e = tid + 256 * i, r = e / kTK, k = e % kTK;
        const int64_t gr = row0 + r;
        ra[i] = (gr < R && k0 + k < d) ? X[gr * d + k0 + k] : T(0);
      }
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int e = tid + 256 * i, k = e / TN, n = e % TN;
        rb[i] = (k0 + k < d && n < width) ? B[(int64_t)(k0 + k) * SC + col0 + n] : T(0);
      }
    };
    auto store = [&](int buf) {
      T* a = As + buf * kTK * SA;
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int e = tid + 256 * i;
        a[(e % kTK) * SA + e / kTK] = ra[i];
      }
      T* b = Bs + buf * kTK * SB;
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int e = tid + 256 * i;
        b[(e / TN) * SB + e % TN] = rb[i];
      }
    };
    const int nk = (d + kTK - 1) / kTK;
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) load(kt + 1);
      mma_stage<T, WM, WN>(As + buf * kTK * SA, SA, Bs + buf * kTK * SB, SB, wm, wn, li, g, acc);
      if (kt + 1 < nk) store(buf ^ 1);
      __syncthreads();
    }
  }

  // ---- epilogue: the tile goes to LDS (the pipeline buffers are free after the last barrier)
  T* Cs = reinterpret_cast<T*>(lds_raw);   // [TM][SCs]
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Cs[(wm + 16 * i + M::row(g, v)) * SCs + wn + 16 * j + li] = acc[i][j][v];
  __syncthreads();
  const int rows_here = (int)(R - row0 < TM ? R - row0 : TM);

  if constexpr (MODE == kRaw) {
#pragma unroll 4
    for (int it = 0; it < RPW; ++it) {
      const int m = wave + 4 * it;
      if (m < rows_here) {
        T* go = Gout + (row0 + m) * SC + col0;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int n = lane + 64 * u;
          if (n < width) __builtin_nontemporal_store(Cs[m * SCs + n], go + n);
        }
      }
    }
    return;
  } else {
    // E2: this wave's rows (m = wave + 4 it), lanes over columns; the row operand (h for
    // kGamma, Gin for kDot) and omega are loaded for every row before any is used, at addresses
    // clamped into the arrays, so that the loads overlap; values outside the tile are masked
    // where they are used.
    T gv[RPW][NU], xv[RPW][NU], omv[RPW];
#pragma unroll
    for (int it = 0; it < RPW; ++it) {
      const int m = wave + 4 * it;
      const int64_t r = row0 + (m < rows_here ? m : 0);
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int n = lane + 64 * u;
        const bool ok = m < rows_here && n < width;
        if constexpr (MODE == kGamma) {
          const int kk = n - (n / c) * c;
          xv[it][u] = H[ok ? r * c + kk : 0];
        } else {
          xv[it][u] = Gin[ok ? r * SC + col0 + n : 0];
        }
      }
    }
    if constexpr (MODE == kGamma) {
      if (omega) {
#pragma unroll
        for (int it = 0; it < RPW; ++it) {
          const int m = wave + 4 * it;
          omv[it] = (T)omega[row0 + (m < rows_here ? m : 0)];
        }
      } else {
#pragma unroll
        for (int it = 0; it < RPW; ++it) omv[it] = T(1);
      }
    }
#pragma unroll
    for (int it = 0; it < RPW; ++it) {
      const int m = wave + 4 * it;
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int n = lane + 64 * u;
        const bool ok = m < rows_here && n < width;
        gv[it][u] = Cs[m * SCs + n];
        // each element is touched by one thread
        Cs[m * SCs + n] = ok ? gv[it][u] * xv[it][u] : T(0);
      }
    }
    __syncthreads();
    // E3: segment sums from LDS, two lanes per (row, segment), FP64, fixed order
    const int L = MODE == kGamma ? c : width;       // segment length
    const int nseg = MODE == kGamma ? np : 1;
    const int hl = (L + 1) >> 1;
    T* Al = Cs + TM * SCs;                          // [TM][kMaxPP] (kGamma)
    for (int item = tid; item < TM * nseg * 2; item += 256) {
      const int half = item & 1, mp = item >> 1;
      const int m = mp / nseg, p = mp - m * nseg;
      const int beg = p * L + half * hl, end = half ? p * L + L : p * L + hl;
      double v = 0.0;
      if (m < rows_here)
        for (int k = beg; k < end; ++k) v += (double)Cs[m * SCs + k];
      v += __shfl_xor(v, 1, 64);
      if (!half && m < rows_here) {
        if constexpr (MODE == kGamma) Al[m * kMaxPP + p] = (T)v;
        else dpart[(int64_t)ct * R + row0 + m] = v;
      }
    }
    if constexpr (MODE == kGamma) {
      __syncthreads();
      // E4: G' = omega (gamma - alpha) h, coalesced row segments
#pragma unroll
      for (int it = 0; it < RPW; ++it) {
        const int m = wave + 4 * it;
        if (m < rows_here) {
          const int64_t r = row0 + m;
          const T om = omv[it];
          T* go = Gout + r * SC + col0;
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            const int n = lane + 64 * u;
            if (n < width)
              __builtin_nontemporal_store(om * ((gv[it][u] - Al[m * kMaxPP + n / c]) * xv[it][u]),
                                          go + n);
          }
        }
      }
    }
  }
}

// Row step of Lemma 1 for probes wider than a column tile: one wave per (row, probe),
// alpha = sum_k G h_k (FP64), then G <- omega (G - alpha) h in place.  VEC: c % 4 == 0 and
// c <= 1024, the row held in registers as float4 (one read of G, one write).
template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_gamma_rows(T* __restrict__ G, int64_t R, int s, int c,
                                                    const T* __restrict__ H,
                                                    const double* __restrict__ omega, Skip skip) {
  if (skip_now(skip)) return;
  const int lane = threadIdx.x & 63;
  const int64_t id = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (id >= R * s) return;   // whole waves
  const int64_t r = id / s;
  T* gr = G + id * c;        // row r, probe id - r s
  const T* hr = H + r * c;
  const T om = omega ? (T)omega[r] : T(1);
  if constexpr (VEC) {
    const int n4 = c >> 2;
    float4 gv[4], hv[4];
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k4 = lane + 64 * q;
      if (k4 < n4) {
        gv[q] = reinterpret_cast<const float4*>(gr)[k4];
        hv[q] = reinterpret_cast<const float4*>(hr)[k4];
      } else {
        gv[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        hv[q] = gv[q];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      a += (double)gv[q].x * hv[q].x + (double)gv[q].y * hv[q].y + (double)gv[q].z * hv[q].z +
           (double)gv[q].w * hv[q].w;
    a = wave_sum(a);
    const float al = (float)a;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k4 = lane + 64 * q;
      if (k4 < n4) {
        float4 o;
        o.x = om * ((gv[q].x - al) * hv[q].x);
        o.y = om * ((gv[q].y - al) * hv[q].y);
        o.z = om * ((gv[q].z - al) * hv[q].z);
        o.w = om * ((gv[q].w - al) * hv[q].w);
        reinterpret_cast<float4*>(gr)[k4] = o;
      }
    }
  } else {
    double a = 0.0;
    for (int k = lane; k < c; k += 64) a += (double)gr[k] * (double)hr[k];
    a = wave_sum(a);
    const T al = (T)a;
    for (int k = lane; k < c; k += 64) gr[k] = om * ((gr[k] - al) * hr[k]);
  }
}

// Kernel 2.  part[split][a, col] (+)= sum over the split's rows r of X[r, a] G'[r, col], with
// a d-tile of TM = 32 WM rows and a column tile of TN = 32 WN.
template <typename T, int WM, int WN, bool BF3>
__global__ __launch_bounds__(256, 2) void k_xtg(
    const T* __restrict__ X, const __bf16* __restrict__ XTh, const __bf16* __restrict__ XTl,
    int64_t ldt, int d, const T* __restrict__ G, int SC, int64_t R, int64_t rows_per_split,
    int nmt, int nct, T* __restrict__ part, int64_t part_stride, int accumulate, Skip skip) {
  if (skip_now(skip)) return;
  constexpr int TM = 32 * WM, TN = 32 * WN;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t lid = xcd_lid(blockIdx.x, gridDim.x);
  const int mt = (int)(lid % nmt);
  const int64_t rest = lid / nmt;
  const int ct = (int)(rest % nct);
  const int sp = (int)(rest / nct);
  const int a0 = mt * TM, col0 = ct * TN;
  const int64_t rb = (int64_t)sp * rows_per_split;
  const int64_t re = rb + rows_per_split < R ? rb + rows_per_split : R;
  const int wm = (wave >> 1) * 16 * WM, wn = (wave & 1) * 16 * WN;
  const int64_t nrows = re > rb ? re - rb : 0;

  typedef Mfma16<T> M;
  typename M::acc acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = M::zero();

  if constexpr (BF3) {
    // X^T from its pre-split transposed planes (row a, 16-byte chunks of 8 rows r; the split's
    // first row is a multiple of 8), G' split once while staged
    static_assert(TM * 4 == 512 && TN * 4 == 512, "two staging tasks per thread and operand");
    __bf16* Ab = reinterpret_cast<__bf16*>(lds_raw);   // [2 bufs][2 planes][TM][32]
    __bf16* Bb = Ab + 2 * 2 * TM * 32;                 // [2 bufs][2 planes][TN][32]
    bf16x8 pah[2], pal[2];
    float pb[2][8];
    auto load = [&](int kt) {
      const int64_t r0 = rb + (int64_t)kt * 32;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int idx = tid + 256 * i, m = idx >> 2, ch = idx & 3;
        const int64_t r = r0 + 8 * ch;
        pah[i] = bf16_zero8();
        pal[i] = bf16_zero8();
        if (a0 + m < d && r < re) {
          const bf16x8 h = *reinterpret_cast<const bf16x8*>(XTh + (int64_t)(a0 + m) * ldt + r);
          const bf16x8 l = *reinterpret_cast<const bf16x8*>(XTl + (int64_t)(a0 + m) * ldt + r);
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (r + u < re) {
              pah[i][u] = h[u];
              pal[i][u] = l[u];
            }
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int n = tid & (TN - 1), ch = (tid / TN) + 2 * i;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t r = r0 + 8 * ch + u;
          pb[i][u] = (r < re && col0 + n < SC) ? (float)G[r * SC + col0 + n] : 0.0f;
        }
      }
    };
    auto store = [&](int buf) {
      __bf16* a = Ab + buf * 2 * TM * 32;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int idx = tid + 256 * i, m = idx >> 2, ch = idx & 3;
        *reinterpret_cast<bf16x8*>(a + pl_off(0, TM, m, ch)) = pah[i];
        *reinterpret_cast<bf16x8*>(a + pl_off(1, TM, m, ch)) = pal[i];
      }
      __bf16* b = Bb + buf * 2 * TN * 32;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int n = tid & (TN - 1), ch = (tid / TN) + 2 * i;
        bf16x8 h, l;
        split8(pb[i], h, l);
        *reinterpret_cast<bf16x8*>(b + pl_off(0, TN, n, ch)) = h;
        *reinterpret_cast<bf16x8*>(b + pl_off(1, TN, n, ch)) = l;
      }
    };
    const int nk = (int)((nrows + 31) / 32);
    if (nk > 0) {
      load(0);
      store(0);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) load(kt + 1);
      mma_stage3<TM, TN, WM, WN>(Ab + buf * 2 * TM * 32, Bb + buf * 2 * TN * 32, wm, wn, li, g,
                                 acc);
      if (kt + 1 < nk) store(buf ^ 1);
      __syncthreads();
    }
  } else {
    constexpr int SA = TM + kPad, SB = TN + kPad;
    constexpr int EA = TM * kTK / 256, EB = TN * kTK / 256;
    constexpr int KA = 256 / TM, KB = 256 / TN;   // k-rows covered by one pass of the threads
    T* As = reinterpret_cast<T*>(lds_raw);   // [2][kTK][SA]
    T* Bs = As + 2 * kTK * SA;               // [2][kTK][SB]
    const int bn = tid % TN, bk = tid / TN;
    const bool bvalid = col0 + bn < SC;
    const int am = tid % TM, ak = tid / TM;
    const bool avalid = a0 + am < d;
    T ra[EA], rb_[EB];
    auto load = [&](int kt) {
      const int64_t r0 = rb + (int64_t)kt * kTK;
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int64_t r = r0 + ak + KA * i;
        ra[i] = (r < re && avalid) ? X[r * d + a0 + am] : T(0);
      }
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int64_t r = r0 + bk + KB * i;
        rb_[i] = (r < re && bvalid) ? G[r * SC + col0 + bn] : T(0);
      }
    };
    auto store = [&](int buf) {
#pragma unroll
      for (int i = 0; i < EA; ++i) As[(buf * kTK + ak + KA * i) * SA + am] = ra[i];
#pragma unroll
      for (int i = 0; i < EB; ++i) Bs[(buf * kTK + bk + KB * i) * SB + bn] = rb_[i];
    };
    const int nk = (int)((nrows + kTK - 1) / kTK);
    if (nk > 0) {
      load(0);
      store(0);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) load(kt + 1);
      mma_stage<T, WM, WN>(As + buf * kTK * SA, SA, Bs + buf * kTK * SB, SB, wm, wn, li, g, acc);
      if (kt + 1 < nk) store(buf ^ 1);
      __syncthreads();
    }
  }

  T* out = part + (int64_t)sp * part_stride;
  if (accumulate) {
    // every earlier partial is loaded first (clamped addresses) so that the loads overlap
    T prev[WM][WN][4];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = a0 + wm + 16 * i + M::row(g, v);
          const int col = col0 + wn + 16 * j + li;
          prev[i][j][v] = out[a < d && col < SC ? (int64_t)a * SC + col : 0];
        }
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = a0 + wm + 16 * i + M::row(g, v);
          const int col = col0 + wn + 16 * j + li;
          if (a < d && col < SC) out[(int64_t)a * SC + col] = prev[i][j][v] + acc[i][j][v];
        }
  } else {
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = a0 + wm + 16 * i + M::row(g, v);
          const int col = col0 + wn + 16 * j + li;
          if (a < d && col < SC) out[(int64_t)a * SC + col] = acc[i][j][v];
        }
  }
}

// g_r = -(1/s) sum over column tiles (in order) of the tile's row dot product.
__global__ __launch_bounds__(256) void k_grad_sum(const double* __restrict__ dpart, int64_t R,
                                                  int ntiles, int s, double* __restrict__ g) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double q = 0.0;
  for (int t = 0; t < ntiles; ++t) q += dpart[(int64_t)t * R + r];
  g[r] = -q / s;
}

// Tile shapes: 128 x 128 (64 x 64 per wave) for FP32 and bf16x3, 64 x 128 for FP64.
template <typename T> struct Shape;
template <> struct Shape<float> {
  static constexpr int WM1 = 4, WN1 = 4, WM2 = 4, WN2 = 4;
};
template <> struct Shape<double> {
  static constexpr int WM1 = 2, WN1 = 4, WM2 = 2, WN2 = 4;
};

template <typename T, int WM, int WN, bool BF3>
constexpr size_t xtg_lds_bytes() {
  return BF3 ? (size_t)(32 * WM + 32 * WN) * 2 * 2 * 32 * 2
             : (size_t)(2 * kTK * (32 * WM + kPad) + 2 * kTK * (32 * WN + kPad)) * sizeof(T);
}

template <typename Kern>
int set_lds(Kern k, size_t bytes, DeviceOnce& once) {
  if (once.done()) return FIRAL_OK;
  if (bytes > 48 * 1024) {
    FIRAL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  }
  once.set();
  return FIRAL_OK;
}

template <typename T>
ColMap colmap_for(int c, int s) {
  return make_colmap(c, s, 32 * Shape<T>::WN1);
}

// The chunk's rows of X in the form each kernel reads them.
template <typename T>
struct XRows {
  const T* x;          // row-major, leading dimension d
  const __bf16* xh;    // bf16x3: hi / lo planes, row-major
  const __bf16* xl;
  const __bf16* xth;   // bf16x3: hi / lo planes of X^T (leading dimension ldt), at the chunk
  const __bf16* xtl;
  int64_t ldt;
};

template <typename T>
XRows<T> chunk_rows_of(const Ctx* x, int64_t r0) {
  XRows<T> c;
  c.x = (const T*)x->X + r0 * x->d;
  c.xh = x->Xhi ? (const __bf16*)x->Xhi + r0 * x->d : nullptr;
  c.xl = x->Xlo ? (const __bf16*)x->Xlo + r0 * x->d : nullptr;
  c.xth = x->XThi ? (const __bf16*)x->XThi + r0 : nullptr;
  c.xtl = x->XTlo ? (const __bf16*)x->XTlo + r0 : nullptr;
  c.ldt = x->ldt;
  return c;
}

// G = Gamma-step(omega, X_chunk B) for the chunk's R rows: the whole-probe epilogue when tiles
// hold whole probes, else the raw product followed by the per-(row, probe) pass.
// prof: attach the profiling event pair of the product's first contraction (product calls
// only; the gradient's use of this step is not timed).
template <typename T, bool BF3>
int xv_gamma(Ctx* x, bool prof, const ColMap& cm, const XRows<T>& xr, int d, int64_t R,
             const T* B, const __bf16* Vh, const __bf16* Vl, const T* Hc, const double* om, T* G,
             Skip skip, hipStream_t st) {
  typedef Shape<T> S_;
  constexpr int TM1 = 32 * S_::WM1;
  const unsigned nwg = (unsigned)(cdiv(R, TM1) * cm.ntiles);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (prof) FIRAL_CHECK(prof_pair(x, FIRAL_PROF_PRODUCT, &e0, &e1));
  if (cm.full) {
    auto k = k_xv<T, S_::WM1, S_::WN1, kGamma, BF3>;
    constexpr size_t lds = xv_lds_bytes<T, S_::WM1, S_::WN1, kGamma, BF3>();
    static DeviceOnce attr;
    FIRAL_CHECK(set_lds(k, lds, attr));
    hipExtLaunchKernelGGL(k, dim3(nwg), dim3(256), lds, st, e0, e1, 0u, xr.x, xr.xh, xr.xl, d, R,
                          B, Vh, Vl, Hc, om, cm, G, (const T*)nullptr, (double*)nullptr, skip);
    FIRAL_LAUNCHED();
  } else {
    auto k = k_xv<T, S_::WM1, S_::WN1, kRaw, BF3>;
    constexpr size_t lds = xv_lds_bytes<T, S_::WM1, S_::WN1, kRaw, BF3>();
    static DeviceOnce attr;
    FIRAL_CHECK(set_lds(k, lds, attr));
    hipExtLaunchKernelGGL(k, dim3(nwg), dim3(256), lds, st, e0, e1, 0u, xr.x, xr.xh, xr.xl, d, R,
                          B, Vh, Vl, Hc, om, cm, G, (const T*)nullptr, (double*)nullptr, skip);
    FIRAL_LAUNCHED();
    const unsigned nb = (unsigned)cdiv(R * cm.s, 4);
    if (sizeof(T) == 4 && cm.c % 4 == 0 && cm.c <= 1024)
      k_gamma_rows<T, true><<<nb, 256, 0, st>>>(G, R, cm.s, cm.c, Hc, om, skip);
    else
      k_gamma_rows<T, false><<<nb, 256, 0, st>>>(G, R, cm.s, cm.c, Hc, om, skip);
    FIRAL_LAUNCHED();
  }
  return FIRAL_OK;
}

}  // namespace

// Buffer sizing of the row-tiled kernels: column tiles of a block of s probes, and output
// tiles of the X^T G' contraction.
int64_t tiled_col_tiles(int prec, int c, int s) {
  return prec == FIRAL_F64 ? colmap_for<double>(c, s).ntiles : colmap_for<float>(c, s).ntiles;
}
int64_t tiled_out_tiles(int prec, int d, int64_t sc) {
  const int TM = 32 * (prec == FIRAL_F64 ? Shape<double>::WM2 : Shape<float>::WM2);
  const int TN = 32 * (prec == FIRAL_F64 ? Shape<double>::WN2 : Shape<float>::WN2);
  return cdiv(d, TM) * cdiv(sc, TN);
}

template <typename T, bool BF3>
static int hvp_tiled_t(Ctx* x, const double* omega, int64_t n_rows, double shift, const T* B,
                       T* out, int s, Skip skip, hipStream_t st) {
  typedef Shape<T> S_;
  constexpr int TM2 = 32 * S_::WM2, TN2 = 32 * S_::WN2;
  const int d = x->d, c = x->c, SC = s * c;
  const ColMap cm = colmap_for<T>(c, s);
  const T* H = (const T*)x->H;
  T* G = (T*)x->G;
  T* part = (T*)x->part;
  const int64_t n_out = (int64_t)d * SC;
  const int nmt = (int)cdiv(d, TM2), nct = (int)cdiv(SC, TN2);
  const int64_t tiles = (int64_t)nmt * nct;
  const int64_t cap = (int64_t)x->max_splits * x->s_max / s;
  // enough row splits for several full rounds of two workgroups per CU
  const int S = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(cdiv(4096, tiles), cap), 256));
  auto k2 = k_xtg<T, S_::WM2, S_::WN2, BF3>;
  constexpr size_t lds2 = xtg_lds_bytes<T, S_::WM2, S_::WN2, BF3>();
  static DeviceOnce attr2;
  FIRAL_CHECK(set_lds(k2, lds2, attr2));
  // bf16x3: the hi/lo planes of V^T, made once for every chunk
  __bf16* Vh = nullptr;
  __bf16* Vl = nullptr;
  if constexpr (BF3) {
    Vh = (__bf16*)x->VTf;
    Vl = Vh + (int64_t)SC * d;
    if (n_rows > 0) FIRAL_CHECK(nt3_split_vt((const float*)B, d, SC, Vh, Vl, st));
  }

  for (int64_t r0 = 0; r0 < n_rows; r0 += x->chunk_rows) {
    const int64_t R = std::min<int64_t>(x->chunk_rows, n_rows - r0);
    const XRows<T> xr = chunk_rows_of<T>(x, r0);
    FIRAL_CHECK((xv_gamma<T, BF3>(x, true, cm, xr, d, R, B, Vh, Vl, H + r0 * c,
                                  omega ? omega + r0 : nullptr, G, skip, st)));
    // splits start on a multiple of 32 rows (the bf16x3 kernel reads X^T in 8-row chunks)
    const int64_t rps = cdiv(cdiv(R, S), 32) * 32;
    hipEvent_t e0, e1;
    FIRAL_CHECK(prof_pair(x, FIRAL_PROF_PRODUCT_T, &e0, &e1));
    hipExtLaunchKernelGGL(k2, dim3((unsigned)(tiles * S)), dim3(256), lds2, st, e0, e1, 0u, xr.x,
                          xr.xth, xr.xtl, xr.ldt, d, (const T*)G, SC, R, rps, nmt, nct, part,
                          n_out, (int)(r0 > 0), skip);
    FIRAL_LAUNCHED();
  }
  return reduce_parts_launch<T>(part, n_out, n_rows > 0 ? S : 0, shift, B, out, skip, st);
}

int hvp_tiled_launch(Ctx* x, const double* omega, int64_t n_rows, double shift, const void* B,
                     void* out, int s, Skip skip, hipStream_t st, bool precise) {
  if (x->prec == FIRAL_F64)
    return hvp_tiled_t<double, false>(x, omega, n_rows, shift, (const double*)B, (double*)out, s,
                                      skip, st);
  if (x->prec == FIRAL_BF16X3 && !precise)
    return hvp_tiled_t<float, true>(x, omega, n_rows, shift, (const float*)B, (float*)out, s,
                                    skip, st);
  return hvp_tiled_t<float, false>(x, omega, n_rows, shift, (const float*)B, (float*)out, s, skip,
                                   st);
}

// Gradient of eq. 11 per chunk of pool rows: u^T H_i w = (U^T x_i) . Gamma_i (W^T x_i), i.e.
// G' = Gamma-step(1, X W) followed by the row-wise dot product of X U with G'.
template <typename T, bool BF3>
static int grad_tiled_t(Ctx* x, const T* U, const T* W, int s, double* g, hipStream_t st) {
  typedef Shape<T> S_;
  constexpr int TM1 = 32 * S_::WM1;
  const int d = x->d, c = x->c;
  const ColMap cm = colmap_for<T>(c, s);
  auto kd = k_xv<T, S_::WM1, S_::WN1, kDot, BF3>;
  constexpr size_t lds = xv_lds_bytes<T, S_::WM1, S_::WN1, kDot, BF3>();
  static DeviceOnce attr;
  FIRAL_CHECK(set_lds(kd, lds, attr));
  T* G = (T*)x->G;
  // bf16x3: hi/lo planes of W^T and U^T, made once for every chunk
  __bf16 *Wh = nullptr, *Wl = nullptr, *Uh = nullptr, *Ul = nullptr;
  if constexpr (BF3) {
    const int64_t SC = (int64_t)s * c;
    Wh = (__bf16*)x->VTf;
    Wl = Wh + SC * d;
    Uh = Wl + SC * d;
    Ul = Uh + SC * d;
    if (x->n_pool > 0) {
      FIRAL_CHECK(nt3_split_vt((const float*)W, d, (int)SC, Wh, Wl, st));
      FIRAL_CHECK(nt3_split_vt((const float*)U, d, (int)SC, Uh, Ul, st));
    }
  }
  for (int64_t r0 = 0; r0 < x->n_pool; r0 += x->chunk_rows) {
    const int64_t R = std::min<int64_t>(x->chunk_rows, x->n_pool - r0);
    const XRows<T> xr = chunk_rows_of<T>(x, r0);
    const T* Hc = (const T*)x->H + r0 * c;
    FIRAL_CHECK((xv_gamma<T, BF3>(x, false, cm, xr, d, R, W, Wh, Wl, Hc, nullptr, G, skip_none(),
                                  st)));
    kd<<<(unsigned)(cdiv(R, TM1) * cm.ntiles), 256, lds, st>>>(
        xr.x, xr.xh, xr.xl, d, R, U, Uh, Ul, Hc, nullptr, cm, nullptr, G, x->gpart, skip_none());
    FIRAL_LAUNCHED();
    k_grad_sum<<<(unsigned)cdiv(R, 256), 256, 0, st>>>(x->gpart, R, cm.ntiles, s, g + r0);
    FIRAL_LAUNCHED();
  }
  return FIRAL_OK;
}

int grad_launch(Ctx* x, const void* U, const void* W, int s, double* g, hipStream_t st) {
  if (x->prec == FIRAL_F32 && !x->force_tiled) {
    int n_tiles = 0;
    FIRAL_CHECK(grad_fused_launch(x, (const float*)U, (const float*)W, s, st, &n_tiles));
    if (n_tiles > 0) {
      k_grad_sum<<<(unsigned)cdiv(x->n_pool, 256), 256, 0, st>>>(x->gpart, x->n_pool, n_tiles, s,
                                                                 g);
      FIRAL_LAUNCHED();
      return FIRAL_OK;
    }
  }
  if (x->prec == FIRAL_F64)
    return grad_tiled_t<double, false>(x, (const double*)U, (const double*)W, s, g, st);
  if (x->prec == FIRAL_BF16X3)
    return grad_tiled_t<float, true>(x, (const float*)U, (const float*)W, s, g, st);
  return grad_tiled_t<float, false>(x, (const float*)U, (const float*)W, s, g, st);
}

// ------------------------------------------------ bf16x3 planes of X (context creation)
// Xh = bf16(x), Xl = bf16(x - Xh) row-major, and the same planes of X^T with leading dimension
// ldt (a multiple of 8, padding zero); 32 x 32 tiles transposed through LDS.
__global__ __launch_bounds__(256) void k_split_x(const float* __restrict__ X, int64_t N, int d,
                                                 int64_t ldt, __bf16* __restrict__ Xh,
                                                 __bf16* __restrict__ Xl, __bf16* __restrict__ XTh,
                                                 __bf16* __restrict__ XTl) {
  __shared__ __bf16 th[32][33], tl[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int a0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 8 rows of 32 per pass
  for (int q = ty; q < 32; q += 8) {
    const int64_t r = r0 + q;
    const int a = a0 + tx;
    __bf16 h = (__bf16)0.0f, l = (__bf16)0.0f;
    if (r < N && a < d) {
      const float v = X[r * d + a];
      h = (__bf16)v;
      l = (__bf16)(v - (float)h);
      Xh[r * d + a] = h;
      Xl[r * d + a] = l;
    }
    th[q][tx] = h;
    tl[q][tx] = l;
  }
  __syncthreads();
  for (int q = ty; q < 32; q += 8) {
    const int a = a0 + q;
    const int64_t r = r0 + tx;
    if (a < d && r < ldt) {
      XTh[(int64_t)a * ldt + r] = th[tx][q];
      XTl[(int64_t)a * ldt + r] = tl[tx][q];
    }
  }
}

int split_x_launch(Ctx* x, hipStream_t st) {
  dim3 grid((unsigned)cdiv(x->ldt, 32), (unsigned)cdiv(x->d, 32));
  k_split_x<<<grid, 256, 0, st>>>((const float*)x->X, x->N, x->d, x->ldt, (__bf16*)x->Xhi,
                                  (__bf16*)x->Xlo, (__bf16*)x->XThi, (__bf16*)x->XTlo);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

}  // namespace firal
