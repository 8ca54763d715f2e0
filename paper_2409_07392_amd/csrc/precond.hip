// Block-diagonal preconditioner of Definition 1 / eq. 12:
//   P_k = shift I_d + sum_i omega_i h_ik (1 - h_ik) x_i x_i^T,   k = 0..c-1,
// followed by an FP64 Cholesky factorisation P_k = L_k L_k^T and the explicit
// inverse P_k^-1 = L_k^-T L_k^-1 used by the PCG apply.
//
// The c weighted Gram matrices are one GEMM over rows, classes against (a, b)
// pairs, with both operands formed from H, omega and X while they are staged;
// slices of rows are reduced afterwards in FP64 in a fixed order.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <type_traits>
#include <utility>
#include <vector>

#include "common.h"

namespace firal {

// Weighted Gram matrices as one GEMM: P[k][(a, b)] = sum_i u_ik w_i,(a,b) with u_ik =
// omega_i h_ik (1 - h_ik) (classes: the M dimension) and w_i,(a,b) = x_ia x_ib (pairs: the N
// dimension), k over the rows.  A pair tile is a 16 x BR block of (a, b) in or below the
// diagonal band; each row stage stages u for the class tile and the tile's 16 + BR x values
// in LDS, and the MFMA B operand is formed as x_a x_b when it is read.  Four waves in a
// WC x (4 / WC) arrangement (classes x pairs), each CMW x PNW blocks of 16 x 16: with few
// classes (c <= 16) all four waves sit along the pairs.
// Rows per stage: 32 for FP32 (half the barriers of 16-row stages: 2.13 -> 2.04 s for the 1000
// blocks of 384 x 384 over 1.28M rows), 16 for FP64 (32 would need 83 KB of LDS, leaving one
// workgroup per CU).
template <typename T> constexpr int kSyrkTK = sizeof(T) == 4 ? 32 : 16;
__constant__ double kSyrkUnitWeight = 1.0;   // the row weight when none is given

// L is the storage type of X and H (FP32 rows feed the FP64 Gram of the Round step).
template <typename T, typename L, int CMW, int PNW, int WC>
__global__ __launch_bounds__(256, 2) void k_syrk(const L* __restrict__ X, const L* __restrict__ H,
                                                 const double* __restrict__ omega, int64_t N,
                                                 int d, int c, const int32_t* __restrict__ tiles,
                                                 int ntiles, int nct, int64_t rows_per_split,
                                                 T* __restrict__ part) {
  constexpr int TK = kSyrkTK<T>;   // rows per stage
  constexpr int WP = 4 / WC;
  constexpr int TC = 16 * CMW * WC, TP = 16 * PNW * WP, BR = TP / 16;
  constexpr int SU = TC + 16;
  constexpr int EU = TC * TK / 256;
  __shared__ __align__(16) T Us[2][TK][SU];
  __shared__ T Xa[2][TK][17];
  __shared__ T Xb[2][TK][BR + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  // logical tile: class tile fastest, then pair tile, then row split
  const int64_t lid = blockIdx.x;
  const int cls_t = (int)(lid % nct);
  const int64_t rest = lid / nct;
  const int pt = (int)(rest % ntiles);
  const int sp = (int)(rest / ntiles);
  const int c0 = cls_t * TC;
  const int a0 = 16 * tiles[2 * pt], b0 = BR * tiles[2 * pt + 1];
  const int64_t rb = (int64_t)sp * rows_per_split;
  const int64_t re = rb + rows_per_split < N ? rb + rows_per_split : N;
  const int wc = (wave / WP) * 16 * CMW, wp = (wave % WP) * 16 * PNW;

  typedef Mfma16<T> M;
  typename M::acc acc[CMW][PNW];
#pragma unroll
  for (int i = 0; i < CMW; ++i)
#pragma unroll
    for (int j = 0; j < PNW; ++j) acc[i][j] = M::zero();

  // staging: u for (row k, class); the 16 x_a and BR x_b values of each row k
  const int ucls = tid % TC, uk = tid / TC;
  constexpr int KU = 256 / TC;
  const bool uvalid = c0 + ucls < c;
  constexpr int XW = 16 + BR, XE = TK * XW, NX = (XE + 255) / 256;
  int xk[NX], xj[NX];
  bool xon[NX], xvalid[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    const int e = tid + 256 * i;
    xon[i] = e < XE;
    xk[i] = e / XW;
    xj[i] = e % XW;
    const int col = xj[i] < 16 ? a0 + xj[i] : b0 + (xj[i] - 16);
    xvalid[i] = xon[i] && col < d;
    xj[i] = xvalid[i] ? col : 0;   // column of X to load (when valid)
  }
  // The loads read rows clamped into the split (rb is a row of it whenever there is a stage) and
  // classes and columns clamped into the arrays; u = w h (1 - h) is formed and the values outside
  // the tile are zeroed when the stage is stored, so no loaded value is consumed before the
  // current stage's MFMAs.
  L rh[EU], rx[NX];   // as stored (converted to T when staged)
  double rw[EU];
  const int uc = uvalid ? c0 + ucls : 0;
  const double* wsrc = omega ? omega : &kSyrkUnitWeight;
  auto load = [&](int kt) {
    const int64_t r0 = rb + (int64_t)kt * TK;
#pragma unroll
    for (int i = 0; i < EU; ++i) {
      const int64_t r = r0 + uk + KU * i;
      rh[i] = H[(r < re ? r : rb) * c + uc];
    }
#pragma unroll
    for (int i = 0; i < EU; ++i) {   // without weights every row reads the one weight 1
      const int64_t r = r0 + uk + KU * i;
      rw[i] = wsrc[omega ? (r < re ? r : rb) : 0];
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      const int64_t r = r0 + xk[i];
      rx[i] = X[(r < re ? r : rb) * d + xj[i]];
    }
  };
  auto store = [&](int buf, int kt) {
    const int64_t r0 = rb + (int64_t)kt * TK;
#pragma unroll
    for (int i = 0; i < EU; ++i) {
      const int64_t r = r0 + uk + KU * i;
      const T h = (T)rh[i];
      const T u = (T)rw[i] * h * (T(1) - h);
      Us[buf][uk + KU * i][ucls] = r < re && uvalid ? u : T(0);
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      // every thread stores (threads without an element write the unread pad column of Xa), so
      // that the compiler keeps each load in the load phase rather than sinking it here
      const int e = tid + 256 * i, j = e % XW;
      const int64_t r = r0 + xk[i];
      const T v = r < re && xvalid[i] ? (T)rx[i] : T(0);
      T* dst = !xon[i] ? &Xa[buf][0][16] : (j < 16 ? &Xa[buf][xk[i]][j] : &Xb[buf][xk[i]][j - 16]);
      *dst = v;
    }
  };

  const int64_t nrows = re > rb ? re - rb : 0;
  const int nk = (int)((nrows + TK - 1) / TK);
  if (nk > 0) {
    load(0);
    store(0, 0);
  }
  __syncthreads();
  // this lane's pairs in the B operand: (a_local, b_local) of column wp + 16 j + li
  int pa[PNW], pb[PNW];
#pragma unroll
  for (int j = 0; j < PNW; ++j) {
    const int pp = wp + 16 * j + li;
    pa[j] = pp / BR;
    pb[j] = pp % BR;
  }
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    load(kt + 1);   // past the last stage every row is out of range (stored as zero, never read)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < TK / 4; ++q) {
      const int k = 4 * q + g;
      T av[CMW], bv[PNW];
#pragma unroll
      for (int i = 0; i < CMW; ++i) av[i] = Us[buf][k][wc + 16 * i + li];
#pragma unroll
      for (int j = 0; j < PNW; ++j) bv[j] = Xa[buf][k][pa[j]] * Xb[buf][k][pb[j]];
#pragma unroll
      for (int i = 0; i < CMW; ++i)
#pragma unroll
        for (int j = 0; j < PNW; ++j) acc[i][j] = M::run(av[i], bv[j], acc[i][j]);
    }
    __builtin_amdgcn_sched_barrier(0);
    store(buf ^ 1, kt + 1);
    __syncthreads();
  }

  T* out = part + (int64_t)sp * c * d * d;
#pragma unroll
  for (int i = 0; i < CMW; ++i)
#pragma unroll
    for (int j = 0; j < PNW; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = c0 + wc + 16 * i + M::row(g, v);
        const int a = a0 + pa[j], b = b0 + pb[j];
        if (k < c && a < d && b < d && b <= a) out[((int64_t)k * d + a) * d + b] = acc[i][j][v];
      }
}

// The same Gram GEMM with the four waves along the pairs, for FP32-storage contexts with c > 64
// classes and d a multiple of 4: a pair tile of 16 a x 16 b columns against 128 classes, wave w
// taking a columns 4 w .. 4 w + 3 against all 16 b columns and all classes of the tile, so a pair
// product x_a x_b is formed once per workgroup and feeds CMW class blocks.  Stages of 32 rows;
// u = omega h (1 - h) is staged as [class][row] and the tile's x values as FP32 [column][row], so
// each lane reads its rows of a class or a column as 16-byte vectors.
//   FP32 (BF3 false): v_mfma_f32_16x16x4f32, the 16-row groups of a stage in the k order of the
//     wide products (lane group g takes rows 4 g + q of the group for instruction q, so one
//     16-byte read of u or x feeds four instructions).
//   bf16x3 (BF3 true, the opt-in of bf16x3 contexts): u split into hi/lo bf16 planes when staged;
//     each lane forms the products for its 8 rows (8 g .. 8 g + 7) in FP32 and splits them in
//     registers; three 16x16x32 bf16 MFMAs per block (hi hi + hi lo + lo hi).
constexpr int kSwTK = 32;                        // rows per stage (the bf16 MFMA's k)
constexpr int kSwXS = kSwTK + 4;                 // LDS row of a staged x column, floats
template <bool BF3> constexpr int kSwUS = BF3 ? kSwTK + 8 : kSwTK + 4;   // LDS row of u
template <int CMW, bool BF3>
__global__ __launch_bounds__(256, 2) void k_syrkw(const float* __restrict__ X,
                                                  const float* __restrict__ H,
                                                  const double* __restrict__ omega, int64_t N,
                                                  int d, int c, const int32_t* __restrict__ tiles,
                                                  int ntiles, int nct, int64_t rows_per_split,
                                                  float* __restrict__ part) {
  constexpr int TC = 16 * CMW, NQ = TC / 64, US = kSwUS<BF3>;
  static_assert(TC % 64 == 0, "u staging: 64 classes per quarter of the workgroup");
  typedef typename std::conditional<BF3, __bf16, float>::type UT;
  __shared__ __align__(16) UT Us[BF3 ? 2 : 1][2][TC][US];   // [hi, lo] or [u]
  __shared__ __align__(16) float XaT[2][16][kSwXS];
  __shared__ __align__(16) float XbT[2][16][kSwXS];
  const int tid = threadIdx.x, lane = tid & 63;
  const int li = lane & 15, g = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t lid = blockIdx.x;
  const int cls_t = (int)(lid % nct);
  const int64_t rest = lid / nct;
  const int pt = (int)(rest % ntiles);
  const int sp = (int)(rest / ntiles);
  const int c0 = cls_t * TC;
  const int a0 = 16 * tiles[2 * pt], b0 = 16 * tiles[2 * pt + 1];
  const int64_t rb = (int64_t)sp * rows_per_split;
  const int64_t re = rb + rows_per_split < N ? rb + rows_per_split : N;

  f32x4 acc[CMW][4];
#pragma unroll
  for (int i = 0; i < CMW; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // staging: u of classes (tid % 64) + 64 q for the 8 rows 8 wave .. 8 wave + 7 of the stage
  // (the row weights are the same for a whole wave); one 4-float x vector per thread: row
  // tid / 8, columns a0 + 4 (tid % 8) (tid % 8 < 4) or b0 + 4 (tid % 8 - 4)
  int ucls[NQ];
  bool uvalid[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    ucls[q] = (tid & 63) + 64 * q;
    uvalid[q] = c0 + ucls[q] < c;
  }
  const int xr = tid >> 3, xp = tid & 7;
  const int xcol = xp < 4 ? a0 + 4 * xp : b0 + 4 * (xp - 4);
  const bool xvalid = xcol < d;   // d and the column a multiple of 4: all four in or all out
  const double* wsrc = omega ? omega : &kSyrkUnitWeight;
  float rh[NQ][8];
  double rw[8];
  f32x4 rx;
  // loads read rows clamped into the split and columns clamped into the arrays; the values
  // outside the tile are zeroed when stored
  auto load = [&](int kt) {
    const int64_t r0 = rb + (int64_t)kt * kSwTK + 8 * wave;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t r = r0 + e < re ? r0 + e : rb;
#pragma unroll
      for (int q = 0; q < NQ; ++q) rh[q][e] = H[r * c + (uvalid[q] ? c0 + ucls[q] : 0)];
      rw[e] = wsrc[omega ? r : 0];
    }
    const int64_t r = rb + (int64_t)kt * kSwTK + xr;
    rx = *reinterpret_cast<const f32x4*>(X + (r < re ? r : rb) * d + (xvalid ? xcol : 0));
  };
  auto store = [&](int buf, int kt) {
    const int64_t r0 = rb + (int64_t)kt * kSwTK + 8 * wave;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      float u[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float h = rh[q][e];
        u[e] = r0 + e < re && uvalid[q] ? (float)rw[e] * h * (1.f - h) : 0.f;
      }
      if constexpr (BF3) {
        bf16x8 hi, lo;
        split8(u, hi, lo);
        *reinterpret_cast<bf16x8*>(&Us[0][buf][ucls[q]][8 * wave]) = hi;
        *reinterpret_cast<bf16x8*>(&Us[1][buf][ucls[q]][8 * wave]) = lo;
      } else {
        *reinterpret_cast<f32x4*>(&Us[0][buf][ucls[q]][8 * wave]) = f32x4{u[0], u[1], u[2], u[3]};
        *reinterpret_cast<f32x4*>(&Us[0][buf][ucls[q]][8 * wave + 4]) =
            f32x4{u[4], u[5], u[6], u[7]};
      }
    }
    const int64_t r = rb + (int64_t)kt * kSwTK + xr;
    const bool ok = r < re && xvalid;
    float* dst = xp < 4 ? &XaT[buf][4 * xp][xr] : &XbT[buf][4 * (xp - 4)][xr];
#pragma unroll
    for (int e = 0; e < 4; ++e) dst[e * kSwXS] = ok ? rx[e] : 0.f;
  };

  const int64_t nrows = re > rb ? re - rb : 0;
  const int nk = (int)((nrows + kSwTK - 1) / kSwTK);
  if (nk > 0) {
    load(0);
    store(0, 0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    load(kt + 1);   // past the last stage every row is out of range (stored as zero, never read)
    __builtin_amdgcn_sched_barrier(0);
    // this lane's pairs: (a0 + 4 wave + j, b0 + li).  The u of class block i + 1 is read while
    // block i's MFMAs run (the scheduler is kept from hoisting all of them, which would not fit
    // two waves per SIMD)
    if constexpr (BF3) {
      const f32x4 xb0 = *reinterpret_cast<const f32x4*>(&XbT[buf][li][8 * g]);
      const f32x4 xb1 = *reinterpret_cast<const f32x4*>(&XbT[buf][li][8 * g + 4]);
      bf16x8 bh[4], bl[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const f32x4 xa0 = *reinterpret_cast<const f32x4*>(&XaT[buf][4 * wave + j][8 * g]);
        const f32x4 xa1 = *reinterpret_cast<const f32x4*>(&XaT[buf][4 * wave + j][8 * g + 4]);
        const float pr[8] = {xa0[0] * xb0[0], xa0[1] * xb0[1], xa0[2] * xb0[2], xa0[3] * xb0[3],
                             xa1[0] * xb1[0], xa1[1] * xb1[1], xa1[2] * xb1[2], xa1[3] * xb1[3]};
        split8(pr, bh[j], bl[j]);
      }
      bf16x8 ah = *reinterpret_cast<const bf16x8*>(&Us[0][buf][li][8 * g]);
      bf16x8 al = *reinterpret_cast<const bf16x8*>(&Us[1][buf][li][8 * g]);
#pragma unroll
      for (int i = 0; i < CMW; ++i) {
        const int in = i + 1 < CMW ? i + 1 : i;
        const bf16x8 nh = *reinterpret_cast<const bf16x8*>(&Us[0][buf][16 * in + li][8 * g]);
        const bf16x8 nl = *reinterpret_cast<const bf16x8*>(&Us[1][buf][16 * in + li][8 * g]);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma3(ah, al, bh[j], bl[j], acc[i][j]);
        __builtin_amdgcn_sched_barrier(0);
        ah = nh;
        al = nl;
      }
    } else {
#pragma unroll
      for (int kg = 0; kg < kSwTK / 16; ++kg) {
        const int k0 = 16 * kg + 4 * g;
        const f32x4 xb = *reinterpret_cast<const f32x4*>(&XbT[buf][li][k0]);
        f32x4 bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const f32x4 xa = *reinterpret_cast<const f32x4*>(&XaT[buf][4 * wave + j][k0]);
          bv[j] = f32x4{xa[0] * xb[0], xa[1] * xb[1], xa[2] * xb[2], xa[3] * xb[3]};
        }
        f32x4 av = *reinterpret_cast<const f32x4*>(&Us[0][buf][li][k0]);
#pragma unroll
        for (int i = 0; i < CMW; ++i) {
          const int in = i + 1 < CMW ? i + 1 : i;
          const f32x4 nv = *reinterpret_cast<const f32x4*>(&Us[0][buf][16 * in + li][k0]);
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], bv[j][q], acc[i][j], 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
          av = nv;
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    store(buf ^ 1, kt + 1);
    __syncthreads();
  }

  float* out = part + (int64_t)sp * c * d * d;
  const int b = b0 + li;
#pragma unroll
  for (int i = 0; i < CMW; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = a0 + 4 * wave + j;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = c0 + 16 * i + 4 * g + v;
        if (k < c && a < d && b < d && b <= a) out[((int64_t)k * d + a) * d + b] = acc[i][j][v];
      }
    }
}

// P[k][a][b] = sum over splits (in order, FP64) of the lower-triangle entry (max, min) +
// shift [a == b]: P is exactly symmetric.
template <typename T>
__global__ __launch_bounds__(256) void k_syrk_reduce(const T* __restrict__ part, int S, int c,
                                                     int d, double shift,
                                                     double* __restrict__ P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t dd = (int64_t)d * d;
  if (idx >= (int64_t)c * dd) return;
  const int64_t k = idx / dd;
  const int rem = (int)(idx - k * dd);
  const int a = rem / d, b = rem - (rem / d) * d;
  const int64_t e = k * dd + (a >= b ? (int64_t)a * d + b : (int64_t)b * d + a);
  double acc = 0.0;
  for (int p = 0; p < S; ++p) acc += (double)part[(int64_t)p * c * dd + e];
  P[idx] = acc + (a == b ? shift : 0.0);
}

// In-place right-looking Cholesky of block k (lower triangle); upper part zeroed.
// A non-positive (or NaN) pivot records k in *bad (smallest k wins) and stops the block.
__global__ __launch_bounds__(256) void k_chol(double* __restrict__ P, int d, int32_t* bad) {
  const int k = blockIdx.x;
  double* A = P + (int64_t)k * d * d;
  const int tid = threadIdx.x;
  for (int j = 0; j < d; ++j) {
    __syncthreads();
    const double piv = A[(int64_t)j * d + j];
    if (!(piv > 0.0)) {
      if (tid == 0) atomicMin(bad, k);
      return;
    }
    const double ljj = sqrt(piv);
    const double inv = 1.0 / ljj;
    __syncthreads();
    if (tid == 0) A[(int64_t)j * d + j] = ljj;
    for (int i = j + 1 + tid; i < d; i += blockDim.x) A[(int64_t)i * d + j] *= inv;
    __syncthreads();
    const int m = d - j - 1;
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int ii = e / m, kk = e % m;
      if (kk <= ii) {
        const int i = j + 1 + ii, q = j + 1 + kk;
        A[(int64_t)i * d + q] -= A[(int64_t)i * d + j] * A[(int64_t)q * d + j];
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < d * d; e += blockDim.x) {
    const int i = e / d, q = e % d;
    if (q > i) A[e] = 0.0;
  }
}

// Pinv_k = (L_k L_k^T)^-1, one column per thread: forward solve L y = e_j, then L^T x = y.
// All lanes walk the same (i, p) sequence (entries above the unit's row are zero), so the
// factor reads are uniform across the wave and the column reads/writes are coalesced.
__global__ __launch_bounds__(256) void k_chol_inv(const double* __restrict__ L,
                                                  double* __restrict__ Pinv, int d,
                                                  const int32_t* bad) {
  if (*bad != INT_MAX) return;
  const int k = blockIdx.x;
  const double* Lk = L + (int64_t)k * d * d;
  double* Y = Pinv + (int64_t)k * d * d;
  for (int j0 = 0; j0 < d; j0 += blockDim.x) {
    const int j = j0 + threadIdx.x;
    const bool on = j < d;
    for (int i = 0; i < d; ++i) {
      double acc = (i == j) ? 1.0 : 0.0;
      for (int p = 0; p < i; ++p) acc -= Lk[(int64_t)i * d + p] * (on ? Y[(int64_t)p * d + j] : 0.0);
      if (on) Y[(int64_t)i * d + j] = acc / Lk[(int64_t)i * d + i];
    }
    for (int i = d - 1; i >= 0; --i) {
      double acc = on ? Y[(int64_t)i * d + j] : 0.0;
      for (int p = i + 1; p < d; ++p) acc -= Lk[(int64_t)p * d + i] * (on ? Y[(int64_t)p * d + j] : 0.0);
      if (on) Y[(int64_t)i * d + j] = acc / Lk[(int64_t)i * d + i];
    }
  }
}

// Cholesky factor and inverse of block k in one pass, the whole block held in registers.
// The symmetric sweep operator on pivot j maps a -> a - a_{:j} a_{j:} / a_jj off row/column j,
// a_{j:} / a_jj on them and -1/a_jj on the pivot; sweeping every pivot of an SPD matrix leaves
// -P^-1.  Before pivot j is swept its unswept column is the Schur complement, so
// L[i][j] = a_ij / sqrt(a_jj) (i >= j) is the Cholesky factor, and a_jj <= 0 means P is not SPD.
// Thread (ty, tx) of a TT x TT grid owns rows ty + TT u and columns tx + TT v (u, v < TB).
// L is written over P (P is read completely before the first pivot).
template <int TT, int TB>
__global__ __launch_bounds__(TT* TT) void k_sweep(double* __restrict__ P, double* __restrict__ Pinv,
                                                  int d, int32_t* bad, int write_l) {
  const int kb = blockIdx.x;
  double* A0 = P + (int64_t)kb * d * d;
  double* Y = Pinv + (int64_t)kb * d * d;
  const int ty = threadIdx.x / TT, tx = threadIdx.x % TT;
  __shared__ double prow[TT * TB];
  double a[TB][TB];
#pragma unroll
  for (int u = 0; u < TB; ++u)
#pragma unroll
    for (int v = 0; v < TB; ++v) {
      const int i = ty + TT * u, q = tx + TT * v;
      a[u][v] = (i < d && q < d) ? A0[(int64_t)i * d + q] : 0.0;
    }
  __syncthreads();
  for (int j = 0; j < d; ++j) {
    const int uj = j / TT;
    if (ty == j % TT) {
#pragma unroll
      for (int u = 0; u < TB; ++u)
        if (u == uj) {
#pragma unroll
          for (int v = 0; v < TB; ++v) prow[tx + TT * v] = a[u][v];
        }
    }
    __syncthreads();
    const double piv = prow[j];
    if (!(piv > 0.0)) {
      if (threadIdx.x == 0) atomicMin(bad, kb);
      return;
    }
    const double ip = 1.0 / piv;
    // the factor's column j (only when asked: each step's barrier then waits for these stores)
    if (write_l && tx == 0) {
      const double sq = sqrt(piv);
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        const int i = ty + TT * u;
        if (i >= j && i < d) A0[(int64_t)i * d + j] = i == j ? sq : prow[i] / sq;
      }
    }
    // rank-1 update of every element, then row j, column j and the pivot rewritten (their
    // owners are known: j = jt + TT vj in both the row and the column decomposition)
    double pri[TB], pc[TB];
#pragma unroll
    for (int u = 0; u < TB; ++u) pri[u] = prow[ty + TT * u] * ip;
#pragma unroll
    for (int v = 0; v < TB; ++v) pc[v] = prow[tx + TT * v];
#pragma unroll
    for (int u = 0; u < TB; ++u)
#pragma unroll
      for (int v = 0; v < TB; ++v) a[u][v] = fma(-pri[u], pc[v], a[u][v]);
    const int jt = j % TT, vj = j / TT;
#pragma unroll
    for (int u = 0; u < TB; ++u)
      if (u == vj && ty == jt) {
#pragma unroll
        for (int v = 0; v < TB; ++v) a[u][v] = pc[v] * ip;       // row j: a_jq / a_jj
      }
#pragma unroll
    for (int v = 0; v < TB; ++v)
      if (v == vj && tx == jt) {
#pragma unroll
        for (int u = 0; u < TB; ++u) a[u][v] = pri[u];           // column j: a_ij / a_jj
#pragma unroll
        for (int u = 0; u < TB; ++u)
          if (u == vj && ty == jt) a[u][v] = -ip;                // pivot
      }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < TB; ++u)
#pragma unroll
    for (int v = 0; v < TB; ++v) {
      const int i = ty + TT * u, q = tx + TT * v;
      if (i < d && q < d) {
        Y[(int64_t)i * d + q] = -a[u][v];
        if (write_l && q > i) A0[(int64_t)i * d + q] = 0.0;
      }
    }
}

// Inverse of each SPD block (d <= 128) by the sweep operator taken sixteen pivots at a time,
// for callers that do not ask for the factor.  Sweeping a pivot block K of the current
// (symmetric) M gives M_KK <- N = -M_KK^-1, M_IK <- T_I = -M_IK N (and M_KI <- T_I^T),
// M_IJ <- M_IJ - T_I M_KJ for the other rows and columns, the same matrix as sweeping K's
// pivots one at a time; after every block M = -P^-1.  Thread (ty, tx) of 16 x 16 keeps
// M[ty + 16u][tx + 16v] in registers (padding: identity); per block one wave sweeps the
// 16 x 16 pivot block in registers (four entries a lane, shuffles, no barrier), then the
// panel T goes through LDS and every thread updates its entries: four barriers per block.
constexpr int kSwLD = 17;   // row stride of the LDS panels (odd: no bank conflicts by column)

struct SweepLds {
  double* Kb;   // [16][kSwLD] the pivot block, then N
  double* PK;   // [DP][kSwLD] column panel M[i][K0 + m]
  double* Tp;   // [DP][kSwLD] T[i][m]
  int* fail;
};

// one pivot block K (a compile-time index into the register tile); false when a pivot of
// the block is not positive (the workgroup stops)
template <int K, int D16>
__device__ __forceinline__ bool sweep_block(double (&a)[D16][D16], const SweepLds& L, int tid,
                                            int32_t* bad, int kb) {
  constexpr int LD = kSwLD;
  const int ty = tid >> 4, tx = tid & 15;
  // the pivot block and the column panel to LDS
  L.Kb[ty * LD + tx] = a[K][K];
#pragma unroll
  for (int u = 0; u < D16; ++u) L.PK[(ty + 16 * u) * LD + tx] = a[u][K];
  __syncthreads();
  // 1. wave 0: N = sweep of the 16 x 16 block; lane l holds row l / 4, columns 4 (l % 4) + k
  if (tid < 64) {
    const int r = tid >> 2, cg = (tid & 3) * 4;
    double b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) b[k] = L.Kb[r * LD + cg + k];
    bool ok = true;
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      const double piv = __shfl(b[p & 3], 4 * p + (p >> 2), 64);
      ok = ok && piv > 0.0;
      const double ip = 1.0 / piv;
      const double arp = __shfl(b[p & 3], 4 * r + (p >> 2), 64);   // M[r][p]
      double apc[4];                                                 // M[p][cg + k]
#pragma unroll
      for (int k = 0; k < 4; ++k) apc[k] = __shfl(b[k], 4 * p + (tid & 3), 64);
      const double pri = arp * ip;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = cg + k;
        b[k] = r != p ? (c != p ? fma(-pri, apc[k], b[k]) : pri) : (c != p ? apc[k] * ip : -ip);
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) L.Kb[r * LD + cg + k] = b[k];
    if (!__all(ok) && tid == 0) {
      *L.fail = 1;
      atomicMin(bad, kb);
    }
  }
  __syncthreads();
  if (*L.fail) return false;   // the same for every thread
  // 2. T[i][c] = -sum_m M[i][K0 + m] N[m][c]
#pragma unroll
  for (int u = 0; u < D16; ++u) {
    const int i = ty + 16 * u;
    double t = 0.0;
#pragma unroll
    for (int m = 0; m < 16; ++m) t = fma(L.PK[i * LD + m], L.Kb[m * LD + tx], t);
    L.Tp[i * LD + tx] = -t;
  }
  __syncthreads();
  // 3. M_IJ -= T_I M_KJ (M_KJ[m][j] = M[j][K0 + m] by symmetry), one m at a time over the
  //    thread's entries (not unrolled: the operands of one m at a time stay in registers);
  //    then the panel becomes T and the pivot block N
#pragma unroll 1
  for (int m = 0; m < 16; ++m) {
    double tu[D16], pv[D16];
#pragma unroll
    for (int u = 0; u < D16; ++u) tu[u] = L.Tp[(ty + 16 * u) * LD + m];
#pragma unroll
    for (int v = 0; v < D16; ++v) pv[v] = L.PK[(tx + 16 * v) * LD + m];
#pragma unroll
    for (int u = 0; u < D16; ++u)
#pragma unroll
      for (int v = 0; v < D16; ++v)
        if (u != K && v != K) a[u][v] = fma(-tu[u], pv[v], a[u][v]);
  }
#pragma unroll
  for (int u = 0; u < D16; ++u) {
    a[u][K] = u == K ? L.Kb[ty * LD + tx] : L.Tp[(ty + 16 * u) * LD + tx];
    if (u != K) a[K][u] = L.Tp[(tx + 16 * u) * LD + ty];
  }
  __syncthreads();
  return true;
}

template <int D16, int... Ks>
__device__ __forceinline__ bool sweep_blocks(double (&a)[D16][D16], const SweepLds& L, int tid,
                                             int32_t* bad, int kb,
                                             std::integer_sequence<int, Ks...>) {
  return (sweep_block<Ks, D16>(a, L, tid, bad, kb) && ...);   // in order, stops at a failure
}

template <int D16>
__global__ __launch_bounds__(256) void k_sweep_blk(const double* __restrict__ P,
                                                   double* __restrict__ Pinv, int d,
                                                   int32_t* bad) {
  constexpr int DP = 16 * D16;
  __shared__ double Kb[16 * kSwLD];
  __shared__ double PK[DP * kSwLD];
  __shared__ double Tp[DP * kSwLD];
  __shared__ int fail;
  const int kb = blockIdx.x, tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  const double* A0 = P + (int64_t)kb * d * d;
  double a[D16][D16];
#pragma unroll
  for (int u = 0; u < D16; ++u)
#pragma unroll
    for (int v = 0; v < D16; ++v) {
      const int i = ty + 16 * u, j = tx + 16 * v;
      a[u][v] = (i < d && j < d) ? A0[(int64_t)i * d + j] : (i == j ? 1.0 : 0.0);
    }
  if (tid == 0) fail = 0;   // seen by all after the first step's barrier
  const SweepLds L{Kb, PK, Tp, &fail};
  if (!sweep_blocks<D16>(a, L, tid, bad, kb, std::make_integer_sequence<int, D16>{})) return;
  double* Y = Pinv + (int64_t)kb * d * d;
#pragma unroll
  for (int u = 0; u < D16; ++u)
#pragma unroll
    for (int v = 0; v < D16; ++v) {
      const int i = ty + 16 * u, j = tx + 16 * v;
      if (i < d && j < d) Y[(int64_t)i * d + j] = -a[u][v];
    }
}

// The sweep for blocks too large for registers (d > 256): block kb is copied to Pinv and swept
// there in global memory, NB pivots at a time.  With the block partitioned at pivots K as
// [[K, B^T], [B, D]], sweeping K leaves [[-K^-1, K^-1 B^T], [B K^-1, D - B K^-1 B^T]].  The NB
// rows of K are staged in LDS twice: as loaded (Bo = [K, B^T], whose columns outside K are B^T)
// and swept pivot by pivot (Rs, ending as [-K^-1, K^-1 B^T]); then every row outside K is updated
// from LDS, D[i][j] -= sum_m Bo[m][i] Rs[m][j] and A[i][k] = Rs[k][i] for k in K (the block stays
// symmetric), four rows by four columns per thread, and the rows of K are written from Rs.
// Before pivot p is swept, its staged row holds column p of the Schur complement, so the
// Cholesky factor's column p is that row over sqrt(pivot) (written to P when asked).  After all
// pivots the block holds -P^-1.  LDS: ((2 NB + 1) d + NB) doubles (NB = 16: 99 KB at d = 384;
// NB = 8 for larger blocks, at twice the passes over the block).
template <int NB>
__global__ __launch_bounds__(256) void k_sweep_glb(double* __restrict__ P, double* __restrict__ Pinv,
                                                   int d, int32_t* bad, int write_l) {
  extern __shared__ __align__(16) double sw_lds[];
  double* Bo = sw_lds;                  // [NB][d] rows of K as loaded
  double* Rs = sw_lds + NB * d;         // [NB][d] rows of K as swept
  double* Rm = sw_lds + 2 * NB * d;     // [d] pivot row before its sweep
  double* Cp = Rm + d;                  // [NB] pivot column before its sweep
  const int kb = blockIdx.x, tid = threadIdx.x;
  double* L = P + (int64_t)kb * d * d;
  double* A = Pinv + (int64_t)kb * d * d;
  for (int64_t e = tid; e < (int64_t)d * d; e += 256) A[e] = L[e];
  __syncthreads();
  const int nq = (d + 3) / 4;            // 4 x 4 tiles of the block
  for (int k0 = 0; k0 < d; k0 += NB) {
    const int nb = d - k0 < NB ? d - k0 : NB;
    for (int e = tid; e < nb * d; e += 256) {
      const int m = e / d, j = e - m * d;
      const double v = A[(int64_t)(k0 + m) * d + j];
      Bo[m * d + j] = v;
      Rs[m * d + j] = v;
    }
    __syncthreads();
    for (int m = 0; m < nb; ++m) {
      const int pc = k0 + m;
      const double piv = Rs[m * d + pc];
      if (!(piv > 0.0)) {
        if (tid == 0) atomicMin(bad, kb);
        return;
      }
      const double ip = 1.0 / piv;
      const double rs = write_l ? 1.0 / sqrt(piv) : 0.0;
      // the pivot row and column as they stand, so that every staged element can then be
      // updated in place by the one thread that owns it
      for (int j = tid; j < d; j += 256) {
        const double v = Rs[m * d + j];
        Rm[j] = v;
        if (write_l && j >= pc) L[(int64_t)j * d + pc] = v * rs;   // factor column pc
      }
      if (tid < nb) Cp[tid] = Rs[tid * d + pc];
      __syncthreads();
      for (int e = tid; e < nb * d; e += 256) {
        const int r = e / d, j = e - r * d;
        double v;
        if (r == m) v = j == pc ? -ip : Rm[j] * ip;
        else if (j == pc) v = Cp[r] * ip;
        else v = Rs[e] - Cp[r] * Rm[j] * ip;
        Rs[e] = v;
      }
      __syncthreads();
    }
    // rows outside K: D -= B K^-1 B^T, and the columns of K from Rs; 4 x 4 tiles
    for (int t = tid; t < nq * nq; t += 256) {
      const int i0 = 4 * (t / nq), j0 = 4 * (t % nq);
      double acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
      for (int m = 0; m < nb; ++m) {
        double bi[4], rj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          bi[u] = i0 + u < d ? Bo[m * d + i0 + u] : 0.0;
          rj[u] = j0 + u < d ? Rs[m * d + j0 + u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(bi[u], rj[v], acc[u][v]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u;
        if (i >= d) continue;
        const bool iin = i >= k0 && i < k0 + nb;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = j0 + v;
          if (j >= d) continue;
          const bool jin = j >= k0 && j < k0 + nb;
          double* a = A + (int64_t)i * d + j;
          if (iin) *a = Rs[(i - k0) * d + j];
          else if (jin) *a = Rs[(j - k0) * d + i];
          else *a -= acc[u][v];
        }
      }
    }
    __syncthreads();
  }
  for (int64_t e = tid; e < (int64_t)d * d; e += 256) {
    A[e] = -A[e];
    if (write_l) {
      const int i = (int)(e / d), j = (int)(e - (int64_t)i * d);
      if (j > i) L[e] = 0.0;
    }
  }
}

typedef void (*SweepBlkKernel)(const double*, double*, int, int32_t*);

static SweepBlkKernel pick_sweep_blk(int d) {
  if (d > 128) return nullptr;
  switch ((d + 15) / 16) {
    case 1: return k_sweep_blk<1>;
    case 2: return k_sweep_blk<2>;
    case 3: return k_sweep_blk<3>;
    case 4: return k_sweep_blk<4>;
    case 5: return k_sweep_blk<5>;
    case 6: return k_sweep_blk<6>;
    case 7: return k_sweep_blk<7>;
    default: return k_sweep_blk<8>;
  }
}

typedef void (*SweepKernel)(double*, double*, int, int32_t*, int);

static SweepKernel pick_sweep(int d, int* threads) {
  if (d <= 128) {
    *threads = 256;
    switch ((d + 15) / 16) {
      case 1: return k_sweep<16, 1>;
      case 2: return k_sweep<16, 2>;
      case 3: return k_sweep<16, 3>;
      case 4: return k_sweep<16, 4>;
      case 5: return k_sweep<16, 5>;
      case 6: return k_sweep<16, 6>;
      case 7: return k_sweep<16, 7>;
      default: return k_sweep<16, 8>;
    }
  }
  if (d <= 256) {
    *threads = 1024;
    switch ((d + 31) / 32) {
      case 5: return k_sweep<32, 5>;
      case 6: return k_sweep<32, 6>;
      case 7: return k_sweep<32, 7>;
      default: return k_sweep<32, 8>;
    }
  }
  return nullptr;
}

__global__ void k_bad_reset(Status* st) { st->bad_block = INT_MAX; }

// Tile shape by c: class blocks per wave (CMW) and waves along the classes (WC); pair tiles
// of 16 x BR with BR = PNW (4 / WC), PNW = 4 (FP32) or 2 (FP64).  The bf16x3 kernel: CMW = 8,
// WC = 1 (its four waves along the pairs), pair tiles of 16 x 16.
struct SyrkShape {
  int cmw, wc, pnw;
  int tc() const { return 16 * cmw * wc; }
  int br() const { return pnw * (4 / wc); }
};
int gram_form_for(int prec, int d, int c, const void* X) {
  if (prec == FIRAL_F64 || c <= 64 || d % 4 != 0 || ((uintptr_t)X & 15) != 0) return kGramClassic;
  const char* w = getenv("FIRAL_GRAM_WIDE");
  if (w && atoi(w) == 0) return kGramClassic;
  const char* g3 = getenv("FIRAL_BF3_GRAM");
  return prec == FIRAL_BF16X3 && g3 && atoi(g3) != 0 ? kGramWideBf3 : kGramWide;
}
SyrkShape syrk_shape(int prec, int c, int form) {
  if (form != kGramClassic) return SyrkShape{8, 1, 4};
  const int pnw = prec == FIRAL_F64 ? 2 : 4;
  if (c <= 16) return SyrkShape{1, 1, pnw};
  if (c <= 32) return SyrkShape{1, 2, pnw};
  if (c <= 64) return SyrkShape{2, 2, pnw};
  return SyrkShape{4, 2, pnw};
}

// Blocks of 256 < d <= kSweepGlbMaxD go to the global-memory sweep: 16-pivot panels up to
// d = 600, 8-pivot panels up to 1200 (its LDS, ((2 NB + 1) d + NB) doubles, fits the 160 KB of
// a CU up to there); larger ones to the column-at-a-time factor and inverse.
constexpr int kSweepGlb16MaxD = 600, kSweepGlbMaxD = 1200;
template <int NB>
constexpr int sweep_glb_lds(int d) { return ((2 * NB + 1) * d + NB) * (int)sizeof(double); }
static DeviceOnce g_sweep_glb_attr;

static int sweep_glb_launch(double* P, double* Pinv, int d, int c, int32_t* bad, bool want_l,
                            hipStream_t st) {
  if (!g_sweep_glb_attr.done()) {
    FIRAL_HIP(hipFuncSetAttribute((const void*)k_sweep_glb<16>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  sweep_glb_lds<16>(kSweepGlb16MaxD)));
    FIRAL_HIP(hipFuncSetAttribute((const void*)k_sweep_glb<8>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  sweep_glb_lds<8>(kSweepGlbMaxD)));
    g_sweep_glb_attr.set();
  }
  if (d <= kSweepGlb16MaxD)
    k_sweep_glb<16><<<c, 256, sweep_glb_lds<16>(d), st>>>(P, Pinv, d, bad, want_l ? 1 : 0);
  else
    k_sweep_glb<8><<<c, 256, sweep_glb_lds<8>(d), st>>>(P, Pinv, d, bad, want_l ? 1 : 0);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

template <typename T, int CMW, int WC>
static void launch_syrk(Ctx* x, const double* omega, int64_t rps, hipStream_t st) {
  constexpr int PNW = sizeof(T) == 4 ? 4 : 2;
  const int nct = (int)cdiv(x->c, 16 * CMW * WC);
  const int64_t nwg = (int64_t)nct * x->syrk_ntiles * x->syrk_splits;
  k_syrk<T, T, CMW, PNW, WC><<<(unsigned)nwg, 256, 0, st>>>(
      (const T*)x->X, (const T*)x->H, omega, x->N, x->d, x->c, x->syrk_tiles, x->syrk_ntiles, nct,
      rps, (T*)x->syrk_part);
}

template <typename T>
static int precond_t(Ctx* x, const double* omega, double shift, bool want_l, hipStream_t st) {
  const int d = x->d, c = x->c;
  const int S = x->syrk_splits;
  const int64_t rps = cdiv(x->N, S);
  k_bad_reset<<<1, 1, 0, st>>>(x->status);
  FIRAL_LAUNCHED();
  const SyrkShape sh = syrk_shape(x->prec, c, x->gram_form);
  if (x->gram_form != kGramClassic) {
    const int nct = (int)cdiv(c, sh.tc());
    const int64_t nwg = (int64_t)nct * x->syrk_ntiles * S;
    auto k = x->gram_form == kGramWideBf3 ? k_syrkw<8, true> : k_syrkw<8, false>;
    k<<<(unsigned)nwg, 256, 0, st>>>((const float*)x->X, (const float*)x->H, omega, x->N, d, c,
                                     x->syrk_tiles, x->syrk_ntiles, nct, rps,
                                     (float*)x->syrk_part);
  } else if (sh.wc == 1) launch_syrk<T, 1, 1>(x, omega, rps, st);
  else if (sh.cmw == 1) launch_syrk<T, 1, 2>(x, omega, rps, st);
  else if (sh.cmw == 2) launch_syrk<T, 2, 2>(x, omega, rps, st);
  else launch_syrk<T, 4, 2>(x, omega, rps, st);
  FIRAL_LAUNCHED();
  const int64_t n = (int64_t)c * d * d;
  k_syrk_reduce<T><<<(unsigned)cdiv(n, 256), 256, 0, st>>>((const T*)x->syrk_part, S, c, d,
                                                           shift, x->P);
  FIRAL_LAUNCHED();
  int threads = 0;
  SweepKernel sw = pick_sweep(d, &threads);
  SweepBlkKernel sb = want_l ? nullptr : pick_sweep_blk(d);
  if (sb) {
    sb<<<c, 256, 0, st>>>(x->P, x->Pinv, d, &x->status->bad_block);
    FIRAL_LAUNCHED();
  } else if (sw) {
    sw<<<c, threads, 0, st>>>(x->P, x->Pinv, d, &x->status->bad_block, want_l ? 1 : 0);
    FIRAL_LAUNCHED();
  } else if (d <= kSweepGlbMaxD) {
    FIRAL_CHECK(sweep_glb_launch(x->P, x->Pinv, d, c, &x->status->bad_block, want_l, st));
  } else {
    k_chol<<<c, 256, 0, st>>>(x->P, d, &x->status->bad_block);
    FIRAL_LAUNCHED();
    k_chol_inv<<<c, 256, 0, st>>>(x->P, x->Pinv, d, &x->status->bad_block);
    FIRAL_LAUNCHED();
  }
  return FIRAL_OK;
}

// Pair tiles (a-block of 16, b-block of BR) that meet the lower triangle, and the row-split
// count, for a context (host side, at creation).  Grids smaller than the device's workgroup
// slots (two per CU) are split over the rows up to about 1024 workgroups (partials within
// 256 MB); larger grids of the wide forms take the split count (up to 8, partials within 4 GiB)
// with the least time in rounds of slots, ceil(wgs S / slots) / S: at configuration 4, 2400
// workgroups on 512 slots run 4.69 rounds unsplit (five, the last one two-thirds empty) and
// 18.75 in four splits (nineteen quarter-length rounds).
void syrk_plan(int prec, int d, int c, int form, int n_cu, std::vector<int32_t>* tiles,
               int* splits) {
  const SyrkShape sh = syrk_shape(prec, c, form);
  const int BR = sh.br();
  const int nab = (int)cdiv(d, 16), nbb = (int)cdiv(d, BR);
  tiles->clear();
  for (int A = 0; A < nab; ++A)
    for (int Bb = 0; Bb < nbb && Bb * BR <= 16 * A + 15; ++Bb) {
      tiles->push_back(A);
      tiles->push_back(Bb);
    }
  const int64_t nt = (int64_t)tiles->size() / 2;
  const int64_t wgs = nt * cdiv(c, sh.tc());
  const int64_t es = prec == FIRAL_F64 ? 8 : 4;
  const int64_t blk = (int64_t)c * d * d * es;
  const int64_t slots = 2 * (int64_t)std::max(1, n_cu);
  if (form != kGramClassic && wgs >= slots) {
    const int64_t cap = std::min<int64_t>(8, std::max<int64_t>(1, ((int64_t)4 << 30) / blk));
    int S = 1;
    for (int64_t t = 2; t <= cap; ++t)   // rounds / S, compared as cross products
      if (cdiv(wgs * t, slots) * S < cdiv(wgs * S, slots) * t) S = (int)t;
    *splits = S;
    return;
  }
  const int64_t mem_cap = std::max<int64_t>(1, ((int64_t)1 << 28) / blk);
  *splits = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(cdiv(1024, wgs), 64),
                                                        mem_cap));
}

int chol_blocks_launch(double* P, double* Pinv, int d, int c, int32_t* bad, bool want_inv,
                       bool want_l, hipStream_t st) {
  int threads = 0;
  SweepKernel sw = pick_sweep(d, &threads);
  SweepBlkKernel sb = want_l ? nullptr : pick_sweep_blk(d);
  if (sb) {
    sb<<<c, 256, 0, st>>>(P, Pinv, d, bad);
    FIRAL_LAUNCHED();
  } else if (sw) {
    sw<<<c, threads, 0, st>>>(P, Pinv, d, bad, want_l ? 1 : 0);
    FIRAL_LAUNCHED();
  } else if (d <= kSweepGlbMaxD) {
    FIRAL_CHECK(sweep_glb_launch(P, Pinv, d, c, bad, want_l, st));
  } else {
    k_chol<<<c, 256, 0, st>>>(P, d, bad);
    FIRAL_LAUNCHED();
    if (want_inv) {
      k_chol_inv<<<c, 256, 0, st>>>(P, Pinv, d, bad);
      FIRAL_LAUNCHED();
    }
  }
  return FIRAL_OK;
}

template <typename L, int CMW, int WC>
static void launch_gram64(const L* X, const L* H, const double* omega, int64_t N, int d, int c,
                          const int32_t* tiles, int ntiles, int S, double* part,
                          hipStream_t st) {
  const int nct = (int)cdiv(c, 16 * CMW * WC);
  const int64_t nwg = (int64_t)nct * ntiles * S;
  k_syrk<double, L, CMW, 2, WC><<<(unsigned)nwg, 256, 0, st>>>(X, H, omega, N, d, c, tiles, ntiles,
                                                               nct, cdiv(std::max<int64_t>(N, 1), S),
                                                               part);
}

template <typename L>
static int gram64_t(const L* X, const L* H, const double* omega, int64_t N, int d, int c,
                    const int32_t* tiles, int ntiles, int S, double shift, double* part,
                    double* out, hipStream_t st) {
  const SyrkShape sh = syrk_shape(FIRAL_F64, c, kGramClassic);
  if (sh.wc == 1) launch_gram64<L, 1, 1>(X, H, omega, N, d, c, tiles, ntiles, S, part, st);
  else if (sh.cmw == 1) launch_gram64<L, 1, 2>(X, H, omega, N, d, c, tiles, ntiles, S, part, st);
  else if (sh.cmw == 2) launch_gram64<L, 2, 2>(X, H, omega, N, d, c, tiles, ntiles, S, part, st);
  else launch_gram64<L, 4, 2>(X, H, omega, N, d, c, tiles, ntiles, S, part, st);
  FIRAL_LAUNCHED();
  const int64_t n = (int64_t)c * d * d;
  k_syrk_reduce<double><<<(unsigned)cdiv(n, 256), 256, 0, st>>>(part, S, c, d, shift, out);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

int gram64_launch(int prec, const void* X, const void* H, const double* omega, int64_t N, int d,
                  int c, const int32_t* tiles, int ntiles, int S, double shift, double* part,
                  double* out, hipStream_t st) {
  if (prec == FIRAL_F64)
    return gram64_t<double>((const double*)X, (const double*)H, omega, N, d, c, tiles, ntiles, S,
                            shift, part, out, st);
  return gram64_t<float>((const float*)X, (const float*)H, omega, N, d, c, tiles, ntiles, S,
                         shift, part, out, st);
}

int precond_launch(Ctx* x, const double* omega, double shift, hipStream_t st, bool want_l) {
  if (x->prec == FIRAL_F64) return precond_t<double>(x, omega, shift, want_l, st);
  return precond_t<float>(x, omega, shift, want_l, st);
}

}  // namespace firal
