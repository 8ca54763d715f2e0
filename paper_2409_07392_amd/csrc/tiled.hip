// Row-tiled MFMA contractions of the general Hessian product (Lemma 1, aggregated over
// rows) and of the per-point gradient contraction (eq. 11), for any d and c.
//
// Product, per chunk of rows:
//   kernel 1   G = X V on a TM x TN tile (pipelined through LDS), then in its epilogue the
//              row-local step of the lemma: alpha_rj = sum_k G[r,j,k] h_rk over the probe
//              columns the tile holds.  When a tile holds whole probes (c <= TN) the epilogue
//              writes G' = omega_r (G - alpha) h directly; for c > TN a probe spans several
//              column windows, so the tile writes raw G and its window's partial alpha.
//   kernel 2   part[split] (+)= X^T G' over the split's rows, applying the row step while
//              staging G when the first kernel could not (windowed probes).
// A final fixed-order pass (reduce_parts_launch) sums the splits and adds shift * V.
//
// Gradient, per chunk of pool rows: one kernel computes A = X U and B = X W on the same tile
// and reduces, per row, probe and column window, sum a h b, sum a h and sum b h in FP64;
// a second pass forms g_r = -(1/s) sum_j [sum a h b - (sum a h)(sum b h)].
//
// All sums are in a fixed order (no float atomics): results are reproducible run to run.
#include <algorithm>

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
    m.pp = std::min(TN / c, kMaxPP);
    m.nw = 1;
    m.ntiles = (int)cdiv(s, m.pp);
  } else {
    m.pp = 1;
    m.nw = (int)cdiv(c, TN);
    m.ntiles = s * m.nw;
  }
  return m;
}

template <typename T, int WM, int WN, int NB, bool GRAD>
constexpr size_t xv_lds_bytes() {
  constexpr int TM = 32 * WM, TN = 32 * WN, SA = TM + 16, SB = TN + 16;
  constexpr size_t main_b = (size_t)(2 * kTK * SA + 2 * NB * kTK * SB) * sizeof(T);
  constexpr size_t epi_b = (size_t)(NB * TM * (TN + 1) + (GRAD ? 0 : TM * kMaxPP)) * sizeof(T);
  return main_b > epi_b ? main_b : epi_b;
}

// Kernel 1.  Tile (row tile rt, column tile ct) of A_nb = X_chunk B_nb (nb < NB); four waves in
// a 2 x 2 arrangement, each WM x WN MFMA blocks of 16 x 16.  Product mode (GRAD false, NB 1):
// writes G' (whole probes) or G and the window's partial alpha (windowed).  Gradient mode
// (NB 2): writes the three FP64 partial sums per row, probe and window to gpart.
template <typename T, int WM, int WN, int NB, bool GRAD>
__global__ __launch_bounds__(256, 2) void k_xv(
    const T* __restrict__ X, int d, int64_t R, const T* __restrict__ B0,
    const T* __restrict__ B1, const T* __restrict__ H, const double* __restrict__ omega,
    ColMap cm, int64_t nrt, T* __restrict__ Gout, T* __restrict__ abuf,
    double* __restrict__ gpart, Skip skip) {
  if (skip_now(skip)) return;
  constexpr int TM = 32 * WM, TN = 32 * WN, SA = TM + 16, SB = TN + 16, SCs = TN + 1;
  constexpr int EA = TM * kTK / 256, EB = TN * kTK / 256;
  constexpr int NU = (TN + 63) / 64;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* As = reinterpret_cast<T*>(lds_raw);   // [2][kTK][SA]
  T* Bs = As + 2 * kTK * SA;               // [2][NB][kTK][SB]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t lid = xcd_lid(blockIdx.x, gridDim.x);
  const int64_t rt = lid / cm.ntiles;
  const int ct = (int)(lid - rt * cm.ntiles);
  const int64_t row0 = rt * TM;
  int col0, width, p0, np, w;
  cm.tile(ct, col0, width, p0, np, w);
  const int c = cm.c, s = cm.s, SC = cm.SC;
  const int wm = (wave >> 1) * 16 * WM, wn = (wave & 1) * 16 * WN;
  typedef Mfma16<T> M;
  typename M::acc acc[NB][WM][WN];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) acc[nb][i][j] = M::zero();

  T ra[EA], rb[NB][EB];
  auto load = [&](int kt) {
    const int k0 = kt * kTK;
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int e = tid + 256 * i, r = e >> 4, k = e & 15;
      const int64_t gr = row0 + r;
      ra[i] = (gr < R && k0 + k < d) ? X[gr * d + k0 + k] : T(0);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const T* Bp = nb ? B1 : B0;
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int e = tid + 256 * i, k = e / TN, n = e % TN;
        rb[nb][i] = (k0 + k < d && n < width) ? Bp[(int64_t)(k0 + k) * SC + col0 + n] : T(0);
      }
    }
  };
  auto store = [&](int buf) {
    T* a = As + buf * kTK * SA;
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int e = tid + 256 * i;
      a[(e & 15) * SA + (e >> 4)] = ra[i];
    }
    T* b = Bs + buf * NB * kTK * SB;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int e = tid + 256 * i;
        b[(nb * kTK + e / TN) * SB + e % TN] = rb[nb][i];
      }
  };

  const int nk = (d + kTK - 1) / kTK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load(kt + 1);
    const T* a = As + buf * kTK * SA;
    const T* b = Bs + buf * NB * kTK * SB;
#pragma unroll
    for (int q = 0; q < kTK / 4; ++q) {
      T av[WM], bv[NB][WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) av[i] = a[(4 * q + g) * SA + wm + 16 * i + li];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int j = 0; j < WN; ++j) bv[nb][j] = b[(nb * kTK + 4 * q + g) * SB + wn + 16 * j + li];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) acc[nb][i][j] = M::run(av[i], bv[nb][j], acc[nb][i][j]);
    }
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  // ---- epilogue: the raw tile goes to LDS (the pipeline buffers are free now)
  T* Cs = reinterpret_cast<T*>(lds_raw);   // [NB][TM][SCs]
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          Cs[(nb * TM + wm + 16 * i + M::row(g, v)) * SCs + wn + 16 * j + li] = acc[nb][i][j][v];
  __syncthreads();

  const int rows_here = (int)(R - row0 < TM ? R - row0 : TM);
  const bool serial = cm.full && c <= 32;   // short probe segments: one thread per (row, probe)
  const int nw = cm.nw;

  if constexpr (GRAD) {
    const T* CA = Cs;
    const T* CB = Cs + TM * SCs;
    if (serial) {
      for (int it = tid; it < TM * np; it += 256) {
        const int m = it / np, p = it - m * np;
        if (m >= rows_here) continue;
        const int64_t r = row0 + m;
        const T* hr = H + r * c;
        double sab = 0.0, sa = 0.0, sb = 0.0;
        for (int k = 0; k < c; ++k) {
          const double h = (double)hr[k];
          const double ah = (double)CA[m * SCs + p * c + k] * h;
          const double b = (double)CB[m * SCs + p * c + k];
          sab += ah * b;
          sa += ah;
          sb += b * h;
        }
        double* o = gpart + ((r * s + p0 + p) * nw + w) * 3;
        o[0] = sab;
        o[1] = sa;
        o[2] = sb;
      }
    } else {
      for (int m = wave; m < rows_here; m += 4) {
        const int64_t r = row0 + m;
        const T* hr = H + r * c;
        double ah[NU], bb[NU], hh[NU];
        int sg[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int n = lane + 64 * u;
          sg[u] = -1;
          ah[u] = bb[u] = hh[u] = 0.0;
          if (n < width) {
            const int p = cm.full ? n / c : 0;
            const int kk = cm.full ? n - p * c : w * TN + n;
            hh[u] = (double)hr[kk];
            ah[u] = (double)CA[m * SCs + n] * hh[u];
            bb[u] = (double)CB[m * SCs + n];
            sg[u] = p;
          }
        }
        for (int p = 0; p < np; ++p) {
          double sab = 0.0, sa = 0.0, sb = 0.0;
#pragma unroll
          for (int u = 0; u < NU; ++u)
            if (sg[u] == p) {
              sab += ah[u] * bb[u];
              sa += ah[u];
              sb += bb[u] * hh[u];
            }
          sab = wave_sum(sab);
          sa = wave_sum(sa);
          sb = wave_sum(sb);
          if (lane == 0) {
            double* o = gpart + ((r * s + p0 + p) * nw + w) * 3;
            o[0] = sab;
            o[1] = sa;
            o[2] = sb;
          }
        }
      }
    }
  } else {
    T* Al = Cs + TM * SCs;   // [TM][kMaxPP]: alpha of each (row, probe) of the tile
    if (serial) {
      for (int it = tid; it < TM * np; it += 256) {
        const int m = it / np, p = it - m * np;
        if (m >= rows_here) continue;
        const T* hr = H + (row0 + m) * c;
        double sa = 0.0;
        for (int k = 0; k < c; ++k) sa += (double)Cs[m * SCs + p * c + k] * (double)hr[k];
        Al[m * kMaxPP + p] = (T)sa;
      }
    } else {
      for (int m = wave; m < rows_here; m += 4) {
        const T* hr = H + (row0 + m) * c;
        double gh[NU];
        int sg[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int n = lane + 64 * u;
          sg[u] = -1;
          gh[u] = 0.0;
          if (n < width) {
            const int p = cm.full ? n / c : 0;
            const int kk = cm.full ? n - p * c : w * TN + n;
            gh[u] = (double)Cs[m * SCs + n] * (double)hr[kk];
            sg[u] = p;
          }
        }
        for (int p = 0; p < np; ++p) {
          double sa = 0.0;
#pragma unroll
          for (int u = 0; u < NU; ++u)
            if (sg[u] == p) sa += gh[u];
          sa = wave_sum(sa);
          if (lane == 0) Al[m * kMaxPP + p] = (T)sa;
        }
      }
    }
    __syncthreads();
    for (int m = wave; m < rows_here; m += 4) {
      const int64_t r = row0 + m;
      T* go = Gout + r * SC + col0;
      if (cm.full) {
        const T* hr = H + r * c;
        const T om = omega ? (T)omega[r] : T(1);
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int n = lane + 64 * u;
          if (n < width) {
            const int p = n / c, kk = n - p * c;
            go[n] = om * ((Cs[m * SCs + n] - Al[m * kMaxPP + p]) * hr[kk]);
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int n = lane + 64 * u;
          if (n < width) go[n] = Cs[m * SCs + n];
        }
        if (lane == 0) abuf[(r * s + p0) * nw + w] = Al[m * kMaxPP];
      }
    }
  }
}

// Windowed probes: alpha_rj = sum over the nw windows, in order, stored in window slot 0.
template <typename T>
__global__ __launch_bounds__(256) void k_alpha_sum(T* __restrict__ abuf, int64_t n, int nw,
                                                   Skip skip) {
  if (skip_now(skip)) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T* a = abuf + i * nw;
  T acc = a[0];
  for (int w = 1; w < nw; ++w) acc += a[w];
  a[0] = acc;
}

// Kernel 2.  part[split][a, col] (+)= sum over the split's rows r of X[r, a] G'[r, col], with
// a d-tile of TM = 32 WM rows and a column tile of TN = 32 WN.  GAM: G holds raw products and
// the row step G' = omega_r (G - alpha_rj) h_rk is applied while staging.
template <typename T, int WM, int WN, bool GAM>
__global__ __launch_bounds__(256, 2) void k_xtg(
    const T* __restrict__ X, int d, const T* __restrict__ G, int SC, int64_t R,
    int64_t rows_per_split, int nmt, int nct, const T* __restrict__ H, int c, int s,
    const double* __restrict__ omega, const T* __restrict__ abuf, int nw, T* __restrict__ part,
    int64_t part_stride, int accumulate, Skip skip) {
  if (skip_now(skip)) return;
  constexpr int TM = 32 * WM, TN = 32 * WN, SA = TM + 16, SB = TN + 16;
  constexpr int EA = TM * kTK / 256, EB = TN * kTK / 256;
  constexpr int KA = 256 / TM, KB = 256 / TN;   // k-rows covered by one pass of the threads
  __shared__ __align__(16) T As[2][kTK][SA];
  __shared__ __align__(16) T Bs[2][kTK][SB];
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
  // this thread's staging column of G (fixed for the whole kernel)
  const int bn = tid % TN, bk = tid / TN;
  const int bcol = col0 + bn;
  const bool bvalid = bcol < SC;
  int bj = 0, bkk = 0;
  if (GAM && bvalid) {
    bj = bcol / c;
    bkk = bcol - bj * c;
  }
  const int am = tid % TM, ak = tid / TM;
  const bool avalid = a0 + am < d;

  typedef Mfma16<T> M;
  typename M::acc acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = M::zero();

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
      T v = T(0);
      if (r < re && bvalid) {
        v = G[r * SC + bcol];
        if (GAM) {
          const T om = omega ? (T)omega[r] : T(1);
          v = om * ((v - abuf[(r * s + bj) * nw]) * H[r * c + bkk]);
        }
      }
      rb_[i] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < EA; ++i) As[buf][ak + KA * i][am] = ra[i];
#pragma unroll
    for (int i = 0; i < EB; ++i) Bs[buf][bk + KB * i][bn] = rb_[i];
  };

  const int64_t nrows = re > rb ? re - rb : 0;
  const int nk = (int)((nrows + kTK - 1) / kTK);
  if (nk > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load(kt + 1);
#pragma unroll
    for (int q = 0; q < kTK / 4; ++q) {
      T av[WM], bv[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) av[i] = As[buf][4 * q + g][wm + 16 * i + li];
#pragma unroll
      for (int j = 0; j < WN; ++j) bv[j] = Bs[buf][4 * q + g][wn + 16 * j + li];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = M::run(av[i], bv[j], acc[i][j]);
    }
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  T* out = part + (int64_t)sp * part_stride;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = a0 + wm + 16 * i + M::row(g, v);
        const int col = col0 + wn + 16 * j + li;
        if (a < d && col < SC) {
          const int64_t o = (int64_t)a * SC + col;
          out[o] = accumulate ? out[o] + acc[i][j][v] : acc[i][j][v];
        }
      }
}

// g_r = -(1/s) sum_j [S_ab - S_a S_b], each S summed over the nw windows in order; one wave per row.
__global__ __launch_bounds__(256) void k_grad_sum(const double* __restrict__ gpart, int64_t R,
                                                  int s, int nw, double* __restrict__ g) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= R) return;
  double q = 0.0;
  for (int j = lane; j < s; j += 64) {
    const double* p = gpart + (r * s + j) * nw * 3;
    double sab = 0.0, sa = 0.0, sb = 0.0;
    for (int w = 0; w < nw; ++w) {
      sab += p[3 * w];
      sa += p[3 * w + 1];
      sb += p[3 * w + 2];
    }
    q += sab - sa * sb;
  }
  q = wave_sum(q);
  if (lane == 0) g[r] = -q / s;
}

// Tile shapes: FP32 product 128 x 128 (64 x 64 per wave); FP64 64 x 128; gradient tiles hold
// two operands and are half as wide.
template <typename T> struct Shape;
template <> struct Shape<float> {
  static constexpr int WM1 = 4, WN1 = 4, WM2 = 4, WN2 = 4, WMG = 4, WNG = 2;
};
template <> struct Shape<double> {
  static constexpr int WM1 = 2, WN1 = 4, WM2 = 2, WN2 = 4, WMG = 2, WNG = 2;
};

template <typename Kern>
int set_lds(Kern k, size_t bytes, bool& done) {
  if (!done && bytes > 65536) {
    FIRAL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  }
  done = true;
  return FIRAL_OK;
}

}  // namespace

// Largest windows-per-probe count and split count the tiled kernels need (buffer sizing).
int tiled_alpha_windows(int prec, int c) {
  const int TN = 32 * (prec == FIRAL_F64 ? Shape<double>::WN1 : Shape<float>::WN1);
  return c <= TN ? 1 : (int)cdiv(c, TN);
}
int tiled_grad_windows(int prec, int c) {
  const int TN = 32 * (prec == FIRAL_F64 ? Shape<double>::WNG : Shape<float>::WNG);
  return c <= TN ? 1 : (int)cdiv(c, TN);
}
int64_t tiled_out_tiles(int prec, int d, int64_t sc) {
  const int TM = 32 * (prec == FIRAL_F64 ? Shape<double>::WM2 : Shape<float>::WM2);
  const int TN = 32 * (prec == FIRAL_F64 ? Shape<double>::WN2 : Shape<float>::WN2);
  return cdiv(d, TM) * cdiv(sc, TN);
}

template <typename T>
static int hvp_tiled_t(Ctx* x, const double* omega, int64_t n_rows, double shift, const T* B,
                       T* out, int s, Skip skip, hipStream_t st) {
  typedef Shape<T> S_;
  constexpr int TM1 = 32 * S_::WM1, TN1 = 32 * S_::WN1;
  constexpr int TM2 = 32 * S_::WM2, TN2 = 32 * S_::WN2;
  const int d = x->d, c = x->c, SC = s * c;
  const ColMap cm = make_colmap(c, s, TN1);
  const T* X = (const T*)x->X;
  const T* H = (const T*)x->H;
  T* G = (T*)x->G;
  T* ab = (T*)x->abuf;
  T* part = (T*)x->part;
  const int64_t n_out = (int64_t)d * SC;
  const int nmt = (int)cdiv(d, TM2), nct = (int)cdiv(SC, TN2);
  const int64_t tiles = (int64_t)nmt * nct;
  const int64_t cap = (int64_t)x->max_splits * x->s_max / s;
  const int S = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(cdiv(1024, tiles), cap), 256));

  auto k1 = k_xv<T, S_::WM1, S_::WN1, 1, false>;
  constexpr size_t lds1 = xv_lds_bytes<T, S_::WM1, S_::WN1, 1, false>();
  static bool attr1 = false;
  FIRAL_CHECK(set_lds(k1, lds1, attr1));

  FIRAL_CHECK(prof_mark(x, st, true));
  for (int64_t r0 = 0; r0 < n_rows; r0 += x->chunk_rows) {
    const int64_t R = std::min<int64_t>(x->chunk_rows, n_rows - r0);
    const int64_t nrt = cdiv(R, TM1);
    const T* Xc = X + r0 * d;
    const T* Hc = H + r0 * c;
    const double* om = omega ? omega + r0 : nullptr;
    k1<<<(unsigned)(nrt * cm.ntiles), 256, lds1, st>>>(Xc, d, R, B, nullptr, Hc, om, cm, nrt, G,
                                                      ab, nullptr, skip);
    FIRAL_LAUNCHED();
    const int64_t rps = cdiv(R, S);
    const unsigned nwg2 = (unsigned)(tiles * S);
    if (cm.full) {
      k_xtg<T, S_::WM2, S_::WN2, false><<<nwg2, 256, 0, st>>>(
          Xc, d, G, SC, R, rps, nmt, nct, nullptr, c, s, nullptr, nullptr, 1, part, n_out,
          r0 > 0, skip);
    } else {
      k_alpha_sum<T><<<(unsigned)cdiv(R * s, 256), 256, 0, st>>>(ab, R * s, cm.nw, skip);
      FIRAL_LAUNCHED();
      k_xtg<T, S_::WM2, S_::WN2, true><<<nwg2, 256, 0, st>>>(
          Xc, d, G, SC, R, rps, nmt, nct, Hc, c, s, om, ab, cm.nw, part, n_out, r0 > 0, skip);
    }
    FIRAL_LAUNCHED();
  }
  FIRAL_CHECK(prof_mark(x, st, false));
  return reduce_parts_launch<T>(part, n_out, n_rows > 0 ? S : 0, shift, B, out, skip, st);
}

int hvp_tiled_launch(Ctx* x, const double* omega, int64_t n_rows, double shift, const void* B,
                     void* out, int s, Skip skip, hipStream_t st) {
  if (x->prec == FIRAL_F64)
    return hvp_tiled_t<double>(x, omega, n_rows, shift, (const double*)B, (double*)out, s, skip,
                               st);
  return hvp_tiled_t<float>(x, omega, n_rows, shift, (const float*)B, (float*)out, s, skip, st);
}

template <typename T>
static int grad_tiled_t(Ctx* x, const T* U, const T* W, int s, double* g, hipStream_t st) {
  typedef Shape<T> S_;
  constexpr int TM = 32 * S_::WMG, TN = 32 * S_::WNG;
  const int d = x->d, c = x->c;
  const ColMap cm = make_colmap(c, s, TN);
  auto k = k_xv<T, S_::WMG, S_::WNG, 2, true>;
  constexpr size_t lds = xv_lds_bytes<T, S_::WMG, S_::WNG, 2, true>();
  static bool attr = false;
  FIRAL_CHECK(set_lds(k, lds, attr));
  for (int64_t r0 = 0; r0 < x->n_pool; r0 += x->chunk_rows) {
    const int64_t R = std::min<int64_t>(x->chunk_rows, x->n_pool - r0);
    const int64_t nrt = cdiv(R, TM);
    k<<<(unsigned)(nrt * cm.ntiles), 256, lds, st>>>((const T*)x->X + r0 * d, d, R, U, W,
                                                    (const T*)x->H + r0 * c, nullptr, cm, nrt,
                                                    nullptr, nullptr, x->gpart, skip_none());
    FIRAL_LAUNCHED();
    k_grad_sum<<<(unsigned)cdiv(R, 4), 256, 0, st>>>(x->gpart, R, s, cm.nw, g + r0);
    FIRAL_LAUNCHED();
  }
  return FIRAL_OK;
}

int grad_launch(Ctx* x, const void* U, const void* W, int s, double* g, hipStream_t st) {
  if (x->prec == FIRAL_F64)
    return grad_tiled_t<double>(x, (const double*)U, (const double*)W, s, g, st);
  return grad_tiled_t<float>(x, (const float*)U, (const float*)W, s, g, st);
}

}  // namespace firal
