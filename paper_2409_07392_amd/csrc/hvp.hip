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
// pass (here) sums in a fixed order (no float atomics: results are reproducible).
// Dispatch: the single-pass fused kernel (hvp_fused.hip) for FP32 / bf16x3 when
// its tile plan fits, else for wide FP32 problems the transposed-operand GEMMs of gemm_nt.hip,
// else the row-tiled two-kernel path (tiled.hip).
#include <algorithm>

#include "common.h"

namespace firal {

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
template int reduce_parts_launch<double>(const double*, int64_t, int, double, const double*,
                                         double*, Skip, hipStream_t);

int hvp_launch(Ctx* x, const double* omega, int64_t n_rows, double shift, const void* B,
               void* out, int s, Skip skip, hipStream_t st, bool precise) {
  FusedPlan plan;
  if (x->prec != FIRAL_F64 && !x->force_tiled && fused_plan(x, s, n_rows, &plan, precise) &&
      plan.part_elems <= x->fused_part_elems)
    return hvp_fused_launch(x, plan, omega, n_rows, shift, (const float*)B, (float*)out, s, skip,
                            st);
  // the wide path's bf16x3 context has no FP32 X^T: its FP32 products (precise) stay row-tiled
  if (x->use_nt && !x->force_tiled && !(x->prec == FIRAL_BF16X3 && precise))
    return hvp_nt_launch(x, omega, n_rows, shift, (const float*)B, (float*)out, s, skip, st);
  return hvp_tiled_launch(x, omega, n_rows, shift, B, out, s, skip, st, precise);
}

}  // namespace firal
