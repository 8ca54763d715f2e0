// The Hessian product of Lemma 1 without a context and without any allocation, for callers
// that cannot allocate device memory (code under stream capture, serving loops that forbid
// hipMalloc).  It runs the fused single-pass FP32 kernel of firal_hvp (d <= 128) and keeps that
// kernel's per-row-range partial sums of the output block in a fixed device array of this file
// instead of a context's workspace.
#include <cstring>
#include <mutex>

#include "common.h"

namespace firal {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB of partial sums per device
constexpr int kMaxDevices = 64;

// The partial sums.  Each device the library runs on holds its own copy until the process
// ends.  Host code never passes this name to a kernel: it is a host-side stand-in, and the
// device address comes from hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per device).
int scratch_address(void** out) {
  int dev = -1;
  FIRAL_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d outside the %d devices the allocation-free product supports", dev,
              kMaxDevices);
    return FIRAL_ENOTSUP;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    FIRAL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FIRAL_OK;
}

}  // namespace
}  // namespace firal

using namespace firal;

extern "C" int firal_hvp_noalloc(const float* X, const float* H, int64_t n_rows, int32_t d,
                                 int32_t c, const double* omega, double shift, const float* B,
                                 float* out, int32_t s, void* stream) {
  if (!X || !H || !B || !out) {
    set_error("firal_hvp_noalloc: null X, H, B or out");
    return FIRAL_EINVAL;
  }
  if (n_rows < 0 || d < 1 || c < 2 || s < 1) {
    set_error("firal_hvp_noalloc: n_rows = %lld, d = %d, c = %d, s = %d out of range",
              (long long)n_rows, d, c, s);
    return FIRAL_EINVAL;
  }
  if (B == out) {
    set_error("firal_hvp_noalloc: out must not alias B");
    return FIRAL_EINVAL;
  }
  if (d > 128) {
    set_error("firal_hvp_noalloc: d = %d; the allocation-free product covers d <= 128", d);
    return FIRAL_ENOTSUP;
  }
  hipStream_t st = (hipStream_t)stream;
  // a context on the stack that holds only what the fused kernel reads (no workspace)
  Ctx x;
  std::memset(&x, 0, sizeof(x));
  x.n_pool = x.N = n_rows;
  x.d = d;
  x.c = c;
  x.s_max = s;
  x.prec = FIRAL_F32;
  x.esize = 4;
  x.X = X;
  x.H = H;
  x.fused_max_ncb = 1;
  // the tile plan and the size check are host arithmetic: an oversized call is refused before
  // any device call
  FusedPlan p;
  if (n_rows > 0) {
    if (!fused_plan(&x, s, n_rows, &p)) {
      set_error("firal_hvp_noalloc: no single-pass tile plan for d = %d, c = %d, s = %d", d, c, s);
      return FIRAL_ENOTSUP;
    }
    if ((size_t)p.part_elems * sizeof(float) > kScratchBytes) {
      set_error("firal_hvp_noalloc: the partial sums need %lld bytes, more than the %zu bytes of "
                "the fixed device array (n_rows %lld, d %d, c %d, s %d)",
                (long long)p.part_elems * 4, kScratchBytes, (long long)n_rows, d, c, s);
      return FIRAL_EINVAL;
    }
  }
  void* part = nullptr;
  FIRAL_CHECK(scratch_address(&part));
  x.fused_part = part;
  if (n_rows == 0)   // no rows: out = shift * B
    return reduce_parts_launch<float>((const float*)part, (int64_t)d * s * c, 0, shift, B, out,
                                      skip_none(), st);
  return hvp_fused_launch(&x, p, omega, n_rows, shift, B, out, s, skip_none(), st);
}
