// Measurement aid: sustained HBM bandwidth of a pure streaming kernel with a
// given read:write mix, the practical ceiling the hopping kernel's roofline is
// compared with (its traffic is about 7 bytes read per byte written).
#include <chrono>

#include "../../include/wdirac.h"
#include "wd_common.h"

namespace wd {

using v2d = double __attribute__((ext_vector_type(2)));

// out[i] = sum of the NR input streams at i; one 16-byte element per lane per
// stream, non-temporal loads and stores.
template <int NR>
__global__ __launch_bounds__(256) void k_stream(const v2d *__restrict__ in, v2d *__restrict__ out, size_t elems) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= elems) return;
  v2d acc = {0.0, 0.0};
#pragma unroll
  for (int s = 0; s < NR; ++s) acc += __builtin_nontemporal_load(in + (size_t)s * elems + i);
  __builtin_nontemporal_store(acc, out + i);
}

template <int NR>
static hipError_t launch_stream(const v2d *in, v2d *out, size_t elems, hipStream_t st) {
  const size_t grid = (elems + 255) / 256;
  hipLaunchKernelGGL(k_stream<NR>, dim3((unsigned)grid), dim3(256), 0, st, in, out, elems);
  return hipGetLastError();
}

static hipError_t launch_stream_n(int nread, const v2d *in, v2d *out, size_t elems, hipStream_t st) {
  switch (nread) {
    case 1: return launch_stream<1>(in, out, elems, st);
    case 2: return launch_stream<2>(in, out, elems, st);
    case 3: return launch_stream<3>(in, out, elems, st);
    case 4: return launch_stream<4>(in, out, elems, st);
    case 5: return launch_stream<5>(in, out, elems, st);
    case 6: return launch_stream<6>(in, out, elems, st);
    case 7: return launch_stream<7>(in, out, elems, st);
    case 8: return launch_stream<8>(in, out, elems, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace wd

extern "C" int wdirac_stream_probe(void *bufs, size_t elems, int nread, int reps, double *gbps, void *stream) {
  if (!bufs || !gbps || elems == 0 || elems > ((size_t)1 << 31) || nread < 1 || nread > 8 || reps < 1 ||
      reps > 1000)
    return WDIRAC_EINVAL;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  using wd::v2d;
  const v2d *in = static_cast<const v2d *>(bufs);
  v2d *out = static_cast<v2d *>(bufs) + (size_t)nread * elems;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return WDIRAC_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return WDIRAC_EHIP;
  }
  int rc = WDIRAC_OK;
  if (wd::launch_stream_n(nread, in, out, elems, st) != hipSuccess) rc = WDIRAC_EHIP;
  if (rc == WDIRAC_OK && hipEventRecord(e0, st) != hipSuccess) rc = WDIRAC_EHIP;
  for (int k = 0; k < reps && rc == WDIRAC_OK; ++k)
    if (wd::launch_stream_n(nread, in, out, elems, st) != hipSuccess) rc = WDIRAC_EHIP;
  if (rc == WDIRAC_OK && hipEventRecord(e1, st) != hipSuccess) rc = WDIRAC_EHIP;
  if (rc == WDIRAC_OK && hipEventSynchronize(e1) != hipSuccess) rc = WDIRAC_EHIP;
  float ms = 0.0f;
  if (rc == WDIRAC_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = WDIRAC_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != WDIRAC_OK) return rc;
  const double bytes = (double)(nread + 1) * (double)elems * 16.0 * reps;
  *gbps = bytes / (ms * 1e-3) / 1e9;
  return WDIRAC_OK;
}
