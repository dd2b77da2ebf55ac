// Allocation-free spectrum image, for callers that cannot call hipMalloc
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// device allocation).  The per-probe sums and the k-axis tables that
// tacaw_spectrum_image keeps in freshly allocated device buffers live here in
// one fixed device array instead; the kernel is the same.
//
// Host code never passes the array's own name to a kernel or a copy: that
// name is a host-side stand-in.  Its device address is looked up once per
// device (with that device current) when a context is created there, and
// only that address is used.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "runtime.h"

namespace tacaw {
namespace {

// per-probe results, then the kx and ky axes
constexpr size_t kMaxProbes = 65536;
constexpr size_t kMaxAxis = 4096;   // nx + ny
constexpr size_t kScratchDoubles = kMaxProbes + kMaxAxis;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device

}  // namespace

tacaw_status noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device %d outside the %d the library tracks", device, kMaxDevices);
    return TACAW_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return TACAW_OK;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess || cur != device) {
    set_error("scratch lookup for device %d with device %d current", device, cur);
    return TACAW_EDEVICE;
  }
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    set_error("hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    return TACAW_EDEVICE;
  }
  g_scratch[device] = (double*)p;
  return TACAW_OK;
}

}  // namespace tacaw

using namespace tacaw;

#define N_TRY(call)                                                         \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      set_error("%s failed: %s", #call, hipGetErrorString(e_));             \
      return TACAW_EDEVICE;                                                 \
    }                                                                       \
  } while (0)

extern "C" tacaw_status tacaw_spectrum_image_noalloc(tacaw_job* job, double f_THz, double k_inner, double k_outer,
                                                     double* dst, size_t n, int dst_on_device) {
  clear_error();
  tacaw_status st = check_ready(job);
  if (st != TACAW_OK) return st;
  const HostPlan& hp = job->hp;
  if (!dst || n != (size_t)hp.P) {
    set_error("dst must hold one value per probe (%d)", hp.P);
    return TACAW_EINVAL;
  }
  if ((size_t)hp.P > kMaxProbes || (size_t)hp.nx + hp.ny > kMaxAxis) {
    set_error("tacaw_spectrum_image_noalloc holds at most %zu probes and nx + ny <= %zu in its fixed scratch "
              "(job: %d probes, nx + ny = %d); use tacaw_spectrum_image",
              kMaxProbes, kMaxAxis, hp.P, hp.nx + hp.ny);
    return TACAW_EINVAL;
  }
  if (!(k_inner >= 0.0) || !(k_outer <= 0.0 || k_outer > k_inner)) {
    set_error("need 0 <= k_inner and (k_outer <= 0 or k_outer > k_inner)");
    return TACAW_EINVAL;
  }
  int m = 0;
  if ((st = nearest_bin(job, f_THz, &m)) != TACAW_OK) return st;
  const int dev = job->ctx->device;
  N_TRY(hipSetDevice(dev));
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    base = dev >= 0 && dev < kMaxDevices ? g_scratch[dev] : nullptr;
  }
  if (!base) {   // contexts look it up at creation; this covers nothing else
    if ((st = noalloc_init(dev)) != TACAW_OK) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    base = g_scratch[dev];
  }
  double* out = base;
  double* axes = base + kMaxProbes;
  // every value the kernel reads is written here first (the axes), and it
  // writes every out[p], p < P: nothing needs clearing between calls
  const std::vector<double> ax = k_axes(hp);
  hipStream_t s = job->last_stream;
  N_TRY(hipMemcpyAsync(axes, ax.data(), ax.size() * sizeof(double), hipMemcpyHostToDevice, s));
  N_TRY(launch_spectrum_image(job->d_spec, out, hp.P, hp.M, hp.nx, hp.ny, m, axes, axes + hp.nx,
                              k_inner * k_inner, k_outer > 0.0 ? k_outer * k_outer : 0.0, s));
  if (dst_on_device) {
    N_TRY(hipMemcpyAsync(dst, out, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    N_TRY(hipStreamSynchronize(s));
  } else {
    N_TRY(hipStreamSynchronize(s));
    N_TRY(hipMemcpy(dst, out, n * sizeof(double), hipMemcpyDeviceToHost));
  }
  return TACAW_OK;
}
