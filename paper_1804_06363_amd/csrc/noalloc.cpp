// Entry points that allocate no device memory.  Their device-side staging lives in one
// file-scope array of fixed size, `scratch`; every GPU the library runs on holds its own
// copy until the process ends.  Host code never passes the array's name to a kernel or
// a copy (on the host that name is only a stand-in): the device address of each GPU's
// copy is looked up once, when the first context on that GPU is created, and kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"
#include "kernels.h"

namespace rb {

static __device__ __align__(256) unsigned char scratch[RB_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

size_t round256(size_t v) { return (v + 255) / 256 * 256; }

// the device address of `scratch` on `device`, or RB_EDEVICE if it was never resolved
unsigned char* scratch_on(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  RB_REQUIRE(device >= 0 && device < kMaxDevices && g_ptr[device], RB_EDEVICE,
             "the fixed scratch buffer of device " + std::to_string(device) +
                 " was not resolved (no context was created on it)");
  return static_cast<unsigned char*>(g_ptr[device]);
}
}  // namespace

void noalloc_attach(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  RB_REQUIRE(device >= 0 && device < kMaxDevices, RB_EUNSUPPORTED,
             "device index beyond the scratch table");
  if (g_ptr[device]) return;
  void* p = nullptr;
  RB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  RB_REQUIRE(p, RB_EDEVICE, "hipGetSymbolAddress returned a null scratch address");
  g_ptr[device] = p;
}

}  // namespace rb

using namespace rb;

extern "C" {

rb_status rb_reduced_factor_batch_noalloc(rb_ctx* ctx, const rb_basis* bs, int B,
                                          const double* theta, double* L, rb_status* status) {
  static_assert(sizeof(rb_status) == sizeof(int), "statuses are copied as int");
  return guarded([&] {
    RB_REQUIRE(ctx && bs && theta && L && status && B >= 1 && B <= 65535, RB_EINVAL,
               "bad arguments");
    const int n = bs->n, Q = bs->prob->g.Q;
    RB_REQUIRE(n >= 1, RB_EINVAL, "empty basis");
    // layout in the buffer: theta [B][Q], L [B][n][n], status [B], each 256-byte aligned
    const size_t th_b = round256(sizeof(double) * (size_t)B * Q);
    const size_t L_b = round256(sizeof(double) * (size_t)B * n * n);
    const size_t st_b = round256(sizeof(int) * (size_t)B);
    const size_t need = th_b + L_b + st_b;
    RB_REQUIRE(need <= (size_t)RB_NOALLOC_SCRATCH_BYTES, RB_EINVAL,
               "B = " + std::to_string(B) + " queries with n = " + std::to_string(n) +
                   ", Q = " + std::to_string(Q) + " need " + std::to_string(need) +
                   " bytes of staging, more than the fixed buffer's " +
                   std::to_string((size_t)RB_NOALLOC_SCRATCH_BYTES));
    check_finite(theta, (size_t)B * Q, "theta");
    DeviceGuard dg(ctx->device);
    unsigned char* base = scratch_on(ctx->device);
    double* th = reinterpret_cast<double*>(base);
    double* Ld = reinterpret_cast<double*>(base + th_b);
    int* sd = reinterpret_cast<int*>(base + th_b + L_b);
    hipStream_t st = ctx->stream;
    RB_HIP(hipMemcpyAsync(th, theta, sizeof(double) * (size_t)B * Q, hipMemcpyHostToDevice, st));
    // the kernel writes every entry of L and every status, so nothing is cleared first
    launch_cholesky(bs->AN.as<double>(), n, Q, B, th, nullptr, Ld, sd, st);
    RB_HIP(hipMemcpyAsync(L, Ld, sizeof(double) * (size_t)B * n * n, hipMemcpyDeviceToHost, st));
    RB_HIP(hipMemcpyAsync(status, sd, sizeof(int) * (size_t)B, hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
  });
}

}  // extern "C"
