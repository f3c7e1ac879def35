// asep_noalloc.hip -- asep_run_noalloc: a whole run whose workspace is one
// fixed device array per GPU instead of buffers allocated per simulation.
//
// The array `scratch` is a device symbol.  Host code never passes its name
// to a kernel or a copy (on the host the name is a stand-in, not a device
// address); it looks the device address up once per device with
// hipGetSymbolAddress, with that device current, and uses that address only.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/asep.h"
#include "asep_internal.h"

namespace asep {
namespace {

static __device__ __align__(256) unsigned char scratch[ASEP_NOALLOC_SCRATCH_BYTES];

// Exact unsigned 128-bit value hi:lo rounded once to binary64 (nearest, ties
// to even): the top 64 significant bits with every lower bit folded into
// their last bit (a sticky bit, which only matters below the rounding
// position), converted as two exact 32-bit halves added with one rounding.
__device__ double u128_to_double(uint64_t hi, uint64_t lo) {
    int sh = 0;
    uint64_t m = lo;
    if (hi) {
        const int lz = __clzll(hi);
        m = lz ? (hi << lz) | (lo >> (64 - lz)) : hi;
        const uint64_t rest = lz ? lo << lz : lo;
        m |= rest != 0 ? 1u : 0u;
        sh = 64 - lz;
    }
    const double d = ldexp((double)(uint32_t)(m >> 32), 32) + (double)(uint32_t)m;
    return ldexp(d, sh);
}

// Records to asep_rough: the integers as they are, W^2 = (L S2 - S1^2) / L^2
// (Eq. W, population variance) with the numerator exact in 128 bits.
__global__ void k_rough_out(const Record* __restrict__ rec, asep_rough* __restrict__ out,
                            uint32_t n, uint64_t L) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Record r = rec[i];
    // L S2: 64 x 128 -> 128 bits (the true value is below 2^128)
    const uint64_t s2lo = r.s2lo, s2hi = (uint64_t)r.s2hi;
    uint64_t lo = L * s2lo;
    uint64_t hi = __umul64hi(L, s2lo) + L * s2hi;
    // S1^2
    const uint64_t a = (uint64_t)(r.s1 < 0 ? -r.s1 : r.s1);
    const uint64_t qlo = a * a, qhi = __umul64hi(a, a);
    // L S2 - S1^2 >= 0 (a variance)
    const uint64_t borrow = lo < qlo ? 1u : 0u;
    lo -= qlo;
    hi = hi - qhi - borrow;
    asep_rough o;
    o.sum_h = r.s1;
    o.sum_h2_lo = r.s2lo;
    o.sum_h2_hi = r.s2hi;
    o.hops = r.hops;
    o.particles = r.n;
    o.w2 = u128_to_double(hi, lo) / ((double)L * (double)L);
    out[i] = o;
}

hipError_t launch_rough_out(const Record* rec, asep_rough* out, uint32_t n, uint64_t L,
                            hipStream_t st) {
    if (n == 0) return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_rough_out, dim3((n + 255) / 256), dim3(256), 0, st, rec, out, n, L);
    return hipGetLastError();
}

// Device address of `scratch` on each device, looked up on the first call
// made with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];

int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return ASEP_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return device_error(e, "hipGetSymbolAddress(scratch)");
        g_ptr[dev] = ptr;
    }
    *out = g_ptr[dev];
    return ASEP_OK;
}

}  // namespace
}  // namespace asep

extern "C" int asep_run_noalloc(const asep_params* p, uint64_t* state_dev, size_t state_bytes,
                                void* hip_stream, const uint64_t* times, uint32_t n_times,
                                asep_rough* out_dev) {
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return asep::device_error(e, "hipGetDevice");
    void* ws = nullptr;
    const int rc = asep::scratch_address(dev, &ws);
    if (rc) return rc;
    return asep::sim_run_scratch(p, state_dev, state_bytes, (hipStream_t)hip_stream, ws,
                                 ASEP_NOALLOC_SCRATCH_BYTES, times, n_times, out_dev,
                                 asep::launch_rough_out);
}
