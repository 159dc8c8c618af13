// Allocation-free semi-Lagrangian transport (claire_transport_noalloc).
//
// The same kernels as claire_transport (RK2 backtrace, per-brick stencil
// boxes, nt LDS-staged tricubic gathers; Section 2.5.2, eq. e:transport), but
// every intermediate buffer lives in one file-scope device array instead of a
// context workspace, so the call makes no device allocation. The array is
// per device (each GPU that runs the call holds its own copy until the
// process ends); its device address is looked up once per device with
// hipGetSymbolAddress and only that address is handed to kernels and runtime
// calls. All calls on one device share the array: calls that overlap in time
// on one device (two streams, two threads) race and must be serialised by
// the caller.

#include "internal.h"

#include <mutex>

namespace claire {
namespace {

// Largest grid served: 2^21 voxels (e.g. 128^3).
constexpr long long kMaxVoxels = 1LL << 21;
// Scratch layout in floats: departure displacements of +v and -v (3 fields
// each), one ping-pong field of the state, then the per-brick box table
// (6 ints per brick, at most kMaxVoxels / 64 bricks).
constexpr long long kScratchFloats = 7 * kMaxVoxels + 6 * (kMaxVoxels / 64);

__device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
float* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of this device's copy of `scratch` (looked up on first use
// with the device current; the array's host-side name is not an address).
int scratch_ptr(float** out) {
    int dev = 0;
    CL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d beyond the %d devices the scratch table covers", dev, kMaxDevices);
        return CLAIRE_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        CL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress returned NULL for the transport scratch array");
            return CLAIRE_EDEVICE;
        }
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

}  // namespace
}  // namespace claire

using namespace claire;

extern "C" long long claire_transport_noalloc_max_voxels(void) { return kMaxVoxels; }

extern "C" int claire_transport_noalloc(const float* m0, const float* v, const int nx[3], int nt,
                                        float* m1_out, void* stream) {
    if (!m0 || !v || !m1_out || !nx) {
        set_error("claire_transport_noalloc: NULL pointer argument");
        return CLAIRE_EINVAL;
    }
    CL_TRY(check_extents(nx));
    if (nt < 1 || nt > 64) {
        set_error("nt = %d out of range [1, 64]", nt);
        return CLAIRE_EINVAL;
    }
    const Geo g = make_geo(nx);
    if (g.n > kMaxVoxels) {
        set_error("claire_transport_noalloc: %lld voxels exceed the scratch limit of %lld "
                  "(use claire_transport)", g.n, kMaxVoxels);
        return CLAIRE_EINVAL;
    }
    if (brick_table_ints(g) > kScratchFloats - 7 * g.n) {
        set_error("claire_transport_noalloc: brick table of %d ints exceeds its scratch slot",
                  brick_table_ints(g));
        return CLAIRE_EINVAL;
    }
    if (m1_out == m0) {
        set_error("claire_transport_noalloc: m1_out must not alias m0");
        return CLAIRE_EINVAL;
    }
    float* base = nullptr;
    CL_TRY(scratch_ptr(&base));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long long n = g.n;
    float* dp = base;              // [3][n] departure displacement of +v
    float* dm = base + 3 * n;      // [3][n] of -v (the backtrace kernel writes both)
    float* ping = base + 6 * n;    // [n] intermediate state
    int* table = reinterpret_cast<int*>(base + 7 * n);
    CL_TRY(launch_backtrace(g, v, dp, dm, 1.0 / nt, s));
    CL_TRY(launch_brick_boxes(g, dp, table, s));
    // m^{j+1} = m^j(y+): alternate between the ping field and m1_out so that
    // the last step lands in m1_out
    const float* src = m0;
    for (int j = 0; j < nt; ++j) {
        float* dst = ((nt - 1 - j) & 1) ? ping : m1_out;
        CL_TRY(launch_interp(g, src, 1, dp, dst, s, table));
        src = dst;
    }
    CL_HIP(hipStreamSynchronize(s));
    return 0;
}
