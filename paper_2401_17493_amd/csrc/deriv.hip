// 8th-order finite-difference gradient and divergence (Section 2.5.3,
// "Differentiation": the first-derivative discretisation of the paper's GPU
// code), periodic:
//   d_i u(x_l) ~ (3 u_{l-4} - 32 u_{l-3} + 168 u_{l-2} - 672 u_{l-1}
//                 + 672 u_{l+1} - 168 u_{l+2} + 32 u_{l+3} - 3 u_{l+4}) / (840 h_i),
// evaluated as 672 (u_{+1} - u_{-1}) - 168 (u_{+2} - u_{-2}) + 32 (u_{+3} - u_{-3})
// - 3 (u_{+4} - u_{-4}) so that neighbouring values cancel before weighting.
// One thread per voxel, x3 fastest across the wave: the x3 neighbours are
// the same cache lines, the x2 and x1 neighbours whole rows read by the wave
// together (L1/L2 hits for all but one of the nine rows per axis).

#include "internal.h"

namespace claire {
namespace {

constexpr int kThreads = 256;

struct Lat {
    int m1, m2, m3;   // extent - 1
    int l3, s1;       // shifts: x2 by l3, x1 by l2 + l3
};

__device__ __forceinline__ float ld(const float* p, unsigned i) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(p) + (i << 2));
}
__device__ __forceinline__ float ldf(const float* p, unsigned i) { return ld(p, i); }

// FD8 sums along the three axes at voxel idx of field u (not yet scaled by
// 1 / (840 h)).
__device__ __forceinline__ void fd8_sums(const float* __restrict__ u, const Lat& L, unsigned idx,
                                         float& d1, float& d2, float& d3) {
    const int i3 = idx & L.m3;
    const int i2 = (idx >> L.l3) & L.m2;
    const int i1 = idx >> L.s1;
    const unsigned r1 = idx & ((1u << L.s1) - 1);                        // i2, i3 part
    const unsigned r2 = idx & ~((unsigned)L.m2 << L.l3);                 // i1, i3 part
    const unsigned r3 = idx & ~(unsigned)L.m3;                           // i1, i2 part
    auto a1 = [&](int s) { return ld(u, ((unsigned)((i1 + s) & L.m1) << L.s1) | r1); };
    auto a2 = [&](int s) { return ld(u, ((unsigned)((i2 + s) & L.m2) << L.l3) | r2); };
    auto a3 = [&](int s) { return ld(u, (unsigned)((i3 + s) & L.m3) | r3); };
    d1 = 672.f * (a1(1) - a1(-1)) - 168.f * (a1(2) - a1(-2)) + 32.f * (a1(3) - a1(-3)) -
         3.f * (a1(4) - a1(-4));
    d2 = 672.f * (a2(1) - a2(-1)) - 168.f * (a2(2) - a2(-2)) + 32.f * (a2(3) - a2(-3)) -
         3.f * (a2(4) - a2(-4));
    d3 = 672.f * (a3(1) - a3(-1)) - 168.f * (a3(2) - a3(-2)) + 32.f * (a3(3) - a3(-3)) -
         3.f * (a3(4) - a3(-4));
}

// out[a] = d_a u, a = 0..2; c_a = 1 / (840 h_a)
__global__ __launch_bounds__(kThreads) void k_fd8_grad(const float* __restrict__ u,
                                                       float* __restrict__ out, Lat L,
                                                       long long n, float c1, float c2, float c3) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    float d1, d2, d3;
    fd8_sums(u, L, (unsigned)i, d1, d2, d3);
    out[i] = c1 * d1;
    out[n + i] = c2 * d2;
    out[2 * n + i] = c3 * d3;
}

// out = d_1 v_1 + d_2 v_2 + d_3 v_3 (only the own-axis sum of each component)
__global__ __launch_bounds__(kThreads) void k_fd8_div(const float* __restrict__ v,
                                                      float* __restrict__ out, Lat L,
                                                      long long n, float c1, float c2, float c3) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const unsigned idx = (unsigned)i;
    const int i3 = idx & L.m3;
    const int i2 = (idx >> L.l3) & L.m2;
    const int i1 = idx >> L.s1;
    const unsigned r1 = idx & ((1u << L.s1) - 1);
    const unsigned r2 = idx & ~((unsigned)L.m2 << L.l3);
    const unsigned r3 = idx & ~(unsigned)L.m3;
    const float* v1 = v;
    const float* v2 = v + n;
    const float* v3 = v + 2 * n;
    auto a1 = [&](int s) { return ld(v1, ((unsigned)((i1 + s) & L.m1) << L.s1) | r1); };
    auto a2 = [&](int s) { return ld(v2, ((unsigned)((i2 + s) & L.m2) << L.l3) | r2); };
    auto a3 = [&](int s) { return ld(v3, (unsigned)((i3 + s) & L.m3) | r3); };
    const float d1 = 672.f * (a1(1) - a1(-1)) - 168.f * (a1(2) - a1(-2)) +
                     32.f * (a1(3) - a1(-3)) - 3.f * (a1(4) - a1(-4));
    const float d2 = 672.f * (a2(1) - a2(-1)) - 168.f * (a2(2) - a2(-2)) +
                     32.f * (a2(3) - a2(-3)) - 3.f * (a2(4) - a2(-4));
    const float d3 = 672.f * (a3(1) - a3(-1)) - 168.f * (a3(2) - a3(-2)) +
                     32.f * (a3(3) - a3(-3)) - 3.f * (a3(4) - a3(-4));
    out[i] = c1 * d1 + c2 * d2 + c3 * d3;
}

// General extents (n1, n2 not powers of two): neighbours along x1 and x2
// by a modulo wrap, x3 (a power of two) by a mask.
struct LatG {
    int n1, n2, m3, l3;
};

__device__ __forceinline__ int wrapn(int x, int n) {
    const int r = x % n;
    return r < 0 ? r + n : r;
}

template <bool DIV>
__global__ __launch_bounds__(kThreads) void k_fd8_gen(const float* __restrict__ u,
                                                      float* __restrict__ out, LatG L,
                                                      long long n, float c1, float c2,
                                                      float c3) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const unsigned idx = (unsigned)i;
    const int i3 = idx & L.m3;
    const unsigned r = idx >> L.l3;
    const int i2 = (int)(r % (unsigned)L.n2);
    const int i1 = (int)(r / (unsigned)L.n2);
    const float* u1 = u;
    const float* u2 = DIV ? u + n : u;
    const float* u3 = DIV ? u + 2 * n : u;
    auto a1 = [&](int s) {
        return ldf(u1, (unsigned)(((wrapn(i1 + s, L.n1) * L.n2 + i2) << L.l3) + i3));
    };
    auto a2 = [&](int s) {
        return ldf(u2, (unsigned)(((i1 * L.n2 + wrapn(i2 + s, L.n2)) << L.l3) + i3));
    };
    auto a3 = [&](int s) { return ldf(u3, (idx & ~(unsigned)L.m3) | ((i3 + s) & L.m3)); };
    const float d1 = 672.f * (a1(1) - a1(-1)) - 168.f * (a1(2) - a1(-2)) +
                     32.f * (a1(3) - a1(-3)) - 3.f * (a1(4) - a1(-4));
    const float d2 = 672.f * (a2(1) - a2(-1)) - 168.f * (a2(2) - a2(-2)) +
                     32.f * (a2(3) - a2(-3)) - 3.f * (a2(4) - a2(-4));
    const float d3 = 672.f * (a3(1) - a3(-1)) - 168.f * (a3(2) - a3(-2)) +
                     32.f * (a3(3) - a3(-3)) - 3.f * (a3(4) - a3(-4));
    if (DIV) {
        out[i] = c1 * d1 + c2 * d2 + c3 * d3;
    } else {
        out[i] = c1 * d1;
        out[n + i] = c2 * d2;
        out[2 * n + i] = c3 * d3;
    }
}

Lat make_lat(const Geo& g) {
    Lat L;
    L.m1 = g.n1 - 1;
    L.m2 = g.n2 - 1;
    L.m3 = g.n3 - 1;
    L.l3 = g.l3;
    L.s1 = g.l2 + g.l3;
    return L;
}

float inv840h(int n) { return (float)((double)n / (2.0 * M_PI * 840.0)); }

}  // namespace

int launch_fd8_grad(const Geo& g, const float* u, float* out, hipStream_t s) {
    const unsigned nb = (unsigned)((g.n + kThreads - 1) / kThreads);
    if (!g.pow2) {
        hipLaunchKernelGGL(k_fd8_gen<false>, dim3(nb), dim3(kThreads), 0, s, u, out,
                           LatG{g.n1, g.n2, g.n3 - 1, g.l3}, g.n, inv840h(g.n1), inv840h(g.n2),
                           inv840h(g.n3));
        CL_LAUNCH_CHECK();
        return 0;
    }
    hipLaunchKernelGGL(k_fd8_grad, dim3(nb), dim3(kThreads), 0, s, u, out, make_lat(g), g.n,
                       inv840h(g.n1), inv840h(g.n2), inv840h(g.n3));
    CL_LAUNCH_CHECK();
    return 0;
}

int launch_fd8_div(const Geo& g, const float* v, float* out, hipStream_t s) {
    const unsigned nb = (unsigned)((g.n + kThreads - 1) / kThreads);
    if (!g.pow2) {
        hipLaunchKernelGGL(k_fd8_gen<true>, dim3(nb), dim3(kThreads), 0, s, v, out,
                           LatG{g.n1, g.n2, g.n3 - 1, g.l3}, g.n, inv840h(g.n1), inv840h(g.n2),
                           inv840h(g.n3));
        CL_LAUNCH_CHECK();
        return 0;
    }
    hipLaunchKernelGGL(k_fd8_div, dim3(nb), dim3(kThreads), 0, s, v, out, make_lat(g), g.n,
                       inv840h(g.n1), inv840h(g.n2), inv840h(g.n3));
    CL_LAUNCH_CHECK();
    return 0;
}

}  // namespace claire
