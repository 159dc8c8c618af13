// Float64 reductions and float32 vector updates for PCG, the objective and
// the line search. Reductions are deterministic: a fixed grid writes one
// partial per block (wavefront shuffles, then LDS), and a single block folds
// the partials in a fixed order.

#include "internal.h"

#include <cfloat>

namespace claire {
namespace {

constexpr int kThreads = 256;
constexpr int kWave = 64;

enum RedOp { OP_SUM = 0, OP_MAX = 1, OP_MIN = 2 };

template <int OP>
__device__ __forceinline__ double combine(double a, double b) {
    if (OP == OP_SUM) return a + b;
    if (OP == OP_MAX) return fmax(a, b);
    return fmin(a, b);
}

template <int OP>
__device__ __forceinline__ double identity() {
    if (OP == OP_SUM) return 0.0;
    if (OP == OP_MAX) return -DBL_MAX;
    return DBL_MAX;
}

template <int OP>
__device__ double block_reduce(double v, double* sh) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = combine<OP>(v, __shfl_down(v, o, kWave));
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = sh[0];
        for (int w = 1; w < kThreads / kWave; ++w) r = combine<OP>(r, sh[w]);
        sh[0] = r;
    }
    __syncthreads();
    const double r = sh[0];
    __syncthreads();
    return r;
}

// KIND 0: sum a*b; 1: sum (a-b)^2; 2: max |a|; 3: sum a
template <int KIND>
__global__ __launch_bounds__(kThreads) void k_partial(const float* __restrict__ a,
                                                      const float* __restrict__ b, long long n,
                                                      double* __restrict__ partial) {
    __shared__ double sh[kThreads / kWave];
    constexpr int OP = (KIND == 2) ? OP_MAX : OP_SUM;
    double acc = identity<OP>();
    const long long stride = (long long)gridDim.x * kThreads;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        if (KIND == 0) acc += (double)a[i] * (double)b[i];
        else if (KIND == 1) { const double d = (double)a[i] - (double)b[i]; acc += d * d; }
        else if (KIND == 2) acc = fmax(acc, fabs((double)a[i]));
        else acc += (double)a[i];
    }
    acc = block_reduce<OP>(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// float64 array statistics: min, sum, max, count(<= 0) -> partial[4*block + q]
__global__ __launch_bounds__(kThreads) void k_partial_stats(const double* __restrict__ a,
                                                            long long n,
                                                            double* __restrict__ partial) {
    __shared__ double sh[kThreads / kWave];
    double mn = DBL_MAX, mx = -DBL_MAX, sm = 0.0, cnt = 0.0;
    const long long stride = (long long)gridDim.x * kThreads;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const double x = a[i];
        mn = fmin(mn, x);
        mx = fmax(mx, x);
        sm += x;
        cnt += (x <= 0.0) ? 1.0 : 0.0;
    }
    mn = block_reduce<OP_MIN>(mn, sh);
    sm = block_reduce<OP_SUM>(sm, sh);
    mx = block_reduce<OP_MAX>(mx, sh);
    cnt = block_reduce<OP_SUM>(cnt, sh);
    if (threadIdx.x == 0) {
        partial[4 * blockIdx.x + 0] = mn;
        partial[4 * blockIdx.x + 1] = sm;
        partial[4 * blockIdx.x + 2] = mx;
        partial[4 * blockIdx.x + 3] = cnt;
    }
}

// r -= kappa Hs over [3][n] (float4 lanes; n % 4 == 0), kappa from the
// device slots when pd.sc is set, with per-block max |r| and per-component
// sums of r -> partial[4 block + {0,1,2,3}]
__global__ __launch_bounds__(kThreads) void k_pcg_update(const float4* __restrict__ hs,
                                                         float4* __restrict__ r, float kappa,
                                                         long long n4,
                                                         double* __restrict__ partial,
                                                         PcgDev pd) {
    __shared__ double sh[kThreads / kWave];
    double mx = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (pd.sc) kappa = pcg_curv_ok(pd) ? (float)(pd.sc[pd.rz] / pd.sc[pd.shs]) : 0.f;
    const long long stride = (long long)gridDim.x * kThreads;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < 3 * n4; i += stride) {
        const float4 h = hs[i];
        float4 q = r[i];
        q.x = fmaf(-kappa, h.x, q.x); q.y = fmaf(-kappa, h.y, q.y);
        q.z = fmaf(-kappa, h.z, q.z); q.w = fmaf(-kappa, h.w, q.w);
        r[i] = q;
        mx = fmax(mx, (double)fmaxf(fmaxf(fabsf(q.x), fabsf(q.y)), fmaxf(fabsf(q.z), fabsf(q.w))));
        const double sum = (double)q.x + (double)q.y + (double)q.z + (double)q.w;
        if (i < n4) s0 += sum; else if (i < 2 * n4) s1 += sum; else s2 += sum;
    }
    mx = block_reduce<OP_MAX>(mx, sh);
    s0 = block_reduce<OP_SUM>(s0, sh);
    s1 = block_reduce<OP_SUM>(s1, sh);
    s2 = block_reduce<OP_SUM>(s2, sh);
    if (threadIdx.x == 0) {
        partial[4 * blockIdx.x + 0] = mx;
        partial[4 * blockIdx.x + 1] = s0;
        partial[4 * blockIdx.x + 2] = s1;
        partial[4 * blockIdx.x + 3] = s2;
    }
}

// fold nb partials (with element stride `stride`, offset `off`) into
// result[slot] on the device and, when given, into the mapped host mirror
// (the host reads it after a stream synchronisation, with no copy). One
// 1024-thread block: few dependent load rounds even for thousands of partials.
constexpr int kFoldThreads = 1024;
template <int OP>
__global__ __launch_bounds__(kFoldThreads) void k_fold(const double* __restrict__ partial,
                                                       int nb, int stride, int off,
                                                       double* __restrict__ result, int slot,
                                                       double* __restrict__ mirror) {
    __shared__ double sh[kFoldThreads / kWave];
    // four independent accumulators keep several loads in flight
    double acc[4] = {identity<OP>(), identity<OP>(), identity<OP>(), identity<OP>()};
    int i = threadIdx.x;
    for (; i + 3 * kFoldThreads < nb; i += 4 * kFoldThreads) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
            acc[u] = combine<OP>(acc[u], partial[(i + u * kFoldThreads) * stride + off]);
    }
    for (; i < nb; i += kFoldThreads) acc[0] = combine<OP>(acc[0], partial[i * stride + off]);
    double a = combine<OP>(combine<OP>(acc[0], acc[1]), combine<OP>(acc[2], acc[3]));
    for (int o = kWave / 2; o > 0; o >>= 1) a = combine<OP>(a, __shfl_down(a, o, kWave));
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = sh[0];
        for (int w = 1; w < kFoldThreads / kWave; ++w) r = combine<OP>(r, sh[w]);
        result[slot] = r;
        if (mirror) mirror[slot] = r;
    }
}

__global__ __launch_bounds__(kThreads) void k_axpy(const float* __restrict__ x,
                                                   float* __restrict__ y, float a, long long n) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) y[i] = fmaf(a, x[i], y[i]);
}

__global__ __launch_bounds__(kThreads) void k_xpby(const float* __restrict__ x,
                                                   float* __restrict__ y, float b, long long n) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) y[i] = fmaf(b, y[i], x[i]);
}

// PCG direction update with the previous direction s and the device
// scalars: v~ += kappa s, then s = z + mu s (n4 float4 groups, then the tail of
// n - 4 n4 floats); a no-op on a curvature that is not positive and finite.
__global__ __launch_bounds__(kThreads) void k_pcg_direction(const float4* __restrict__ z,
                                                            float4* __restrict__ sd,
                                                            float4* __restrict__ vt,
                                                            long long n4, long long n,
                                                            PcgDev pd) {
    if (!pcg_curv_ok(pd)) return;   // uniform over the grid
    const float kappa = (float)(pd.sc[pd.rz] / pd.sc[pd.shs]);
    const float mu = (float)(pd.sc[pd.rz_new] / pd.sc[pd.rz]);
    const long long stride = (long long)gridDim.x * kThreads;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride) {
        const float4 a = z[i];
        float4 v = sd[i], t = vt[i];
        t.x = fmaf(kappa, v.x, t.x); t.y = fmaf(kappa, v.y, t.y);
        t.z = fmaf(kappa, v.z, t.z); t.w = fmaf(kappa, v.w, t.w);
        v.x = fmaf(mu, v.x, a.x);
        v.y = fmaf(mu, v.y, a.y);
        v.z = fmaf(mu, v.z, a.z);
        v.w = fmaf(mu, v.w, a.w);
        vt[i] = t;
        sd[i] = v;
    }
    const float* zs = reinterpret_cast<const float*>(z);
    float* ss = reinterpret_cast<float*>(sd);
    float* ts = reinterpret_cast<float*>(vt);
    for (long long i = 4 * n4 + (long long)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += stride) {
        ts[i] = fmaf(kappa, ss[i], ts[i]);
        ss[i] = fmaf(mu, ss[i], zs[i]);
    }
}

__global__ __launch_bounds__(kThreads) void k_lincomb(const float* __restrict__ x,
                                                      const float* __restrict__ z,
                                                      float* __restrict__ y, float b,
                                                      long long n) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) y[i] = fmaf(b, z[i], x[i]);
}

// als_a = (r_a - mean_a) + mu als_a for the three components of a vector field
// (with pd.sc: mu and the means from the device slots, a no-op on a bad curvature)
__device__ __forceinline__ bool als_scalars(const PcgDev& pd, float& m0, float& m1, float& m2,
                                            float& mu) {
    return !pd.sc || pcg_als_scalars(pd, m0, m1, m2, mu);
}

__global__ __launch_bounds__(kThreads) void k_als_update(const float* __restrict__ r,
                                                         float* __restrict__ als, float m0,
                                                         float m1, float m2, float mu,
                                                         long long n, PcgDev pd) {
    if (!als_scalars(pd, m0, m1, m2, mu)) return;
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= 3 * n) return;
    const float mean = (i < n) ? m0 : (i < 2 * n ? m1 : m2);
    als[i] = fmaf(mu, als[i], r[i] - mean);
}

// 16-byte variants of xpby, the als update and fill for aligned vectors
// whose length is a multiple of 4 (every field here: n3 >= 8); grid-stride.
__global__ __launch_bounds__(kThreads) void k_xpby4(const float4* __restrict__ x,
                                                    float4* __restrict__ y, float b,
                                                    long long n4) {
    const long long stride = (long long)gridDim.x * kThreads;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride) {
        const float4 a = x[i];
        float4 v = y[i];
        v.x = fmaf(b, v.x, a.x);
        v.y = fmaf(b, v.y, a.y);
        v.z = fmaf(b, v.z, a.z);
        v.w = fmaf(b, v.w, a.w);
        y[i] = v;
    }
}

__global__ __launch_bounds__(kThreads) void k_als_update4(const float4* __restrict__ r,
                                                          float4* __restrict__ als, float m0,
                                                          float m1, float m2, float mu,
                                                          long long n4, PcgDev pd) {
    if (!als_scalars(pd, m0, m1, m2, mu)) return;
    const long long stride = (long long)gridDim.x * kThreads;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < 3 * n4; i += stride) {
        const float mean = (i < n4) ? m0 : (i < 2 * n4 ? m1 : m2);
        const float4 a = r[i];
        float4 v = als[i];
        v.x = fmaf(mu, v.x, a.x - mean);
        v.y = fmaf(mu, v.y, a.y - mean);
        v.z = fmaf(mu, v.z, a.z - mean);
        v.w = fmaf(mu, v.w, a.w - mean);
        als[i] = v;
    }
}

__global__ __launch_bounds__(kThreads) void k_fill4(float4* __restrict__ y, float v,
                                                    long long n4) {
    const long long stride = (long long)gridDim.x * kThreads;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride)
        y[i] = make_float4(v, v, v, v);
}

__global__ __launch_bounds__(kThreads) void k_fill(float* __restrict__ y, float v, long long n) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) y[i] = v;
}

// y = a x: 16-byte accesses over the first 4 floor(n/4) elements, then the
// tail (the pointers are 16-byte aligned, checked by the launcher)
__global__ __launch_bounds__(kThreads) void k_scale_copy(const float4* __restrict__ x,
                                                         float4* __restrict__ y, float a,
                                                         long long n4, long long n) {
    const long long stride = (long long)gridDim.x * kThreads;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride) {
        const float4 v = x[i];
        y[i] = make_float4(a * v.x, a * v.y, a * v.z, a * v.w);
    }
    const float* xs = reinterpret_cast<const float*>(x);
    float* ys = reinterpret_cast<float*>(y);
    for (long long i = 4 * n4 + (long long)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += stride)
        ys[i] = a * xs[i];
}

__global__ __launch_bounds__(kThreads) void k_finite(const float* __restrict__ x, long long n,
                                                     int* __restrict__ flag) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n && !isfinite(x[i])) *flag = 1;
}

unsigned blocks_for(long long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

unsigned red_blocks(long long n) {
    long long b = (n + kThreads - 1) / kThreads;
    if (b > kRedBlocks) b = kRedBlocks;
    if (b < 1) b = 1;
    return (unsigned)b;
}

template <int KIND>
int red_generic(Reducer& r, const float* a, const float* b, long long n, int slot, hipStream_t s) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_partial<KIND>, dim3(nb), dim3(kThreads), 0, s, a, b, n, r.partial);
    CL_LAUNCH_CHECK();
    constexpr int OP = (KIND == 2) ? OP_MAX : OP_SUM;
    hipLaunchKernelGGL(k_fold<OP>, dim3(1), dim3(kFoldThreads), 0, s, r.partial, (int)nb, 1, 0,
                       r.result, slot, r.mirror);
    CL_LAUNCH_CHECK();
    return 0;
}

}  // namespace

int reducer_init(Reducer& r, long long n) {
    long long np = (long long)kRedBlocks * 4;
    if ((n + kThreads - 1) / kThreads > np) np = (n + kThreads - 1) / kThreads;
    CL_HIP(hipMalloc(&r.partial, sizeof(double) * np));
    CL_HIP(hipMalloc(&r.result, sizeof(double) * 8));
    // pinned, mapped, coherent: the folds store their results here as well
    CL_HIP(hipHostMalloc(&r.host, sizeof(double) * 8,
                         hipHostMallocMapped | hipHostMallocCoherent));
    CL_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&r.mirror), r.host, 0));
    return 0;
}

void reducer_free(Reducer& r) {
    if (r.partial) (void)hipFree(r.partial);
    if (r.result) (void)hipFree(r.result);
    if (r.host) (void)hipHostFree(r.host);
    r = Reducer();
}

int red_dot(Reducer& r, const float* a, const float* b, long long n, int slot, hipStream_t s) {
    return red_generic<0>(r, a, b, n, slot, s);
}

int red_sumsq_diff(Reducer& r, const float* a, const float* b, long long n, int slot,
                   hipStream_t s) {
    return red_generic<1>(r, a, b, n, slot, s);
}

int red_absmax(Reducer& r, const float* a, long long n, int slot, hipStream_t s) {
    return red_generic<2>(r, a, a, n, slot, s);
}

int red_sum(Reducer& r, const float* a, long long n, int slot, hipStream_t s) {
    return red_generic<3>(r, a, a, n, slot, s);
}

int red_stats_f64(Reducer& r, const double* a, long long n, hipStream_t s) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_partial_stats, dim3(nb), dim3(kThreads), 0, s, a, n, r.partial);
    CL_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_fold<OP_MIN>, dim3(1), dim3(kFoldThreads), 0, s, r.partial, (int)nb, 4, 0, r.result, 0, r.mirror);
    hipLaunchKernelGGL(k_fold<OP_SUM>, dim3(1), dim3(kFoldThreads), 0, s, r.partial, (int)nb, 4, 1, r.result, 1, r.mirror);
    hipLaunchKernelGGL(k_fold<OP_MAX>, dim3(1), dim3(kFoldThreads), 0, s, r.partial, (int)nb, 4, 2, r.result, 2, r.mirror);
    hipLaunchKernelGGL(k_fold<OP_SUM>, dim3(1), dim3(kFoldThreads), 0, s, r.partial, (int)nb, 4, 3, r.result, 3, r.mirror);
    CL_LAUNCH_CHECK();
    return 0;
}

int red_fold_sum(Reducer& r, int nb, int stride, int off, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_fold<OP_SUM>, dim3(1), dim3(kFoldThreads), 0, s, r.partial, nb, stride, off,
                       r.result, slot, r.mirror);
    CL_LAUNCH_CHECK();
    return 0;
}

static int pcg_update_impl(Reducer& red, const float* hs, float* r, float kappa,
                           const PcgDev& pd, long long n, int smax, int ssum, hipStream_t st) {
    const long long n4 = n / 4;
    unsigned nb = red_blocks(3 * n4);
    hipLaunchKernelGGL(k_pcg_update, dim3(nb), dim3(kThreads), 0, st,
                       reinterpret_cast<const float4*>(hs), reinterpret_cast<float4*>(r), kappa,
                       n4, red.partial, pd);
    CL_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_fold<OP_MAX>, dim3(1), dim3(kFoldThreads), 0, st, red.partial, (int)nb, 4, 0,
                       red.result, smax, red.mirror);
    for (int a = 0; a < 3; ++a)
        hipLaunchKernelGGL(k_fold<OP_SUM>, dim3(1), dim3(kFoldThreads), 0, st, red.partial, (int)nb, 4,
                           1 + a, red.result, ssum + a, red.mirror);
    CL_LAUNCH_CHECK();
    return 0;
}

int pcg_update(Reducer& red, const float* hs, float* r, float kappa, long long n, int smax,
               int ssum, hipStream_t st) {
    return pcg_update_impl(red, hs, r, kappa, PcgDev(), n, smax, ssum, st);
}

int pcg_update_dev(Reducer& red, const float* hs, float* r, const PcgDev& pd, long long n,
                   int smax, int ssum, hipStream_t st) {
    return pcg_update_impl(red, hs, r, 0.f, pd, n, smax, ssum, st);
}

// every fold also wrote its slot to the mapped host mirror r.host: waiting
// for the stream is enough
int red_fetch(Reducer& r, hipStream_t s) {
    CL_HIP(hipStreamSynchronize(s));
    return 0;
}

int launch_axpy(const float* x, float* y, float a, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n)), dim3(kThreads), 0, s, x, y, a, n);
    CL_LAUNCH_CHECK();
    return 0;
}

// true when both pointers are 16-byte aligned and n is a multiple of 4
static bool vec4(const void* a, const void* b, long long n) {
    return ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15u) == 0 &&
           (n & 3) == 0;
}

int launch_xpby(const float* x, float* y, float b, long long n, hipStream_t s) {
    if (vec4(x, y, n))
        hipLaunchKernelGGL(k_xpby4, dim3(red_blocks(n)), dim3(kThreads), 0, s,
                           reinterpret_cast<const float4*>(x), reinterpret_cast<float4*>(y), b,
                           n / 4);
    else
        hipLaunchKernelGGL(k_xpby, dim3(blocks_for(n)), dim3(kThreads), 0, s, x, y, b, n);
    CL_LAUNCH_CHECK();
    return 0;
}

int launch_pcg_direction_dev(const float* z, float* sd, float* vt, const PcgDev& pd,
                             long long n, hipStream_t s) {
    if ((reinterpret_cast<uintptr_t>(z) | reinterpret_cast<uintptr_t>(sd) |
         reinterpret_cast<uintptr_t>(vt)) & 15u) {
        set_error("pcg direction update needs 16-byte aligned vectors");
        return CLAIRE_EINVAL;
    }
    hipLaunchKernelGGL(k_pcg_direction, dim3(red_blocks(n)), dim3(kThreads), 0, s,
                       reinterpret_cast<const float4*>(z), reinterpret_cast<float4*>(sd),
                       reinterpret_cast<float4*>(vt), n / 4, n, pd);
    CL_LAUNCH_CHECK();
    return 0;
}

int launch_lincomb(const float* x, const float* z, float* y, float b, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_lincomb, dim3(blocks_for(n)), dim3(kThreads), 0, s, x, z, y, b, n);
    CL_LAUNCH_CHECK();
    return 0;
}

static int als_update_impl(const float* r, float* als, const double mean[3], float mu,
                           const PcgDev& pd, long long n, hipStream_t s) {
    if (vec4(r, als, n))
        hipLaunchKernelGGL(k_als_update4, dim3(red_blocks(3 * n)), dim3(kThreads), 0, s,
                           reinterpret_cast<const float4*>(r), reinterpret_cast<float4*>(als),
                           (float)mean[0], (float)mean[1], (float)mean[2], mu, n / 4, pd);
    else
        hipLaunchKernelGGL(k_als_update, dim3(blocks_for(3 * n)), dim3(kThreads), 0, s, r, als,
                           (float)mean[0], (float)mean[1], (float)mean[2], mu, n, pd);
    CL_LAUNCH_CHECK();
    return 0;
}

int launch_als_update(const float* r, float* als, const double mean[3], float mu, long long n,
                      hipStream_t s) {
    return als_update_impl(r, als, mean, mu, PcgDev(), n, s);
}

int launch_als_update_dev(const float* r, float* als, const PcgDev& pd, long long n,
                          hipStream_t s) {
    const double none[3] = {0.0, 0.0, 0.0};
    return als_update_impl(r, als, none, 0.f, pd, n, s);
}

int launch_fill(float* y, float value, long long n, hipStream_t s) {
    if (vec4(y, y, n))
        hipLaunchKernelGGL(k_fill4, dim3(red_blocks(n)), dim3(kThreads), 0, s,
                           reinterpret_cast<float4*>(y), value, n / 4);
    else
        hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kThreads), 0, s, y, value, n);
    CL_LAUNCH_CHECK();
    return 0;
}

int launch_scale_copy(const float* x, float* y, float a, long long n, hipStream_t s) {
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15) {
        set_error("scale_copy: pointers must be 16-byte aligned");
        return CLAIRE_EINVAL;
    }
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_scale_copy, dim3(nb), dim3(kThreads), 0, s,
                       reinterpret_cast<const float4*>(x), reinterpret_cast<float4*>(y), a, n / 4,
                       n);
    CL_LAUNCH_CHECK();
    return 0;
}

int launch_check_finite(const float* x, long long n, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_finite, dim3(blocks_for(n)), dim3(kThreads), 0, s, x, n, flag);
    CL_LAUNCH_CHECK();
    return 0;
}

}  // namespace claire
