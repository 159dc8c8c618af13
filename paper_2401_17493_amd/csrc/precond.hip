// Two-level zero-velocity preconditioner of the reduced Hessian (Section
// 2.5.6), in the original variables so that PCG keeps its residual and
// stopping rule:
//
//   P r = R^{-1/2} [ Q_P F_L K0_c^{-1} Q_R F_L + F_H ] R^{-1/2} r,
//
// R = alpha L with the k = 0 mode replaced by one, F_L / F_H cut-off filters
// below / above the Nyquist of the grid of half the extents, Q_R / Q_P
// spectral restriction and prolongation, and K0_c the coarse discretisation
// of R^{-1/2} H0 R^{-1/2}, H0 = alpha L + grad m (x) grad m at the current
// state m(t = 1) (the zero-velocity approximation, moved to the current
// iterate):
//
//   K0_c w = w - mean(w) + R_c^{-1/2} [ g (g . R_c^{-1/2} w) ],  g = Q_R F_L grad m(1),
//
// inverted by CG to a relative tolerance. One application costs one fine
// forward and one fine inverse transform (as the regularisation
// preconditioner does) plus coarse transforms and the inner iterations. In
// spectral space the fine passes are fused with the transfer: the restricted
// right-hand side is sigma R^/n on the kept modes, and the result is
// sigma S_L^/n_c on the kept modes and sigma^2 R^/n on the others
// (sigma = (alpha |k|^{2p})^{-1/2}).

#include "internal.h"

namespace claire {
namespace {

constexpr int kThreads = 256;

unsigned blocks(long long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// y_a <- g_a (g . y) in place (the data term of H0 at one voxel)
__global__ __launch_bounds__(kThreads) void k_h0_data(const float* __restrict__ g, float* y,
                                                      long long n) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const float g0 = g[i], g1 = g[n + i], g2 = g[2 * n + i];
    const float t = g0 * y[i] + g1 * y[n + i] + g2 * y[2 * n + i];
    y[i] = g0 * t;
    y[n + i] = g1 * t;
    y[2 * n + i] = g2 * t;
}

// q_a <- q_a + p_a - sum(p_a) / n
__global__ __launch_bounds__(kThreads) void k_k0_finish(const float* __restrict__ p, float* q,
                                                        const double* __restrict__ sums,
                                                        long long n) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const double inv = 1.0 / (double)n;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long j = a * n + i;
        q[j] = q[j] + (p[j] - (float)(sums[a] * inv));
    }
}

// CG step with the step length formed on the device: a = rr / <p, q>;
// x += a p, r -= a q; the block's share of <r, r> -> partial[block]
__global__ __launch_bounds__(kThreads) void k_cg_step(float* __restrict__ x, float* __restrict__ r,
                                                      const float* __restrict__ p,
                                                      const float* __restrict__ q, double rr,
                                                      const double* __restrict__ pq,
                                                      long long n3, double* __restrict__ partial) {
    __shared__ double sh[4];
    const float a = (float)(rr / *pq);
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n3;
         i += (long long)gridDim.x * kThreads) {
        x[i] += a * p[i];
        const float ri = r[i] - a * q[i];
        r[i] = ri;
        acc += (double)ri * ri;
    }
    const double t = block_sum_256(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

}  // namespace

int twolevel_init(TwoLevel& T, const Geo& gf) {
    if (T.ready) return 0;
    const int nc[3] = {gf.n1 / 2, gf.n2 / 2, gf.n3 / 2};
    if (check_extents(nc) != 0) {
        set_error("the two-level preconditioner's coarse grid %dx%dx%d (half the extents) is "
                  "not a supported grid: every extent >= 16 and n1/2, n2/2 even needed",
                  nc[0], nc[1], nc[2]);
        return CLAIRE_EINVAL;
    }
    T.gc = make_geo(nc);
    CL_TRY(spectral_init(T.swc, T.gc));
    const long long n3 = 3 * T.gc.n;
    float** bufs[] = {&T.gm, &T.b, &T.x, &T.r, &T.p, &T.q, &T.y};
    for (float** b : bufs) CL_HIP(hipMalloc(reinterpret_cast<void**>(b), sizeof(float) * n3));
    CL_TRY(reducer_init(T.red, n3));
    T.ready = true;
    return 0;
}

void twolevel_free(TwoLevel& T) {
    float* bufs[] = {T.gm, T.b, T.x, T.r, T.p, T.q, T.y};
    for (float* b : bufs)
        if (b) (void)hipFree(b);
    if (T.ready) {
        spectral_free(T.swc);
        reducer_free(T.red);
    }
    T = TwoLevel();
}

int twolevel_setup(TwoLevel& T, const Geo& gf, SpectralWork& swf, const float* gradm,
                   hipStream_t s) {
    CL_TRY(spectral_forward(gf, swf, gradm, swf.spec, 3, s));
    CL_TRY(spectral_restrict_modes(gf, T.gc, swf.spec, T.swc.spec, 3, 0.0, 1, false, s));
    return spectral_inverse(T.gc, T.swc, T.swc.spec, T.gm, 3, s);
}

// q = K0_c p
static int k0_apply(TwoLevel& T, const float* p, float* q, double alpha, int pw, hipStream_t s) {
    const Geo& g = T.gc;
    const long long n = g.n;
    CL_TRY(spectral_apply(g, T.swc, SPEC_REG_ISQRT, p, T.y, alpha, pw, s));
    hipLaunchKernelGGL(k_h0_data, dim3(blocks(n)), dim3(kThreads), 0, s, T.gm, T.y, n);
    CL_LAUNCH_CHECK();
    CL_TRY(spectral_apply(g, T.swc, SPEC_REG_ISQRT, T.y, q, alpha, pw, s));
    for (int a = 0; a < 3; ++a) CL_TRY(red_sum(T.red, p + a * n, n, a, s));
    hipLaunchKernelGGL(k_k0_finish, dim3(blocks(n)), dim3(kThreads), 0, s, p, q, T.red.result, n);
    CL_LAUNCH_CHECK();
    return 0;
}

int twolevel_apply(TwoLevel& T, const Geo& gf, SpectralWork& swf, const float* r, float* z,
                   double alpha, int pw, double inner_rtol, int max_inner, int* inner_its,
                   hipStream_t s) {
    const Geo& gc = T.gc;
    const long long n3 = 3 * gc.n;
    // right-hand side sigma R^ / n on the kept modes, on the coarse grid
    CL_TRY(spectral_forward(gf, swf, r, swf.spec, 3, s));
    CL_TRY(spectral_restrict_modes(gf, gc, swf.spec, T.swc.spec, 3, alpha, pw, true, s));
    // the fine spectrum stays in swf.spec: the coarse transforms use T.swc
    CL_TRY(spectral_inverse(gc, T.swc, T.swc.spec, T.b, 3, s));
    // CG on K0_c x = b from x = 0
    CL_TRY(launch_fill(T.x, 0.f, n3, s));
    CL_HIP(hipMemcpyAsync(T.r, T.b, sizeof(float) * n3, hipMemcpyDeviceToDevice, s));
    CL_HIP(hipMemcpyAsync(T.p, T.b, sizeof(float) * n3, hipMemcpyDeviceToDevice, s));
    CL_TRY(red_dot(T.red, T.r, T.r, n3, 4, s));
    CL_TRY(red_fetch(T.red, s));
    double rr = T.red.host[4];
    const double stop = inner_rtol * inner_rtol * rr;
    int its = 0;
    const int nb = (int)std::min<long long>(kRedBlocks, blocks(n3));
    while (its < max_inner && rr > stop && rr > 0.0) {
        CL_TRY(k0_apply(T, T.p, T.q, alpha, pw, s));
        CL_TRY(red_dot(T.red, T.p, T.q, n3, 3, s));
        hipLaunchKernelGGL(k_cg_step, dim3(nb), dim3(kThreads), 0, s, T.x, T.r, T.p, T.q, rr,
                           T.red.result + 3, n3, T.red.partial);
        CL_LAUNCH_CHECK();
        CL_TRY(red_fold_sum(T.red, nb, 1, 0, 5, s));
        CL_TRY(red_fetch(T.red, s));
        ++its;
        if (!(T.red.host[3] > 0.0)) {
            set_error("coarse H0 curvature %g is not positive", T.red.host[3]);
            return CLAIRE_ENONFINITE;
        }
        const double rr_new = T.red.host[5];
        if (!std::isfinite(rr_new)) {
            set_error("coarse CG residual is not finite");
            return CLAIRE_ENONFINITE;
        }
        if (rr_new <= stop) { rr = rr_new; break; }
        CL_TRY(launch_xpby(T.r, T.p, (float)(rr_new / rr), n3, s));   // p = r + beta p
        rr = rr_new;
    }
    if (inner_its) *inner_its = its;
    // back to the fine grid: sigma S_L^ / n_c on the kept modes, sigma^2 R^ / n elsewhere
    CL_TRY(spectral_forward(gc, T.swc, T.x, T.swc.spec, 3, s));
    CL_TRY(spectral_combine_modes(gf, gc, swf.spec, T.swc.spec, 3, alpha, pw, s));
    return spectral_inverse(gf, swf, swf.spec, z, 3, s);
}

}  // namespace claire
