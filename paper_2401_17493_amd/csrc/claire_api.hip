// Context, Gauss--Newton--Krylov driver and the exported C ABI.
//
// Per-velocity setup (Algorithm 1 lines 3-6), Hessian matvec (eq. e:matvec,
// Gauss--Newton form), PCG (Algorithm 2) with the regularisation
// preconditioner (Section 2.5.6), Armijo line search and parameter
// continuation (Sections 2.5.5, 2.6). All field work runs in the HIP kernels
// of fft.hip, sl.hip and blas.hip; this file only sequences them and makes
// the scalar decisions (step lengths, stopping tests) in float64 on the host.

#include "internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

namespace claire {

namespace {
thread_local char g_err[1024] = "";
}

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
    set_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? CLAIRE_ENOMEM
                                                                       : CLAIRE_EDEVICE;
}

namespace {
bool pow2(int v) { return v >= 8 && v <= 1024 && (v & (v - 1)) == 0; }

// even, in [8, 1024], no prime factor other than 2, 3 and 5
bool smooth_even(int v) {
    if (v < 8 || v > 1024 || (v & 1)) return false;
    for (int f : {2, 3, 5})
        while (v % f == 0) v /= f;
    return v == 1;
}
}  // namespace

int check_extents(const int nx[3]) {
    if (!pow2(nx[2])) {
        set_error("n3 = %d: the contiguous extent must be a power of two in [8, 1024]", nx[2]);
        return CLAIRE_EINVAL;
    }
    for (int a = 0; a < 2; ++a)
        if (!smooth_even(nx[a])) {
            set_error("n%d = %d: must be an even product of 2, 3 and 5 in [8, 1024]", a + 1,
                      nx[a]);
            return CLAIRE_EINVAL;
        }
    return 0;
}

Geo make_geo(const int nx[3]) {
    Geo g;
    g.n1 = nx[0];
    g.n2 = nx[1];
    g.n3 = nx[2];
    auto lg = [](int v) { int l = 0; while ((1 << l) < v) ++l; return l; };
    g.l1 = lg(g.n1);
    g.l2 = lg(g.n2);
    g.l3 = lg(g.n3);
    g.nh = g.n3 / 2 + 1;
    g.hp = spec_pitch(g.nh);
    g.n = (long long)g.n1 * g.n2 * g.n3;
    g.nspec = (long long)g.n1 * g.n2 * g.hp;
    g.pow2 = (1 << g.l1) == g.n1 && (1 << g.l2) == g.n2 && (1 << g.l3) == g.n3;
    return g;
}

}  // namespace claire

using namespace claire;

struct claire_ctx {
    Geo g;
    int nt = 0;
    double alpha = 0;
    int p = 1;
    hipStream_t s = nullptr;
    // side stream (default priority) on which a standalone Hessian matvec runs
    // the FFTs of alpha L v~ while the main stream runs the gathers; forked
    // and joined with the two events
    hipStream_t s2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_pcg = nullptr;   // after a PCG iteration's preconditioner
    std::vector<hipEvent_t> ev_state;   // [nt + 1]: state m^j written (setup overlap)
    double cell = 0;   // h1 h2 h3

    // per-velocity state
    float* m0 = nullptr;     // [n]
    float* m1 = nullptr;     // [n]
    float* v = nullptr;      // [3][n]
    float* dp = nullptr;     // [3][n] departure displacement of +v (voxels)
    float* dm = nullptr;     // [3][n] departure displacement of -v
    float* m = nullptr;      // [nt+1][n]   m^j
    float* gm = nullptr;     // [nt+1][3][n] grad m^j
    float* divv = nullptr;   // [n]
    float* A = nullptr;      // [n] adjoint step factor
    float* grad = nullptr;   // [3][n] reduced gradient
    float* regv = nullptr;   // [3][n] alpha L v
    float* lam = nullptr;    // [nt+1][n] adjoint / incremental adjoint
    float* w0 = nullptr;     // [n] incremental-state ping-pong
    float* w1 = nullptr;     // [n]
    float* tmp3 = nullptr;   // [3][n]
    int* box_p = nullptr;    // per-brick stencil boxes of dp
    int* box_m = nullptr;    // per-brick stencil boxes of dm

    // mixed precision (half storage in the Hessian matvec), allocated on demand
    int precision = 0;       // 0 float32, 1 mixed
    __half* gm16 = nullptr;  // [nt+1][3][n] grad m^j
    bool half_valid = false; // gm16 belongs to the current setup
    SpectralWork sw;
    Reducer red;
    TwoLevel tl;             // two-level preconditioner, allocated on first use
    int* flag = nullptr;     // device int (non-finite check)

    // solver vectors (allocated on first solve)
    float* vt = nullptr;
    float* r = nullptr;
    float* z = nullptr;
    float* sd = nullptr;
    float* hs = nullptr;
    float* vtrial = nullptr;
    float* als = nullptr;    // alpha L s, kept by recursion inside PCG

    // near-incompressible model (beta > 0), buffers allocated on demand
    double beta = 0;
    float* ni_tmp = nullptr; // [3][n] data term int lambda grad m dt before projection
    float* gradJ = nullptr;  // [3][n] L2 gradient of J (Armijo slope)
    double Jdiv = 0;         // divergence penalty part of J

    int deriv = CLAIRE_DERIV_SPECTRAL;   // first-derivative discretisation
    bool have_images = false;
    bool state_valid = false;      // dp, dm, m valid for the content of v
    bool gm0_valid = false;        // gm slot 0 holds grad m0 (independent of v)
    bool have_velocity = false;    // full setup done: gm, A, g, J valid
    double J = 0, Jdist = 0, Jreg = 0, gnorm = 0;

    // trace of the last solve (host): kTraceWidth values per visited iterate
    // (level, k, J, ||g||_inf, PCG matvecs, step length, line-search trials,
    // residual values recorded) and the concatenated PCG residual histories
    // ||r_l||_inf
    std::vector<double> trace_iters;
    std::vector<double> trace_res;
};

namespace {

template <typename T>
int dalloc(T** p, long long count) {
    CL_HIP(hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)count));
    return 0;
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

int check_args(const int nx[3], int nt, double alpha, int reg_order) {
    if (!nx) { set_error("nx is NULL"); return CLAIRE_EINVAL; }
    CL_TRY(check_extents(nx));
    if (nt < 1 || nt > 64) { set_error("nt = %d out of range [1, 64]", nt); return CLAIRE_EINVAL; }
    if (!(alpha > 0.0) || !std::isfinite(alpha)) { set_error("alpha must be positive"); return CLAIRE_EINVAL; }
    if (reg_order != 1 && reg_order != 2) { set_error("reg_order must be 1 or 2"); return CLAIRE_EINVAL; }
    return 0;
}

int ctx_alloc(claire_ctx* c) {
    const long long n = c->g.n;
    const int nt = c->nt;
    CL_TRY(dalloc(&c->m0, n));
    CL_TRY(dalloc(&c->m1, n));
    CL_TRY(dalloc(&c->v, 3 * n));
    CL_TRY(dalloc(&c->dp, 3 * n));
    CL_TRY(dalloc(&c->dm, 3 * n));
    CL_TRY(dalloc(&c->m, (nt + 1) * n));
    CL_TRY(dalloc(&c->gm, 3 * (nt + 1) * n));
    CL_TRY(dalloc(&c->divv, n));
    CL_TRY(dalloc(&c->A, n));
    CL_TRY(dalloc(&c->grad, 3 * n));
    CL_TRY(dalloc(&c->regv, 3 * n));
    CL_TRY(dalloc(&c->lam, (nt + 1) * n));
    CL_TRY(dalloc(&c->w0, n));
    CL_TRY(dalloc(&c->w1, n));
    CL_TRY(dalloc(&c->tmp3, 3 * n));
    CL_TRY(dalloc(&c->flag, 1));
    CL_TRY(dalloc(&c->box_p, brick_table_ints(c->g)));
    CL_TRY(dalloc(&c->box_m, brick_table_ints(c->g)));
    CL_TRY(spectral_init(c->sw, c->g));
    CL_TRY(reducer_init(c->red, c->g.n));
    CL_HIP(hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking));
    CL_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    CL_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    CL_HIP(hipEventCreateWithFlags(&c->ev_pcg, hipEventDisableTiming));
    c->ev_state.assign(c->nt + 1, nullptr);
    for (auto& e : c->ev_state) CL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return 0;
}

void ctx_release(claire_ctx* c) {
    float* bufs[] = {c->m0, c->m1, c->v, c->dp, c->dm, c->m, c->gm, c->divv, c->A, c->grad,
                     c->regv, c->lam, c->w0, c->w1, c->tmp3, c->vt, c->r, c->z, c->sd, c->hs,
                     c->vtrial, c->als, c->ni_tmp, c->gradJ};
    for (float* b : bufs) dfree(b);
    dfree(c->gm16);
    dfree(c->flag);
    dfree(c->box_p);
    dfree(c->box_m);
    spectral_free(c->sw);
    reducer_free(c->red);
    twolevel_free(c->tl);
    if (c->s2) {
        (void)hipStreamSynchronize(c->s2);
        (void)hipStreamDestroy(c->s2);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->ev_pcg) (void)hipEventDestroy(c->ev_pcg);
    for (hipEvent_t e : c->ev_state)
        if (e) (void)hipEventDestroy(e);
}

int copy_d2d(float* dst, const float* src, long long count, hipStream_t s) {
    if (dst == src) return 0;
    CL_HIP(hipMemcpyAsync(dst, src, sizeof(float) * (size_t)count, hipMemcpyDeviceToDevice, s));
    return 0;
}

// First derivatives with the context's discretisation (Section 2.5.3), on
// stream st.
int ctx_grad(claire_ctx* c, const float* u, float* out, hipStream_t st) {
    if (c->deriv == CLAIRE_DERIV_FD8) return launch_fd8_grad(c->g, u, out, st);
    return spectral_apply(c->g, c->sw, SPEC_GRAD, u, out, c->alpha, c->p, st);
}
int ctx_div(claire_ctx* c, const float* v, float* out, hipStream_t st) {
    if (c->deriv == CLAIRE_DERIV_FD8) return launch_fd8_div(c->g, v, out, st);
    return spectral_apply(c->g, c->sw, SPEC_DIV, v, out, c->alpha, c->p, st);
}

// grad m^j on the side stream once the main stream has written m^j
int side_grad(claire_ctx* c, int j) {
    const long long n = c->g.n;
    CL_HIP(hipEventRecord(c->ev_state[j], c->s));
    CL_HIP(hipStreamWaitEvent(c->s2, c->ev_state[j], 0));
    return ctx_grad(c, c->m + (long long)j * n, c->gm + (long long)j * 3 * n, c->s2);
}

// Backtrace and state solve for the velocity held in c->v (Section 2.5.2,
// eq. e:transport): m^0 = m0, m^{j+1} = m^j(y+). grads_on_side: hand each
// new m^j to the side stream for its gradient (the setup's overlap).
int run_state(claire_ctx* c, bool grads_on_side = false) {
    const Geo& g = c->g;
    const double ht = 1.0 / c->nt;
    CL_TRY(launch_backtrace(g, c->v, c->dp, c->dm, ht, c->s));
    CL_TRY(launch_brick_boxes(g, c->dp, c->box_p, c->s));
    CL_TRY(launch_brick_boxes(g, c->dm, c->box_m, c->s));
    CL_TRY(copy_d2d(c->m, c->m0, g.n, c->s));
    for (int j = 0; j < c->nt; ++j) {
        CL_TRY(launch_interp(g, c->m + (long long)j * g.n, 1, c->dp, c->m + (long long)(j + 1) * g.n,
                             c->s, c->box_p));
        if (grads_on_side) CL_TRY(side_grad(c, j + 1));
    }
    c->state_valid = true;
    return 0;
}

int ensure_ni_buffers(claire_ctx* c) {
    if (!c->ni_tmp) CL_TRY(dalloc(&c->ni_tmp, 3 * c->g.n));
    if (!c->gradJ) CL_TRY(dalloc(&c->gradJ, 3 * c->g.n));
    return 0;
}

int ensure_half_buffers(claire_ctx* c) {
    const long long n = c->g.n;
    const int nt = c->nt;
    if (!c->gm16) CL_TRY(dalloc(&c->gm16, 3 * (nt + 1) * n));
    return 0;
}

// Full per-velocity setup; the state is reused when state_valid says the
// backtrace and m^j already belong to c->v (accepted line-search trial).

int run_setup(claire_ctx* c) {
    const Geo& g = c->g;
    const long long n = g.n;
    const int nt = c->nt;
    const double ht = 1.0 / nt;
    // The Fourier work runs on the side stream beside the state solve's
    // gathers: alpha L v, div v and grad m0 (which does not depend on v and is
    // kept across setups) at once, grad m^j (Section 2.5.3; stored, not
    // recomputed per matvec) as soon as m^j exists.
    CL_HIP(hipEventRecord(c->ev_fork, c->s));
    CL_HIP(hipStreamWaitEvent(c->s2, c->ev_fork, 0));
    CL_TRY(spectral_apply(g, c->sw, SPEC_REG, c->v, c->regv, c->alpha, c->p, c->s2));
    CL_TRY(ctx_div(c, c->v, c->divv, c->s2));
    if (!c->gm0_valid) {
        CL_TRY(ctx_grad(c, c->m0, c->gm, c->s2));
        c->gm0_valid = true;
    }
    if (!c->state_valid) {
        CL_TRY(run_state(c, true));
    } else {
        for (int j = 1; j <= nt; ++j)
            CL_TRY(ctx_grad(c, c->m + (long long)j * n, c->gm + (long long)j * 3 * n, c->s2));
    }
    CL_HIP(hipEventRecord(c->ev_join, c->s2));
    // objective parts: 1/2 ||m^nt - m1||^2 and 1/2 <alpha L v, v>
    CL_TRY(red_sumsq_diff(c->red, c->m + nt * n, c->m1, n, 0, c->s));
    CL_HIP(hipStreamWaitEvent(c->s, c->ev_join, 0));
    CL_TRY(red_dot(c->red, c->regv, c->v, 3 * n, 1, c->s));
    // the adjoint step factor
    CL_TRY(launch_make_A(g, c->divv, c->dm, c->A, ht, c->s, c->box_m));
    // adjoint (eq. e:adjoint): lam^nt = -(m^nt - m1), lam^j = A lam^{j+1}(y-)
    CL_TRY(launch_final_adjoint(g, c->m + nt * n, c->m1, c->lam + nt * n, c->s));
    for (int j = nt - 1; j >= 0; --j)
        CL_TRY(launch_adjoint_step(g, c->lam + (long long)(j + 1) * n, c->dm, c->A,
                                   c->lam + (long long)j * n, c->s, c->box_m));
    // half copies for the mixed-precision matvec
    c->half_valid = false;
    if (c->precision == 1) {
        CL_TRY(ensure_half_buffers(c));
        CL_TRY(launch_to_half(c->gm, c->gm16, 3 * (nt + 1) * n, c->s));
        c->half_valid = true;
    }
    // reduced gradient (eq. e:rgrad), trapezoid in time
    if (c->beta > 0.0) {
        // near-incompressible model (appendix): g = alpha L v + K b with
        // K = I - grad M Delta^{-1} div and b the data term; J gains the
        // divergence penalty 1/2 <P v, v>, P = -grad beta (-Delta^{-1} + id) div
        CL_TRY(ensure_ni_buffers(c));
        CL_TRY(launch_assemble(g, c->lam, c->gm, nt, nullptr, c->ni_tmp, c->s));
        CL_TRY(spectral_ni(g, c->sw, NI_PROJECT, c->ni_tmp, c->grad, c->alpha, c->beta, c->s,
                           c->regv));
        CL_TRY(spectral_ni(g, c->sw, NI_PENALTY, c->v, c->gradJ, c->alpha, c->beta, c->s,
                           nullptr, c->v, &c->red, 3));   // P v and <P v, v> -> slot 3
        // L2 gradient of J for the Armijo slope: b + alpha L v + P v
        CL_TRY(launch_axpy(c->ni_tmp, c->gradJ, 1.f, 3 * n, c->s));
        CL_TRY(launch_axpy(c->regv, c->gradJ, 1.f, 3 * n, c->s));
    } else {
        CL_TRY(launch_assemble(g, c->lam, c->gm, nt, c->regv, c->grad, c->s));
    }
    CL_TRY(red_absmax(c->red, c->grad, 3 * n, 2, c->s));
    CL_TRY(red_fetch(c->red, c->s));
    c->Jdist = 0.5 * c->cell * c->red.host[0];
    c->Jreg = 0.5 * c->cell * c->red.host[1];
    c->Jdiv = c->beta > 0.0 ? 0.5 * c->cell * c->red.host[3] : 0.0;
    c->J = c->Jdist + c->Jreg + c->Jdiv;
    c->gnorm = c->red.host[2];
    if (!std::isfinite(c->J) || !std::isfinite(c->gnorm)) {
        set_error("non-finite objective or gradient");
        c->have_velocity = false;
        return CLAIRE_ENONFINITE;
    }
    c->have_velocity = true;
    return 0;
}

// Gauss--Newton Hessian matvec (eqs. e:matvec, e:incstate, e:incadj).
// reg_part: alpha L vt when the caller already has it (PCG), else NULL and
// it is computed here by FFT (on the side stream, beside the gathers).
// dot_slot >= 0: also <vt, out> into that reduction slot.
int finish_ni_matvec(claire_ctx* c, const float* vt, float* out, const float* reg_part,
                     int dot_slot);

// alpha L v~ into tmp3 on the side stream, ordered after the work already
// enqueued on the main stream; join_reg() makes the main stream wait for it.
// The FFT passes are bound by HBM streaming, the gathers they overlap by the
// LDS and the VALU. Uses the spectral workspace, which the gathers do not.
int fork_reg(claire_ctx* c, const float* vt) {
    CL_HIP(hipEventRecord(c->ev_fork, c->s));
    CL_HIP(hipStreamWaitEvent(c->s2, c->ev_fork, 0));
    // the mixed matvec transforms in float32 (the gradient keeps SPEC_REG)
    const SpecMode mode = c->precision == 1 ? SPEC_REG32 : SPEC_REG;
    CL_TRY(spectral_apply(c->g, c->sw, mode, vt, c->tmp3, c->alpha, c->p, c->s2));
    CL_HIP(hipEventRecord(c->ev_join, c->s2));
    return 0;
}
int join_reg(claire_ctx* c) {
    CL_HIP(hipStreamWaitEvent(c->s, c->ev_join, 0));
    return 0;
}

// PCG direction update (v~ += kappa s, s = z + mu s, as k_pcg_direction)
// fused with the first incremental-state source of the next matvec,
// w0 = -(h_t/2) grad m^0 . s for the new s (as k_inc_first forms it: the
// product of component 1, then components 0 and 2 by fused multiply-adds,
// the order the compiler gives that kernel), so the matvec need not read s
// for it again. Four voxels per thread (n a multiple of 4); a no-op on a
// bad curvature.
namespace {
constexpr int kDirThreads = 256;
__device__ __forceinline__ float4 load4(const float* p) {
    return *reinterpret_cast<const float4*>(p);
}
__device__ __forceinline__ float4 load4(const __half* p) {
    const uint2 u = *reinterpret_cast<const uint2*>(p);
    const __half2 a = *reinterpret_cast<const __half2*>(&u.x);
    const __half2 b = *reinterpret_cast<const __half2*>(&u.y);
    return make_float4(__low2float(a), __high2float(a), __low2float(b), __high2float(b));
}
__device__ __forceinline__ float w0_of(float g0, float g1, float g2, float s0, float s1,
                                       float s2, float half_ht) {
    return -half_ht * fmaf(g2, s2, fmaf(g0, s0, g1 * s1));
}
template <typename GT>
__global__ __launch_bounds__(kDirThreads) void k_pcg_direction_w0(
    const float* __restrict__ z, float* __restrict__ sd, float* __restrict__ vt,
    const GT* __restrict__ gm0, float* __restrict__ w0, long long n, float half_ht, PcgDev pd) {
    if (!pcg_curv_ok(pd)) return;   // uniform over the grid
    const float kappa = (float)(pd.sc[pd.rz] / pd.sc[pd.shs]);
    const float mu = (float)(pd.sc[pd.rz_new] / pd.sc[pd.rz]);
    const long long stride = (long long)gridDim.x * kDirThreads * 4;
    for (long long i = ((long long)blockIdx.x * kDirThreads + threadIdx.x) * 4; i < n;
         i += stride) {
        float4 sn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float4 zz = load4(z + a * n + i);
            float4 v = load4(sd + a * n + i), t = load4(vt + a * n + i);
            t.x = fmaf(kappa, v.x, t.x); t.y = fmaf(kappa, v.y, t.y);
            t.z = fmaf(kappa, v.z, t.z); t.w = fmaf(kappa, v.w, t.w);
            v.x = fmaf(mu, v.x, zz.x); v.y = fmaf(mu, v.y, zz.y);
            v.z = fmaf(mu, v.z, zz.z); v.w = fmaf(mu, v.w, zz.w);
            *reinterpret_cast<float4*>(vt + a * n + i) = t;
            *reinterpret_cast<float4*>(sd + a * n + i) = v;
            sn[a] = v;
        }
        const float4 g0 = load4(gm0 + i), g1 = load4(gm0 + n + i), g2 = load4(gm0 + 2 * n + i);
        float4 w;
        w.x = w0_of(g0.x, g1.x, g2.x, sn[0].x, sn[1].x, sn[2].x, half_ht);
        w.y = w0_of(g0.y, g1.y, g2.y, sn[0].y, sn[1].y, sn[2].y, half_ht);
        w.z = w0_of(g0.z, g1.z, g2.z, sn[0].z, sn[1].z, sn[2].z, half_ht);
        w.w = w0_of(g0.w, g1.w, g2.w, sn[0].w, sn[1].w, sn[2].w, half_ht);
        *reinterpret_cast<float4*>(w0 + i) = w;
    }
}
}  // namespace

template <typename GT>
int launch_pcg_direction_w0(claire_ctx* c, const GT* gm0, const PcgDev& pd) {
    const long long n = c->g.n;
    long long nb = (n / 4 + kDirThreads - 1) / kDirThreads;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_pcg_direction_w0<GT>, dim3((unsigned)nb), dim3(kDirThreads), 0, c->s,
                       c->z, c->sd, c->vt, gm0, c->w0, n, (float)(0.5 / c->nt), pd);
    CL_LAUNCH_CHECK();
    return 0;
}

// GT: storage of grad m^j read by the matvec (float; __half in the mixed
// path, whose only difference is these 16-bit reads -- the sources
// f^j = -grad m^j . v~, the fields m~, lam~, A and the displacements stay
// float32, R23).
template <typename GT>
int matvec_steps(claire_ctx* c, const GT* gm, const float* vt, float* out,
                 const float* reg_part, int dot_slot, const PcgDev* als_pd, bool w0_ready) {
    const Geo& g = c->g;
    const long long n = g.n;
    const int nt = c->nt;
    const double ht = 1.0 / nt;
    const bool fork = !reg_part;
    if (fork) CL_TRY(fork_reg(c, vt));
    // incremental state, forward in time; the last step writes lambda~^nt = -m~^nt
    // (w0 may have been formed with the direction update that produced vt)
    if (!w0_ready) CL_TRY(launch_inc_state_first(g, gm, vt, c->w0, ht, c->s));
    float* src = c->w0;
    float* nxt = c->w1;
    for (int j = 0; j < nt; ++j) {
        const GT* gnext = gm + (long long)(j + 1) * 3 * n;
        if (j + 1 < nt) {
            CL_TRY(launch_inc_state_step(g, src, c->dp, gnext, vt, nxt, (float)ht, 1.0f, c->s,
                                         c->box_p));
            float* t = src;
            src = nxt;
            nxt = t;
        } else {
            CL_TRY(launch_inc_state_step(g, src, c->dp, gnext, vt, c->lam + (long long)nt * n,
                                         (float)(0.5 * ht), -1.0f, c->s, c->box_p));
        }
    }
    if (fork) {
        CL_TRY(join_reg(c));
        reg_part = c->tmp3;
    }
    // incremental adjoint (GN), backward in time, then
    // H v~ = alpha L v~ + h_t sum_j c_j lambda~^j grad m^j in one pass
    for (int j = nt - 1; j >= 0; --j)
        CL_TRY(launch_adjoint_step(g, c->lam + (long long)(j + 1) * n, c->dm, c->A,
                                   c->lam + (long long)j * n, c->s, c->box_m));
    if (c->beta > 0.0) {
        // near-incompressible model: the data term projected by K
        CL_TRY(launch_assemble(g, c->lam, gm, nt, (const float*)nullptr, c->ni_tmp, c->s));
        return finish_ni_matvec(c, vt, out, reg_part, dot_slot);
    }
    if (als_pd)   // reg_part is c->als, advanced inside the assembly
        return launch_assemble(g, c->lam, gm, nt, (const float*)nullptr, out, c->s, vt, &c->red,
                               dot_slot, als_pd, c->r, c->als);
    if (dot_slot >= 0)
        return launch_assemble(g, c->lam, gm, nt, reg_part, out, c->s, vt, &c->red, dot_slot);
    return launch_assemble(g, c->lam, gm, nt, reg_part, out, c->s);
}

// out = reg_part + K ni_tmp (near-incompressible projection of the data term
// in ni_tmp), and <vt, out> -> dot_slot when >= 0
int finish_ni_matvec(claire_ctx* c, const float* vt, float* out, const float* reg_part,
                     int dot_slot) {
    CL_TRY(spectral_ni(c->g, c->sw, NI_PROJECT, c->ni_tmp, out, c->alpha, c->beta, c->s,
                       reg_part));
    if (dot_slot >= 0) CL_TRY(red_dot(c->red, vt, out, 3 * c->g.n, dot_slot, c->s));
    return 0;
}

// als_pd (PCG, plain model): the assembly first advances the alpha L s
// recursion in reg_part (= c->als) with the device scalars of the previous
// iteration and the residual c->r
int run_matvec(claire_ctx* c, const float* vt, float* out, const float* reg_part = nullptr,
               int dot_slot = -1, const PcgDev* als_pd = nullptr, bool w0_ready = false) {
    if (als_pd && (c->beta > 0.0 || reg_part != c->als || dot_slot < 0)) {
        set_error("the als update rides only on the plain model's PCG matvec");
        return CLAIRE_EINVAL;
    }
    if (c->precision == 1)
        return matvec_steps(c, c->gm16, vt, out, reg_part, dot_slot, als_pd, w0_ready);
    return matvec_steps(c, c->gm, vt, out, reg_part, dot_slot, als_pd, w0_ready);
}

// Objective of a trial velocity held in c->v: backtrace, state, mismatch.
int run_trial_mismatch(claire_ctx* c, double* half_sumsq) {
    const long long n = c->g.n;
    c->state_valid = false;
    c->have_velocity = false;
    CL_TRY(run_state(c));
    CL_TRY(red_sumsq_diff(c->red, c->m + c->nt * n, c->m1, n, 0, c->s));
    CL_TRY(red_fetch(c->red, c->s));
    *half_sumsq = 0.5 * c->cell * c->red.host[0];
    return 0;
}

int ensure_solver_buffers(claire_ctx* c) {
    const long long n3 = 3 * c->g.n;
    if (!c->vt) CL_TRY(dalloc(&c->vt, n3));
    if (!c->r) CL_TRY(dalloc(&c->r, n3));
    if (!c->z) CL_TRY(dalloc(&c->z, n3));
    if (!c->sd) CL_TRY(dalloc(&c->sd, n3));
    if (!c->hs) CL_TRY(dalloc(&c->hs, n3));
    if (!c->vtrial) CL_TRY(dalloc(&c->vtrial, n3));
    if (!c->als) CL_TRY(dalloc(&c->als, n3));
    return 0;
}

constexpr int kTraceWidth = 8;

struct PcgResult {
    int its = 0;
    int inner = 0;           // coarse CG iterations of the two-level preconditioner
    bool hit_max = false;
    bool neg_curv = false;   // stopped on <s, Hs> <= 0
};

// PCG (Algorithm 2) on H v~ = -g; v~^0 = 0. Stopping per Section 2.5.5:
// ||r||_inf <= eta ||g||_inf, or a fixed number of matvecs.
//
// With M = alpha L the regularisation part of H s needs no FFT: with
// z = (alpha L)^{-1} r (mean passed through), alpha L z = r - mean(r), so the
// directions s_{l+1} = z_{l+1} + mu s_l satisfy
//   alpha L s_{l+1} = (r_{l+1} - mean(r_{l+1})) + mu alpha L s_l,
// which is carried along in c->als; only the data part of H s is computed.
// With the two-level preconditioner (Section 2.5.6) the matvec computes
// alpha L s itself, and the coarse operator takes grad m(1) of the current
// iterate, restricted once per PCG solve; its inner CG runs to a tenth of eta.
int run_pcg(claire_ctx* c, const claire_opts& o, PcgResult& res) {
    c->trace_res.push_back(c->gnorm);   // ||r_0||_inf = ||g||_inf
    const long long n = c->g.n, n3 = 3 * n;
    const hipStream_t s = c->s;
    const double gn = c->gnorm;
    const double eta = (o.forcing == 1) ? std::fmin(0.5, gn) : std::fmin(0.5, std::sqrt(gn));
    const double tol = eta * gn;
    const bool fixed = o.fixed_pcg_iters > 0;
    const int limit = fixed ? o.fixed_pcg_iters : o.max_pcg;
    const bool two = o.precond == CLAIRE_PRECOND_TWOLEVEL;
    res = PcgResult();
    if (two) {
        CL_TRY(twolevel_init(c->tl, c->g));
        CL_TRY(twolevel_setup(c->tl, c->g, c->sw, c->gm + (long long)c->nt * n3, s));
    }
    // z = M^{-1} r and <z, r> -> slot
    auto precond = [&](int slot) -> int {
        if (!two)
            return spectral_apply(c->g, c->sw, SPEC_REG_INV, c->r, c->z, c->alpha, c->p, s,
                                  nullptr, c->r, &c->red, slot);
        int its = 0;
        CL_TRY(twolevel_apply(c->tl, c->g, c->sw, c->r, c->z, c->alpha, c->p, 0.1 * eta,
                              kMaxInner, &its, s));
        res.inner += its;
        return red_dot(c->red, c->z, c->r, n3, slot, s);
    };
    // Slots of the reducer: 0 <s, Hs>, 1 max|r|, 3..5 the component sums of r,
    // 6 and 7 <z, r> of alternate iterations. kappa, mu and the means are
    // taken on the device (PcgDev), so within an iteration the host waits
    // once, for the event after the preconditioner, while the direction and
    // als updates already run; it then checks the curvature and the residual.
    int rz_slot = 6;
    CL_TRY(launch_fill(c->vt, 0.f, n3, s));
    CL_TRY(launch_scale_copy(c->grad, c->r, -1.f, n3, s));
    CL_TRY(precond(rz_slot));   // z and <z, r>
    CL_TRY(copy_d2d(c->sd, c->z, n3, s));
    for (int a = 0; a < 3; ++a) CL_TRY(red_sum(c->red, c->r + a * n, n, 3 + a, s));
    CL_TRY(red_fetch(c->red, s));
    double rz = c->red.host[rz_slot];
    double mean[3] = {c->red.host[3] / n, c->red.host[4] / n, c->red.host[5] / n};
    if (!two) {
        CL_TRY(launch_fill(c->als, 0.f, n3, s));
        CL_TRY(launch_als_update(c->r, c->als, mean, 0.f, n, s));
    }
    bool converged = false;
    auto curvature_stop = [&](double shs) -> int {
        if (!std::isfinite(shs)) {
            set_error("PCG curvature <s, Hs> = %g is not finite", shs);
            return CLAIRE_ENONFINITE;
        }
        // nonpositive curvature (the discrete Gauss--Newton Hessian is
        // semidefinite only up to discretisation error): truncated CG -- keep
        // the current step (the device updates were no-ops), or take s itself
        // on the first direction
        if (shs <= 0.0) {
            if (res.its == 1) CL_TRY(copy_d2d(c->vt, c->sd, n3, s));
            res.neg_curv = true;
            return 1;
        }
        return 0;
    };
    // plain model, (alpha L)^{-1}: the als update of each direction after the
    // first rides on the next matvec's assembly
    const bool als_fused = !two && !(c->beta > 0.0);
    // the direction update also forms the next matvec's first source w0
    auto a16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    const bool w0_fused = (n & 3) == 0 && a16(c->z) && a16(c->sd) && a16(c->vt) &&
                          a16(c->w0) && a16(c->gm) && (c->precision != 1 || a16(c->gm16));
    bool w0_ready = false;
    PcgDev prev;
    bool have_prev = false;
    while (res.its < limit) {
        // <s, Hs> -> slot 0
        CL_TRY(run_matvec(c, c->sd, c->hs, two ? nullptr : c->als, 0,
                          als_fused && have_prev ? &prev : nullptr, w0_ready));
        w0_ready = false;
        ++res.its;
        if (res.its == limit) {
            // last matvec: r -= kappa Hs and v~ += kappa s, no preconditioner
            CL_TRY(red_fetch(c->red, s));
            const int st = curvature_stop(c->red.host[0]);
            if (st < 0) return st;
            if (st) break;
            const double kappa = rz / c->red.host[0];
            CL_TRY(pcg_update(c->red, c->hs, c->r, (float)kappa, n, 1, 3, s));
            CL_TRY(launch_axpy(c->sd, c->vt, (float)kappa, n3, s));
            CL_TRY(red_fetch(c->red, s));
            c->trace_res.push_back(c->red.host[1]);
            break;
        }
        PcgDev pd;
        pd.sc = c->red.result;
        pd.shs = 0;
        pd.rz = rz_slot;
        pd.rz_new = rz_slot ^ 1;   // 6 <-> 7
        pd.ssum = 3;
        pd.n = n;
        // r -= kappa Hs, with max|r| -> slot 1 and the residual's component sums
        CL_TRY(pcg_update_dev(c->red, c->hs, c->r, pd, n, 1, 3, s));
        CL_TRY(precond(pd.rz_new));   // z and <z, r>
        CL_HIP(hipEventRecord(c->ev_pcg, s));
        // v~ += kappa s, s = z + mu s, als: needed unless the test below stops
        // the solve, and v~ is right in that case too
        if (w0_fused) {
            CL_TRY(c->precision == 1 ? launch_pcg_direction_w0(c, c->gm16, pd)
                                     : launch_pcg_direction_w0(c, c->gm, pd));
            w0_ready = true;
        } else {
            CL_TRY(launch_pcg_direction_dev(c->z, c->sd, c->vt, pd, n3, s));
        }
        if (!two && !als_fused) CL_TRY(launch_als_update_dev(c->r, c->als, pd, n, s));
        CL_HIP(hipEventSynchronize(c->ev_pcg));
        const int st = curvature_stop(c->red.host[0]);
        if (st < 0) return st;
        if (st) break;
        c->trace_res.push_back(c->red.host[1]);
        if (!fixed && c->red.host[1] <= tol) {
            converged = true;
            break;
        }
        rz_slot = pd.rz_new;
        rz = c->red.host[rz_slot];
        prev = pd;
        have_prev = true;
    }
    if (!fixed && !converged && !res.neg_curv && res.its >= limit) {
        // the last residual was not tested inside the loop
        CL_TRY(red_absmax(c->red, c->r, n3, 1, s));
        CL_TRY(red_fetch(c->red, s));
        res.hit_max = c->red.host[1] > tol;
    }
    return 0;
}

// J and ||g||_inf at v = 0 for the plain model, without transport solves:
// with zero velocity every departure point is its grid point (the gathers
// return grid values exactly) and div v = 0, so the state is m0 and the
// adjoint m1 - m0 at every time step, and J = 1/2 ||m0 - m1||^2 (Section
// 2.3). The time slots are filled with those values and the gradient is
// assembled by the same kernel as in a setup, so J and ||g||_inf equal a
// setup's at v = 0 bit for bit. Leaves c->lam, c->gm (slots 1..nt) and
// c->grad overwritten and the state invalid.
int zero_velocity_reference(claire_ctx* c, double* J, double* gnorm) {
    const long long n = c->g.n, n3 = 3 * n;
    const int nt = c->nt;
    const hipStream_t s = c->s;
    if (!c->gm0_valid) {
        CL_TRY(ctx_grad(c, c->m0, c->gm, s));
        c->gm0_valid = true;
    }
    c->state_valid = false;
    CL_TRY(red_sumsq_diff(c->red, c->m0, c->m1, n, 0, s));
    for (int j = 0; j <= nt; ++j)
        CL_TRY(launch_final_adjoint(c->g, c->m0, c->m1, c->lam + (long long)j * n, s));
    for (int j = 1; j <= nt; ++j) CL_TRY(copy_d2d(c->gm + (long long)j * n3, c->gm, n3, s));
    CL_TRY(launch_assemble(c->g, c->lam, c->gm, nt, nullptr, c->grad, s));
    CL_TRY(red_absmax(c->red, c->grad, n3, 2, s));
    CL_TRY(red_fetch(c->red, s));
    *J = 0.5 * c->cell * c->red.host[0];
    *gnorm = c->red.host[2];
    if (!std::isfinite(*J) || !std::isfinite(*gnorm)) {
        set_error("non-finite objective or gradient at v = 0");
        return CLAIRE_ENONFINITE;
    }
    return 0;
}

int run_solve(claire_ctx* c, const claire_opts& o, float* v_io, claire_stats* st) {
    const auto t0 = std::chrono::steady_clock::now();
    const Geo& g = c->g;
    const long long n = g.n, n3 = 3 * n;
    const hipStream_t s = c->s;
    CL_TRY(ensure_solver_buffers(c));
    std::vector<double> levels;
    if (o.alpha_levels && o.n_levels > 0) levels.assign(o.alpha_levels, o.alpha_levels + o.n_levels);
    else levels.push_back(c->alpha);
    for (double a : levels)
        if (!(a > 0.0)) { set_error("alpha levels must be positive"); return CLAIRE_EINVAL; }
    claire_stats S;
    std::memset(&S, 0, sizeof(S));
    c->trace_iters.clear();
    c->trace_res.clear();
    int warn = 0;
    auto note = [&](int w) { if (!warn) warn = w; };
    bool stop_all = false;
    double g0 = 0.0;
    for (size_t li = 0; li < levels.size() && !stop_all; ++li) {
        c->alpha = levels[li];
        double J_zero = 0.0;
        if (o.tol_from_zero) {
            // reference gradient at v = 0 for the stopping test
            if (c->beta > 0.0) {
                CL_TRY(launch_fill(c->v, 0.f, n3, s));
                c->state_valid = false;
                CL_TRY(run_setup(c));
                S.pde_solves += 2;
                g0 = c->gnorm;
                J_zero = c->J;
            } else {
                CL_TRY(zero_velocity_reference(c, &J_zero, &g0));
            }
        }
        CL_TRY(copy_d2d(c->v, v_io, n3, s));
        c->state_valid = false;
        const bool may_reject = o.tol_from_zero && li == 0;
        const int rc0 = run_setup(c);
        if (rc0 < 0 && !(may_reject && rc0 == CLAIRE_ENONFINITE)) return rc0;
        S.pde_solves += 2;
        if (may_reject && (rc0 < 0 || !(c->J <= J_zero))) {
            // a (learned) initial guess no better than v = 0: the plain solve
            // from v = 0 takes over (v_io is the iterate the steps update)
            S.initial_rejected = 1;
            CL_TRY(launch_fill(v_io, 0.f, n3, s));
            CL_TRY(launch_fill(c->v, 0.f, n3, s));
            c->state_valid = false;
            CL_TRY(run_setup(c));
            S.pde_solves += 2;
        }
        if (li == 0) S.J0 = c->J;
        if (!o.tol_from_zero) g0 = c->gnorm;
        int k = 0;
        while (true) {
            const size_t rec = c->trace_iters.size();
            for (double x : {(double)li, (double)k, c->J, c->gnorm, 0.0, 0.0, 0.0, 0.0})
                c->trace_iters.push_back(x);
            if (c->gnorm <= o.gtol * g0 || c->gnorm <= o.gabs) break;
            if (k >= o.max_gn) { note(CLAIRE_WNOTCONV); break; }
            PcgResult pr;
            const size_t res_before = c->trace_res.size();
            CL_TRY(run_pcg(c, o, pr));
            c->trace_iters[rec + 7] = (double)(c->trace_res.size() - res_before);
            S.matvecs += pr.its;
            S.inner_iters += pr.inner;
            S.pde_solves += 2 * pr.its;
            if (pr.hit_max) { ++S.pcg_max_hits; note(CLAIRE_WPCGMAX); }
            if (pr.neg_curv) note(CLAIRE_WNEGCURV);
            // Armijo line search on J(v + gamma v~). The regulariser is
            // quadratic: J_reg(v + gamma v~) = J_reg + gamma <aLv, v~> + gamma^2/2 <aLv~, v~>.
            // With beta > 0 the merit function carries the divergence penalty
            // 1/2 <P v, v> (quadratic too) and the slope is <grad J, v~>.
            const bool ni = c->beta > 0.0;
            CL_TRY(red_dot(c->red, ni ? c->gradJ : c->grad, c->vt, n3, 3, s));
            CL_TRY(red_dot(c->red, c->regv, c->vt, n3, 4, s));
            CL_TRY(spectral_apply(g, c->sw, SPEC_REG, c->vt, c->tmp3, c->alpha, c->p, s));
            CL_TRY(red_dot(c->red, c->tmp3, c->vt, n3, 5, s));
            if (ni) {
                // <P v, v~> = <v, P v~> (P symmetric) and <P v~, v~>
                CL_TRY(spectral_ni(g, c->sw, NI_PENALTY, c->vt, c->ni_tmp, c->alpha, c->beta, s));
                CL_TRY(red_dot(c->red, c->ni_tmp, c->v, n3, 6, s));
                CL_TRY(red_dot(c->red, c->ni_tmp, c->vt, n3, 7, s));
            }
            CL_TRY(red_fetch(c->red, s));
            const double slope = c->cell * c->red.host[3];
            double ra = c->cell * c->red.host[4];
            double rb = c->cell * c->red.host[5];
            if (ni) {
                ra += c->cell * c->red.host[6];
                rb += c->cell * c->red.host[7];
            }
            const double J = c->J, Jreg = c->Jreg + c->Jdiv;
            const int trials_before = S.linesearch_trials;
            double gamma = 1.0;
            bool accepted = false;
            for (int t = 0; t < o.max_linesearch; ++t) {
                CL_TRY(launch_lincomb(v_io, c->vt, c->v, (float)gamma, n3, s));
                double jd = 0.0;
                CL_TRY(run_trial_mismatch(c, &jd));
                ++S.linesearch_trials;
                ++S.pde_solves;
                const double jt = jd + Jreg + gamma * ra + 0.5 * gamma * gamma * rb;
                if (std::isfinite(jt) && jt <= J + o.armijo_c1 * gamma * slope) {
                    accepted = true;
                    break;
                }
                gamma *= 0.5;
            }
            c->trace_iters[rec + 4] = pr.its;
            c->trace_iters[rec + 5] = accepted ? gamma : 0.0;
            c->trace_iters[rec + 6] = S.linesearch_trials - trials_before;
            if (!accepted) {
                note(CLAIRE_WLINESEARCH);
                // restore the setup at the last accepted iterate
                CL_TRY(copy_d2d(c->v, v_io, n3, s));
                c->state_valid = false;
                CL_TRY(run_setup(c));
                stop_all = true;
                break;
            }
            CL_TRY(copy_d2d(v_io, c->v, n3, s));
            CL_TRY(run_setup(c));   // reuses the accepted trial's state
            ++S.pde_solves;          // adjoint solve
            ++k;
            ++S.gn_iters;
        }
        S.rel_grad = g0 > 0 ? c->gnorm / g0 : 0.0;
    }
    S.J = c->J;
    CL_TRY(red_sumsq_diff(c->red, c->m + c->nt * n, c->m1, n, 0, s));
    CL_TRY(red_sumsq_diff(c->red, c->m0, c->m1, n, 1, s));
    CL_TRY(red_fetch(c->red, s));
    S.rel_mismatch = c->red.host[1] > 0 ? std::sqrt(c->red.host[0] / c->red.host[1]) : 0.0;
    S.det_min = S.det_mean = S.det_max = 0.0;
    S.det_nonpositive = 0;
    if (o.compute_det) {
        double ds[4];
        int rc = claire_ctx_detdefgrad(c, nullptr, ds);
        if (rc < 0) return rc;
        S.det_min = ds[0];
        S.det_mean = ds[1];
        S.det_max = ds[2];
        S.det_nonpositive = (long long)ds[3];
        if (rc > 0) note(rc);
    }
    CL_HIP(hipStreamSynchronize(s));
    S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = S;
    return warn;
}

int need(claire_ctx* c, bool velocity) {
    if (!c) { set_error("ctx is NULL"); return CLAIRE_EINVAL; }
    if (!c->have_images) { set_error("call claire_ctx_set_images first"); return CLAIRE_ESTATE; }
    if (velocity && !c->have_velocity) {
        set_error("call claire_ctx_set_velocity first");
        return CLAIRE_ESTATE;
    }
    return 0;
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_ptr(const void* p, const char* name) {
    if (!p) { set_error("%s is NULL", name); return CLAIRE_EINVAL; }
    if (!aligned(p)) { set_error("%s is not 16-byte aligned", name); return CLAIRE_EINVAL; }
    return 0;
}

}  // namespace

// ===================================================================== ABI
extern "C" {

void claire_opts_default(claire_opts* o) {
    if (!o) return;
    o->reg_order = 1;
    o->precision = 0;
    o->gtol = 5e-2;
    o->gabs = 1e-6;
    o->forcing = 0;
    o->max_gn = 50;
    o->max_pcg = 100;
    o->fixed_pcg_iters = 0;
    o->max_linesearch = 16;
    o->armijo_c1 = 1e-4;
    o->alpha_levels = nullptr;
    o->n_levels = 0;
    o->compute_det = 0;
    o->tol_from_zero = 0;
    o->derivative = CLAIRE_DERIV_SPECTRAL;
    o->precond = CLAIRE_PRECOND_REG;
    o->beta = 0.0;
}

const char* claire_last_error(void) { return g_err; }

int claire_ctx_create(claire_ctx** out, const int nx[3], int nt, double alpha, int reg_order,
                      void* stream) {
    if (!out) { set_error("out is NULL"); return CLAIRE_EINVAL; }
    *out = nullptr;
    CL_TRY(check_args(nx, nt, alpha, reg_order));
    claire_ctx* c = new (std::nothrow) claire_ctx();
    if (!c) { set_error("host allocation failed"); return CLAIRE_ENOMEM; }
    c->g = make_geo(nx);
    c->nt = nt;
    c->alpha = alpha;
    c->p = reg_order;
    c->s = reinterpret_cast<hipStream_t>(stream);
    c->cell = (2.0 * M_PI / nx[0]) * (2.0 * M_PI / nx[1]) * (2.0 * M_PI / nx[2]);
    int rc = ctx_alloc(c);
    if (rc < 0) {
        ctx_release(c);
        delete c;
        return rc;
    }
    *out = c;
    return 0;
}

int claire_ctx_destroy(claire_ctx* c) {
    if (!c) return 0;
    if (c->s) (void)hipStreamSynchronize(c->s);
    else (void)hipDeviceSynchronize();
    ctx_release(c);
    delete c;
    return 0;
}

int claire_ctx_set_alpha(claire_ctx* c, double alpha) {
    if (!c) { set_error("ctx is NULL"); return CLAIRE_EINVAL; }
    if (!(alpha > 0.0)) { set_error("alpha must be positive"); return CLAIRE_EINVAL; }
    c->alpha = alpha;
    c->have_velocity = false;
    return 0;
}

int claire_ctx_set_images(claire_ctx* c, const float* m0, const float* m1) {
    if (!c) { set_error("ctx is NULL"); return CLAIRE_EINVAL; }
    CL_TRY(check_ptr(m0, "m0"));
    CL_TRY(check_ptr(m1, "m1"));
    CL_TRY(copy_d2d(c->m0, m0, c->g.n, c->s));
    CL_TRY(copy_d2d(c->m1, m1, c->g.n, c->s));
    c->have_images = true;
    c->state_valid = false;
    c->have_velocity = false;
    c->gm0_valid = false;
    return 0;
}

int claire_ctx_set_velocity(claire_ctx* c, const float* v) {
    CL_TRY(need(c, false));
    CL_TRY(check_ptr(v, "v"));
    CL_TRY(copy_d2d(c->v, v, 3 * c->g.n, c->s));
    c->state_valid = false;
    return run_setup(c);
}

int claire_ctx_gradient(claire_ctx* c, float* g, double* J) {
    CL_TRY(need(c, true));
    if (g) {
        CL_TRY(check_ptr(g, "g"));
        CL_TRY(copy_d2d(g, c->grad, 3 * c->g.n, c->s));
    }
    if (J) *J = c->J;
    return 0;
}

int claire_ctx_objective(claire_ctx* c, const float* v, double* J) {
    CL_TRY(need(c, false));
    CL_TRY(check_ptr(v, "v"));
    if (!J) { set_error("J is NULL"); return CLAIRE_EINVAL; }
    CL_TRY(copy_d2d(c->v, v, 3 * c->g.n, c->s));
    double jd = 0.0;
    CL_TRY(run_trial_mismatch(c, &jd));
    CL_TRY(spectral_apply(c->g, c->sw, SPEC_REG, c->v, c->tmp3, c->alpha, c->p, c->s));
    CL_TRY(red_dot(c->red, c->tmp3, c->v, 3 * c->g.n, 1, c->s));
    if (c->beta > 0.0) {
        CL_TRY(ensure_ni_buffers(c));
        CL_TRY(spectral_ni(c->g, c->sw, NI_PENALTY, c->v, c->ni_tmp, c->alpha, c->beta, c->s,
                           nullptr, c->v, &c->red, 2));
    }
    CL_TRY(red_fetch(c->red, c->s));
    *J = jd + 0.5 * c->cell * c->red.host[1] +
         (c->beta > 0.0 ? 0.5 * c->cell * c->red.host[2] : 0.0);
    return 0;
}

int claire_ctx_hessian_matvec(claire_ctx* c, const float* vt, float* Hvt) {
    CL_TRY(need(c, true));
    CL_TRY(check_ptr(vt, "vt"));
    CL_TRY(check_ptr(Hvt, "Hvt"));
    if (vt == Hvt) { set_error("vt and Hvt must not overlap"); return CLAIRE_EINVAL; }
    return run_matvec(c, vt, Hvt);
}

int claire_ctx_precond(claire_ctx* c, const float* r, float* z) {
    if (!c) { set_error("ctx is NULL"); return CLAIRE_EINVAL; }
    CL_TRY(check_ptr(r, "r"));
    CL_TRY(check_ptr(z, "z"));
    return spectral_apply(c->g, c->sw, SPEC_REG_INV, r, z, c->alpha, c->p, c->s);
}

int claire_ctx_precond_twolevel(claire_ctx* c, const float* r, float* z, double inner_rtol,
                                int max_inner, int* inner_iters) {
    CL_TRY(need(c, true));
    CL_TRY(check_ptr(r, "r"));
    CL_TRY(check_ptr(z, "z"));
    if (r == z) { set_error("r and z must not overlap"); return CLAIRE_EINVAL; }
    if (!(inner_rtol >= 0.0) || max_inner < 1 || max_inner > 1000) {
        set_error("need inner_rtol >= 0 and 1 <= max_inner <= 1000");
        return CLAIRE_EINVAL;
    }
    CL_TRY(twolevel_init(c->tl, c->g));
    CL_TRY(twolevel_setup(c->tl, c->g, c->sw, c->gm + (long long)c->nt * 3 * c->g.n, c->s));
    int its = 0;
    CL_TRY(twolevel_apply(c->tl, c->g, c->sw, r, z, c->alpha, c->p, inner_rtol, max_inner, &its,
                          c->s));
    CL_HIP(hipStreamSynchronize(c->s));
    if (inner_iters) *inner_iters = its;
    return 0;
}

int claire_ctx_solve(claire_ctx* c, const claire_opts* opts, float* v_inout,
                     claire_stats* stats) {
    CL_TRY(need(c, false));
    CL_TRY(check_ptr(v_inout, "v_inout"));
    claire_opts o;
    if (opts) o = *opts;
    else claire_opts_default(&o);
    if (opts && o.reg_order != c->p) {
        set_error("opts->reg_order %d differs from the context's %d", o.reg_order, c->p);
        return CLAIRE_EINVAL;
    }
    if (o.precision != 0 && o.precision != 1) {
        set_error("precision must be 0 (float32) or 1 (mixed)");
        return CLAIRE_EINVAL;
    }
    if (o.max_gn < 0 || o.max_pcg < 1 || o.max_linesearch < 1 || !(o.gtol >= 0)) {
        set_error("invalid solver limits");
        return CLAIRE_EINVAL;
    }
    if (o.derivative != CLAIRE_DERIV_SPECTRAL && o.derivative != CLAIRE_DERIV_FD8) {
        set_error("derivative must be CLAIRE_DERIV_SPECTRAL or CLAIRE_DERIV_FD8");
        return CLAIRE_EINVAL;
    }
    if (o.precond != CLAIRE_PRECOND_REG && o.precond != CLAIRE_PRECOND_TWOLEVEL) {
        set_error("precond must be CLAIRE_PRECOND_REG or CLAIRE_PRECOND_TWOLEVEL");
        return CLAIRE_EINVAL;
    }
    if (!(o.beta >= 0.0)) { set_error("beta must be >= 0"); return CLAIRE_EINVAL; }
    if (o.beta > 0.0 && c->p != 1) {
        set_error("the near-incompressible model (beta > 0) uses the H1 seminorm (reg_order 1)");
        return CLAIRE_EINVAL;
    }
    if (o.beta > 0.0 && o.precond == CLAIRE_PRECOND_TWOLEVEL) {
        set_error("the two-level preconditioner is not combined with beta > 0");
        return CLAIRE_EINVAL;
    }
    if (o.precond == CLAIRE_PRECOND_TWOLEVEL) CL_TRY(twolevel_init(c->tl, c->g));
    if (o.beta > 0.0) CL_TRY(ensure_ni_buffers(c));
    const int saved = c->precision;
    const int saved_deriv = c->deriv;
    const double saved_beta = c->beta;
    c->precision = o.precision;
    if (o.derivative != c->deriv) c->gm0_valid = false;
    c->deriv = o.derivative;
    c->beta = o.beta;
    const int rc = run_solve(c, o, v_inout, stats);
    c->precision = saved;
    if (c->deriv != saved_deriv) {   // setup used the other operators
        c->have_velocity = false;
        c->gm0_valid = false;
    }
    c->deriv = saved_deriv;
    if (c->beta != saved_beta) c->have_velocity = false;
    c->beta = saved_beta;
    if (saved == 1 && o.precision != 1) c->have_velocity = false;   // half copies not made
    return rc;
}

int claire_ctx_set_beta(claire_ctx* c, double beta) {
    if (!c) { set_error("ctx is NULL"); return CLAIRE_EINVAL; }
    if (!(beta >= 0.0)) { set_error("beta must be >= 0"); return CLAIRE_EINVAL; }
    if (beta > 0.0 && c->p != 1) {
        set_error("the near-incompressible model (beta > 0) uses the H1 seminorm (reg_order 1)");
        return CLAIRE_EINVAL;
    }
    if (beta > 0.0) CL_TRY(ensure_ni_buffers(c));
    if (beta != c->beta) c->have_velocity = false;   // redo the setup
    c->beta = beta;
    return 0;
}

int claire_ctx_set_derivative(claire_ctx* c, int derivative) {
    if (!c) { set_error("ctx is NULL"); return CLAIRE_EINVAL; }
    if (derivative != CLAIRE_DERIV_SPECTRAL && derivative != CLAIRE_DERIV_FD8) {
        set_error("derivative must be CLAIRE_DERIV_SPECTRAL or CLAIRE_DERIV_FD8");
        return CLAIRE_EINVAL;
    }
    if (derivative != c->deriv) {   // redo the setup, grad m0 included
        c->have_velocity = false;
        c->gm0_valid = false;
    }
    c->deriv = derivative;
    return 0;
}

int claire_ctx_set_precision(claire_ctx* c, int precision) {
    if (!c) { set_error("ctx is NULL"); return CLAIRE_EINVAL; }
    if (precision != 0 && precision != 1) {
        set_error("precision must be 0 (float32) or 1 (mixed)");
        return CLAIRE_EINVAL;
    }
    if (precision == 1) CL_TRY(ensure_half_buffers(c));
    if (precision != c->precision) c->have_velocity = false;   // redo the setup
    c->precision = precision;
    return 0;
}

int claire_ctx_solve_trace(claire_ctx* c, double* iters, int max_iters, double* pcg_res,
                           int max_res, int counts[2]) {
    if (!c || !counts) { set_error("ctx or counts is NULL"); return CLAIRE_EINVAL; }
    const int ni = (int)(c->trace_iters.size() / kTraceWidth);
    const int nr = (int)c->trace_res.size();
    counts[0] = ni;
    counts[1] = nr;
    if (iters && max_iters > 0)
        std::memcpy(iters, c->trace_iters.data(),
                    sizeof(double) * kTraceWidth * (size_t)std::min(ni, max_iters));
    if (pcg_res && max_res > 0)
        std::memcpy(pcg_res, c->trace_res.data(), sizeof(double) * (size_t)std::min(nr, max_res));
    return 0;
}

int claire_ctx_detdefgrad(claire_ctx* c, double* det_out, double stats[4]) {
    CL_TRY(need(c, false));
    if (!c->state_valid) {
        set_error("no velocity set");
        return CLAIRE_ESTATE;
    }
    const Geo& g = c->g;
    const long long n = g.n;
    float* G = nullptr;    // [9][n] grad v, G_ab = d_b v_a
    float* Gy = nullptr;   // [9][n] G at y+
    float* F = nullptr;    // [9][n]
    float* Fy = nullptr;   // [9][n] F^j at y+
    double* det = det_out;
    int rc = 0;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(c->s);
        dfree(G);
        dfree(Gy);
        dfree(F);
        dfree(Fy);
        if (!det_out) dfree(det);
    };
    if ((rc = dalloc(&G, 9 * n)) < 0 || (rc = dalloc(&Gy, 9 * n)) < 0 ||
        (rc = dalloc(&F, 9 * n)) < 0 || (rc = dalloc(&Fy, 9 * n)) < 0 ||
        (!det_out && (rc = dalloc(&det, n)) < 0)) {
        cleanup();
        return rc;
    }
    const double ht = 1.0 / c->nt;
    for (int a = 0; a < 3 && rc >= 0; ++a)
        rc = ctx_grad(c, c->v + (long long)a * n, G + (long long)a * 3 * n, c->s);
    for (int q = 0; q < 9 && rc >= 0; ++q)
        rc = launch_interp(g, G + (long long)q * n, 1, c->dp, Gy + (long long)q * n, c->s, c->box_p);
    if (rc >= 0) rc = launch_defgrad_update(g, nullptr, Gy, G, F, ht, c->s);
    for (int j = 1; j < c->nt && rc >= 0; ++j) {
        for (int q = 0; q < 9 && rc >= 0; ++q)
            rc = launch_interp(g, F + (long long)q * n, 1, c->dp, Fy + (long long)q * n, c->s,
                               c->box_p);
        if (rc >= 0) rc = launch_defgrad_update(g, Fy, Gy, G, F, ht, c->s);
    }
    if (rc >= 0) rc = launch_det(g, F, det, c->s);
    if (rc >= 0) rc = red_stats_f64(c->red, det, n, c->s);
    if (rc >= 0) rc = red_fetch(c->red, c->s);
    if (rc >= 0 && stats) {
        stats[0] = c->red.host[0];
        stats[1] = c->red.host[1] / (double)n;
        stats[2] = c->red.host[2];
        stats[3] = c->red.host[3];
    }
    const bool bad = rc >= 0 && c->red.host[3] > 0;
    cleanup();
    if (rc < 0) return rc;
    return bad ? CLAIRE_WDETBOUND : 0;
}

int claire_ctx_spectral(claire_ctx* c, int op, const float* in, float* out) {
    if (!c) { set_error("ctx is NULL"); return CLAIRE_EINVAL; }
    CL_TRY(check_ptr(in, "in"));
    CL_TRY(check_ptr(out, "out"));
    if (in == out) { set_error("in and out must not overlap"); return CLAIRE_EINVAL; }
    if (op == CLAIRE_OP_FD8_GRAD) return launch_fd8_grad(c->g, in, out, c->s);
    if (op == CLAIRE_OP_FD8_DIV) return launch_fd8_div(c->g, in, out, c->s);
    if (op == CLAIRE_OP_NI_PROJECT || op == CLAIRE_OP_NI_PENALTY) {
        if (!(c->beta > 0.0)) {
            set_error("the near-incompressible operators need beta > 0 (claire_ctx_set_beta)");
            return CLAIRE_EINVAL;
        }
        return spectral_ni(c->g, c->sw, op == CLAIRE_OP_NI_PROJECT ? NI_PROJECT : NI_PENALTY,
                           in, out, c->alpha, c->beta, c->s);
    }
    SpecMode m;
    switch (op) {
    case CLAIRE_OP_GRAD: m = SPEC_GRAD; break;
    case CLAIRE_OP_DIV: m = SPEC_DIV; break;
    case CLAIRE_OP_REG: m = SPEC_REG; break;
    case CLAIRE_OP_REG_INV: m = SPEC_REG_INV; break;
    default: set_error("unknown op %d", op); return CLAIRE_EINVAL;
    }
    return spectral_apply(c->g, c->sw, m, in, out, c->alpha, c->p, c->s);
}

int claire_ctx_interpolate(claire_ctx* c, const float* f, int nfield, const float* disp,
                           float* out) {
    if (!c) { set_error("ctx is NULL"); return CLAIRE_EINVAL; }
    CL_TRY(check_ptr(f, "f"));
    CL_TRY(check_ptr(disp, "disp"));
    CL_TRY(check_ptr(out, "out"));
    if (nfield < 1 || nfield > 64) { set_error("nfield must be in [1, 64]"); return CLAIRE_EINVAL; }
    if (f == out) { set_error("out must not overlap f"); return CLAIRE_EINVAL; }
    return launch_interp(c->g, f, nfield, disp, out, c->s);
}

int claire_ctx_get_field(claire_ctx* c, int which, int index, float* out) {
    if (!c) { set_error("ctx is NULL"); return CLAIRE_EINVAL; }
    CL_TRY(check_ptr(out, "out"));
    const long long n = c->g.n;
    const bool state_field = which == CLAIRE_FIELD_DISP_PLUS || which == CLAIRE_FIELD_DISP_MINUS ||
                             which == CLAIRE_FIELD_STATE;
    if (state_field ? !c->state_valid : !c->have_velocity) {
        set_error("field %d not available: call claire_ctx_set_velocity first", which);
        return CLAIRE_ESTATE;
    }
    if ((which == CLAIRE_FIELD_STATE || which == CLAIRE_FIELD_GRAD_STATE ||
         which == CLAIRE_FIELD_ADJOINT) && (index < 0 || index > c->nt)) {
        set_error("index %d out of range [0, %d]", index, c->nt);
        return CLAIRE_EINVAL;
    }
    switch (which) {
    case CLAIRE_FIELD_DISP_PLUS: return copy_d2d(out, c->dp, 3 * n, c->s);
    case CLAIRE_FIELD_DISP_MINUS: return copy_d2d(out, c->dm, 3 * n, c->s);
    case CLAIRE_FIELD_STATE: return copy_d2d(out, c->m + index * n, n, c->s);
    case CLAIRE_FIELD_GRAD_STATE: return copy_d2d(out, c->gm + index * 3 * n, 3 * n, c->s);
    case CLAIRE_FIELD_ADJOINT: return copy_d2d(out, c->lam + index * n, n, c->s);
    case CLAIRE_FIELD_DIVV: return copy_d2d(out, c->divv, n, c->s);
    default: set_error("unknown field %d", which); return CLAIRE_EINVAL;
    }
}

int claire_ctx_time_kernel(claire_ctx* c, int kernel, int reps, double* avg_ms) {
    CL_TRY(need(c, true));
    if (!avg_ms) { set_error("avg_ms is NULL"); return CLAIRE_EINVAL; }
    if (reps < 1 || reps > 100000) { set_error("reps must be in [1, 100000]"); return CLAIRE_EINVAL; }
    if (kernel < CLAIRE_KERNEL_INC_STATE_STEP || kernel > CLAIRE_KERNEL_INC_STATE_STEP_MIXED) {
        set_error("unknown kernel id %d", kernel);
        return CLAIRE_EINVAL;
    }
    if (kernel == CLAIRE_KERNEL_INC_STATE_STEP_MIXED &&
        (c->precision != 1 || !c->gm16 || !c->half_valid)) {
        set_error("the mixed incremental-state step needs set_precision(1) before set_velocity");
        return CLAIRE_EINVAL;
    }
    const Geo& g = c->g;
    const long long n = g.n;
    const double ht = 1.0 / c->nt;
    auto launch = [&]() -> int {
        switch (kernel) {
        case CLAIRE_KERNEL_INC_STATE_STEP:
            return launch_inc_state_step(g, c->w0, c->dp, c->gm + 3 * n, c->regv, c->w1,
                                         (float)ht, 1.0f, c->s, c->box_p);
        case CLAIRE_KERNEL_INC_STATE_STEP_MIXED:
            return launch_inc_state_step(g, c->w0, c->dp, c->gm16 + 3 * n, c->regv, c->w1,
                                         (float)ht, 1.0f, c->s, c->box_p);
        case CLAIRE_KERNEL_ADJOINT_STEP:
            return launch_adjoint_step(g, c->lam + n, c->dm, c->A, c->lam, c->s, c->box_m);
        case CLAIRE_KERNEL_ASSEMBLE:
            return launch_assemble(g, c->lam, c->gm, c->nt, c->tmp3, c->tmp3, c->s);
        case CLAIRE_KERNEL_BACKTRACE:
            return launch_backtrace(g, c->v, c->dp, c->dm, ht, c->s);
        default:
            return launch_scale_copy(c->regv, c->tmp3, 1.0f, 3 * n, c->s);
        }
    };
    CL_TRY(launch());   // warm-up
    hipEvent_t e0, e1;
    CL_HIP(hipEventCreate(&e0));
    CL_HIP(hipEventCreate(&e1));
    int rc = 0;
    if (hipEventRecord(e0, c->s) != hipSuccess) rc = CLAIRE_EDEVICE;
    for (int i = 0; i < reps && rc == 0; ++i) rc = launch();
    float ms = 0.f;
    if (rc == 0 && hipEventRecord(e1, c->s) != hipSuccess) rc = CLAIRE_EDEVICE;
    if (rc == 0 && hipEventSynchronize(e1) != hipSuccess) rc = CLAIRE_EDEVICE;
    if (rc == 0 && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = CLAIRE_EDEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == CLAIRE_EDEVICE) set_error("HIP event timing failed");
    if (rc < 0) return rc;
    *avg_ms = (double)ms / reps;
    return 0;
}

// ------------------------------------------------------------- stateless
namespace {
struct Owned {
    claire_ctx* c = nullptr;
    ~Owned() { if (c) claire_ctx_destroy(c); }
};
}  // namespace

int claire_transport(const float* m0, const float* v, const int nx[3], int nt, float* m1_out,
                     void* stream) {
    CL_TRY(check_ptr(m0, "m0"));
    CL_TRY(check_ptr(v, "v"));
    CL_TRY(check_ptr(m1_out, "m1_out"));
    Owned o;
    CL_TRY(claire_ctx_create(&o.c, nx, nt, 1.0, 1, stream));
    CL_TRY(claire_ctx_set_images(o.c, m0, m0));
    CL_TRY(copy_d2d(o.c->v, v, 3 * o.c->g.n, o.c->s));
    CL_TRY(run_state(o.c));
    CL_TRY(copy_d2d(m1_out, o.c->m + (long long)nt * o.c->g.n, o.c->g.n, o.c->s));
    CL_HIP(hipStreamSynchronize(o.c->s));
    return 0;
}

int claire_gradient(const float* m0, const float* m1, const float* v, const int nx[3],
                    double alpha, int nt, int reg_order, float* g_out, double* J_out,
                    void* stream) {
    Owned o;
    CL_TRY(claire_ctx_create(&o.c, nx, nt, alpha, reg_order, stream));
    CL_TRY(claire_ctx_set_images(o.c, m0, m1));
    CL_TRY(claire_ctx_set_velocity(o.c, v));
    CL_TRY(claire_ctx_gradient(o.c, g_out, J_out));
    CL_HIP(hipStreamSynchronize(o.c->s));
    return 0;
}

int claire_hessian_matvec(const float* m0, const float* m1, const float* v, const float* vt,
                          const int nx[3], double alpha, int nt, int reg_order, float* Hvt_out,
                          void* stream) {
    Owned o;
    CL_TRY(claire_ctx_create(&o.c, nx, nt, alpha, reg_order, stream));
    CL_TRY(claire_ctx_set_images(o.c, m0, m1));
    CL_TRY(claire_ctx_set_velocity(o.c, v));
    CL_TRY(claire_ctx_hessian_matvec(o.c, vt, Hvt_out));
    CL_HIP(hipStreamSynchronize(o.c->s));
    return 0;
}

int claire_solve(const float* m0, const float* m1, const int nx[3], double alpha, int nt,
                 const claire_opts* opts, float* v_inout, claire_stats* stats, void* stream) {
    const int reg = opts ? opts->reg_order : 1;
    Owned o;
    CL_TRY(claire_ctx_create(&o.c, nx, nt, alpha, reg, stream));
    CL_TRY(claire_ctx_set_images(o.c, m0, m1));
    return claire_ctx_solve(o.c, opts, v_inout, stats);
}

}  // extern "C"
