// Internal declarations of the gfx950 registration engine (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <hip/hip_fp16.h>

#include <cstdint>

#include "claire.h"

namespace claire {

// Grid geometry. n3 (the contiguous axis) is a power of two; n1 and n2 are
// even products of 2, 3 and 5. When all three are powers of two (pow2) the
// tuned kernels run, with masks and shifts for the periodic wrap; otherwise
// the general-extent kernels (modulo wrap, mixed-radix column FFTs).
struct Geo {
    int n1, n2, n3;     // extents
    int l1, l2, l3;     // log2 of the extents (l1, l2 only meaningful when pow2)
    int nh;             // n3/2 + 1: bins of a half-complex x3 row
    int hp;             // row pitch of the spectra: nh rounded up to 16 complex (128 B)
    long long n;        // voxels
    long long nspec;    // half-complex spectrum length n1*n2*hp
    bool pow2;          // every extent a power of two
};

Geo make_geo(const int nx[3]);
// Row pitch of a half-complex spectrum with nh bins: a multiple of 16 complex
// values, so that column tiles read whole 128-byte lines.
__host__ __device__ __forceinline__ int spec_pitch(int nh) { return (nh + 15) & ~15; }

// Exact a / b for 0 <= a < 2^14 and 1 <= b <= 4096 from one float product:
// with inv_b = (1 + 2^-16) / b rounded to float, trunc(a * inv_b) = floor(a/b)
// (the bias lifts exact multiples above the rounding error and stays below
// 1/b for a < 2^14; verified exhaustively in IEEE single precision over that
// range). 24-bit integer products keep the remainder full-rate.
__device__ __forceinline__ float quot_inv(int b) { return (1.0f + 0x1p-16f) / (float)b; }
__device__ __forceinline__ int quot(int a, int b, float inv_b, int& r) {
    const int q = (int)((float)a * inv_b);
    r = a - (int)__umul24((unsigned)q, (unsigned)b);
    return q;
}
// CLAIRE_OK if nx is a supported grid (n3 a power of two, n1 and n2 even
// products of 2, 3 and 5, all in [8, 1024]); else CLAIRE_EINVAL with a message
int check_extents(const int nx[3]);

struct Reducer;

// PCG scalars taken on the device from the reducer's result slots, so the
// host need not wait for them: kappa = rz / <s, Hs>, mu = rz_new / rz, and the
// means of the residual's components (their sums / n). A curvature <s, Hs>
// that is not positive and finite turns every update that reads these into a
// no-op (the host, reading the same slot afterwards, ends the iteration).
struct PcgDev {
    const double* sc = nullptr;   // Reducer::result (device)
    int shs = 0;                  // slot of <s, Hs>
    int rz = 0, rz_new = 0;       // slots of <z, r> before and after the update
    int ssum = 0;                 // first of the three component sums of r
    long long n = 0;              // voxels (the means' divisor)
};
__device__ __forceinline__ bool pcg_curv_ok(const PcgDev& p) {
    const double shs = p.sc[p.shs];
    return shs > 0.0 && shs <= 1.7976931348623157e308;   // false for NaN and infinity too
}
// mu and the residual means from the device slots (false on a bad curvature)
__device__ __forceinline__ bool pcg_als_scalars(const PcgDev& pd, float& m0, float& m1,
                                                float& m2, float& mu) {
    if (!pcg_curv_ok(pd)) return false;
    mu = (float)(pd.sc[pd.rz_new] / pd.sc[pd.rz]);
    m0 = (float)(pd.sc[pd.ssum] / (double)pd.n);
    m1 = (float)(pd.sc[pd.ssum + 1] / (double)pd.n);
    m2 = (float)(pd.sc[pd.ssum + 2] / (double)pd.n);
    return true;
}

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what, const char* file, int line);

#define CL_HIP(call)                                                      \
    do {                                                                  \
        hipError_t _e = (call);                                           \
        if (_e != hipSuccess) return ::claire::hip_fail(_e, #call, __FILE__, __LINE__); \
    } while (0)

#define CL_TRY(call)                                                      \
    do {                                                                  \
        int _s = (call);                                                  \
        if (_s < 0) return _s;                                            \
    } while (0)

#define CL_LAUNCH_CHECK() CL_HIP(hipGetLastError())

// ------------------------------------------------------------ spectral
// Workspace of the FFT-based operators: three half-complex spectra in float
// and in double (the forward half of alpha L runs in double), and the twiddle
// tables exp(-2 pi i k / tw_n), k < tw_n, tw_n = max extent.
struct SpectralWork {
    float2* spec = nullptr;     // [3][nspec]
    double2* spec64 = nullptr;  // [3][nspec]
    float2* tw = nullptr;       // [tw_n]
    double2* tw64 = nullptr;    // [tw_n]
    int tw_n = 0;               // max extent (power-of-two grids), n3 otherwise
    // general grids: exp(-2 pi i q / n_a), q < n_a, for the x1 and x2 columns
    float2* tw1 = nullptr;
    double2* tw1_64 = nullptr;
    float2* tw2 = nullptr;
    double2* tw2_64 = nullptr;
};

int spectral_init(SpectralWork& w, const Geo& g);
void spectral_free(SpectralWork& w);

// Multiplier applied between the forward and inverse transforms.
enum SpecMode {
    SPEC_GRAD = 0,     // 1 input  -> 3 outputs: i k_a (Nyquist zero)
    SPEC_DIV = 1,      // 3 inputs -> 1 output:  sum_a i k_a u_a
    SPEC_REG = 2,      // 3 -> 3: alpha |k|^{2p}
    SPEC_REG_INV = 3,  // 3 -> 3: 1/(alpha |k|^{2p}), 1 at k = 0
    SPEC_REG_ISQRT = 4,  // 3 -> 3: (alpha |k|^{2p})^{-1/2}, 1 at k = 0
    SPEC_REG32 = 5,    // 3 -> 3: alpha |k|^{2p} with a float32 forward transform
                       // (power-of-two grids; others take SPEC_REG)
};

// out = F^{-1}[ sigma F[in] ] for the mode above; in and out are real fields
// (SoA). `add` (nullable, same shape as out) is added to the result. in and
// out must not overlap. With dot_with (SPEC_REG_INV only), <out, dot_with>
// is also summed into red->result[slot].
int spectral_apply(const Geo& g, SpectralWork& w, SpecMode mode, const float* in,
                   float* out, double alpha, int p, hipStream_t s,
                   const float* add = nullptr, const float* dot_with = nullptr,
                   Reducer* red = nullptr, int slot = 0);

// Near-incompressible model (3 -> 3, components coupled per Fourier mode;
// k_d the odd-derivative wavenumbers, Nyquist 0):
//   NI_PROJECT: out = (I - grad M Delta^{-1} div) in,
//               M = (alpha (beta (-Delta^{-1} + id))^{-1} + id)^{-1};
//   NI_PENALTY: out = -grad beta (-Delta^{-1} + id) div in.
// `add` (nullable) is added to the result; with dot_with, <out, dot_with> is
// summed into red->result[slot] (not together with add). in and out must not
// overlap. beta > 0.
enum NiMode { NI_PROJECT = 0, NI_PENALTY = 1 };
int spectral_ni(const Geo& g, SpectralWork& w, NiMode mode, const float* in, float* out,
                double alpha, double beta, hipStream_t s, const float* add = nullptr,
                const float* dot_with = nullptr, Reducer* red = nullptr, int slot = 0);

// ----------------------------------------------- finite differences
// FD8 gradient (1 -> 3 fields) and divergence (3 -> 1), periodic.
int launch_fd8_grad(const Geo& g, const float* u, float* out, hipStream_t s);
int launch_fd8_div(const Geo& g, const float* v, float* out, hipStream_t s);

// Split transforms (unnormalised both ways: inverse(forward(u)) = n u) of
// ncomp fields into / out of half-complex spectra [ncomp][n1][n2][n3/2+1]
// (float32), and the spectral grid transfer of the two-level preconditioner
// between a grid and the grid of half its extents (cut-off below the coarse
// Nyquist |k_a| < n_a/4).
int spectral_forward(const Geo& g, const SpectralWork& w, const float* in, float2* spec,
                     int ncomp, hipStream_t s);
int spectral_inverse(const Geo& g, const SpectralWork& w, float2* spec, float* out, int ncomp,
                     hipStream_t s);
// C = sigma F / n_f on the kept modes (zero elsewhere); sigma = (alpha
// |k|^{2p})^{-1/2} (1 at k = 0) when isqrt, else 1
int spectral_restrict_modes(const Geo& gf, const Geo& gc, const float2* F, float2* C, int ncomp,
                            double alpha, int p, bool isqrt, hipStream_t s);
// in place over F: kept modes sigma S / n_c, the others sigma^2 F / n_f
int spectral_combine_modes(const Geo& gf, const Geo& gc, float2* F, const float2* S, int ncomp,
                           double alpha, int p, hipStream_t s);

// ------------------------------------------------------ semi-Lagrangian
// Single-field gathers accept an optional per-brick box table of their
// departure field (from launch_brick_boxes); NULL computes the boxes inline.
int brick_table_ints(const Geo& g);
int launch_brick_boxes(const Geo& g, const float* disp, int* table, hipStream_t s);
int launch_backtrace(const Geo& g, const float* v, float* dplus, float* dminus,
                     double ht, hipStream_t s);
int launch_interp(const Geo& g, const float* f, int nfield, const float* disp,
                  float* out, hipStream_t s, const int* boxes = nullptr);
int launch_make_A(const Geo& g, const float* divv, const float* dminus, float* A,
                  double ht, hipStream_t s, const int* boxes = nullptr);
int launch_final_adjoint(const Geo& g, const float* mT, const float* m1, float* lamT,
                         hipStream_t s);
int launch_adjoint_step(const Geo& g, const float* lam_next, const float* dminus,
                        const float* A, float* lam, hipStream_t s, const int* boxes = nullptr);
// Hessian matvec kernels; GT is the storage type of grad m^j: float, or
// __half in the mixed-precision matvec (arithmetic in float either way).
// w^0 = -(h_t/2) grad m^0 . v~
template <typename GT>
int launch_inc_state_first(const Geo& g, const GT* gradm0, const float* vt, float* w0,
                           double ht, hipStream_t s);
// out = sign (w_prev(y+) + coef f), f = -grad m^{j+1} . v~ formed on the grid
template <typename GT>
int launch_inc_state_step(const Geo& g, const float* w_prev, const float* dplus,
                          const GT* gradm_next, const float* vt, float* out, float coef,
                          float sign, hipStream_t s, const int* boxes = nullptr);
// out = add + h_t sum_j c_j lam^j grad m^j; with dot_with (nullable), also
// <dot_with, out> summed into red.result[slot]. With als_pd (PCG; add NULL),
// the alpha L s recursion `als` is first advanced in place to
// (r - mean(r)) + mu als with the device scalars (r: the residual) and added.
template <typename GT>
int launch_assemble(const Geo& g, const float* lam, const GT* gradm, int nt,
                    const float* add, float* out, hipStream_t s,
                    const float* dot_with = nullptr, Reducer* red = nullptr, int slot = 0,
                    const PcgDev* als_pd = nullptr, const float* r = nullptr,
                    float* als = nullptr);
// float16 copy of grad m^j for the mixed-precision matvec
int launch_to_half(const float* x, __half* y, long long n, hipStream_t s);

// one RK2 step of the deformation-gradient transport from gathered F_y, G_y
// (Fy NULL: F^0 = I); F may alias Fy
int launch_defgrad_update(const Geo& g, const float* Fy, const float* Gy, const float* G,
                          float* F, double ht, hipStream_t s);
int launch_det(const Geo& g, const float* F, double* det, hipStream_t s);

// --------------------------------------------------------- reductions
// Device partial buffer + pinned host landing zone for float64 scalars.
struct Reducer {
    double* partial = nullptr;   // [max(4 kRedBlocks, one per 256 voxels)]
    double* result = nullptr;    // [8] device
    double* host = nullptr;      // [8] pinned, mapped host memory: the last fold of each slot
    double* mirror = nullptr;    // device address of `host`
};
constexpr int kRedBlocks = 1024;

// Sum of v over a 256-thread block (sh: 4 doubles of LDS); every thread
// receives the total.
__device__ __forceinline__ double block_sum_256(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double t = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return t;
}

int reducer_init(Reducer& r, long long n);
void reducer_free(Reducer& r);

// Enqueue reductions; results land in r.result[slot]. fetch() copies
// r.result to r.host and synchronises the stream.
int red_dot(Reducer& r, const float* a, const float* b, long long n, int slot, hipStream_t s);
int red_sumsq_diff(Reducer& r, const float* a, const float* b, long long n, int slot,
                   hipStream_t s);
int red_absmax(Reducer& r, const float* a, long long n, int slot, hipStream_t s);
int red_sum(Reducer& r, const float* a, long long n, int slot, hipStream_t s);
// min, sum, max and count of non-positive values of a float64 array -> slots 0..3
int red_stats_f64(Reducer& r, const double* a, long long n, hipStream_t s);
int red_fetch(Reducer& r, hipStream_t s);
// fold nb partial sums (r.partial[i*stride + off]) into r.result[slot]
int red_fold_sum(Reducer& r, int nb, int stride, int off, int slot, hipStream_t s);
// r -= kappa Hs with kappa from the device slots (no v~ update), the same
// reductions as pcg_update
int pcg_update_dev(Reducer& red, const float* hs, float* r, const PcgDev& pd, long long n,
                   int smax, int ssum, hipStream_t st);
// v~ += kappa sd, sd = z + mu sd and als_a = (r_a - mean_a) + mu als_a with
// the device scalars
int launch_pcg_direction_dev(const float* z, float* sd, float* vt, const PcgDev& pd,
                             long long n, hipStream_t s);
int launch_als_update_dev(const float* r, float* als, const PcgDev& pd, long long n,
                          hipStream_t s);
// PCG residual update r -= kappa Hs on [3][n] vectors (16-byte aligned, n a
// multiple of 4), fused with the reductions of the new residual: max |r| ->
// slot smax, sum of each component of r -> slots ssum..ssum+2
int pcg_update(Reducer& red, const float* hs, float* r, float kappa, long long n, int smax,
               int ssum, hipStream_t st);

// ------------------------------------------- two-level preconditioner
// Coarse grid (half the extents) of the two-level zero-velocity
// preconditioner, its transforms, the restricted grad m(1) and the vectors of
// the inner CG (each [3][n_c]).
struct TwoLevel {
    Geo gc{};
    SpectralWork swc;
    Reducer red;
    float* gm = nullptr;   // Q_R F_L grad m(1)
    float* b = nullptr;    // restricted right-hand side
    float* x = nullptr;    // inner CG iterate
    float* r = nullptr;
    float* p = nullptr;
    float* q = nullptr;
    float* y = nullptr;    // scratch of the coarse operator
    bool ready = false;
};
constexpr int kMaxInner = 200;

int twolevel_init(TwoLevel& T, const Geo& gf);
void twolevel_free(TwoLevel& T);
// restrict grad m(1) ([3][n] on the fine grid) to the coarse grid
int twolevel_setup(TwoLevel& T, const Geo& gf, SpectralWork& swf, const float* gradm,
                   hipStream_t s);
// z = P r ([3][n] each, may not alias); the inner CG stops at ||r_c|| <=
// inner_rtol ||b_c|| or after max_inner iterations (count in *inner_its).
// Synchronises the stream once per inner iteration.
int twolevel_apply(TwoLevel& T, const Geo& gf, SpectralWork& swf, const float* r, float* z,
                   double alpha, int pw, double inner_rtol, int max_inner, int* inner_its,
                   hipStream_t s);

// ------------------------------------------------------- vector updates
// y = a*x + y
int launch_axpy(const float* x, float* y, float a, long long n, hipStream_t s);
// y = x + b*y
int launch_xpby(const float* x, float* y, float b, long long n, hipStream_t s);
// y = x + b*z
int launch_lincomb(const float* x, const float* z, float* y, float b, long long n,
                   hipStream_t s);
int launch_fill(float* y, float value, long long n, hipStream_t s);
// als_a = (r_a - mean[a]) + mu als_a, a = 0..2 (vector fields of 3 components of n)
int launch_als_update(const float* r, float* als, const double mean[3], float mu, long long n,
                      hipStream_t s);
int launch_scale_copy(const float* x, float* y, float a, long long n, hipStream_t s);
int launch_check_finite(const float* x, long long n, int* flag, hipStream_t s);

}  // namespace claire
