// 3D real FFTs and the pseudo-spectral operators built on them
// (Section 2.5.3: Fourier differentiation; Section 2.2: L = (-Laplacian)^p;
// Sections 2.5.5-2.5.6: (alpha L)^{-1}).
//
// Layout: real fields [n1][n2][n3] (x3 contiguous); spectra are half-complex
// [n1][n2][nh], nh = n3/2 + 1, float2.
//
// A spectral operator is five passes over HBM:
//   1. x3 R2C: rows of n3 reals read as n3/2 complex (even + i odd), an
//      n3/2-point complex FFT in LDS, then the split into n3/2 + 1 bins;
//   2. x2 C2C forward on [n2][C] column tiles (C consecutive k3 bins);
//   3. x1: forward C2C, pointwise multiplier, inverse C2C, all on one tile in
//      LDS (the x1 transform completes the 3D spectrum, so the multiplier can
//      be applied there without another round trip);
//   4. x2 C2C inverse;
//   5. x3 C2R: the inverse split, an n3/2-point inverse FFT, interleaved
//      real output, with an optional fused addend.
// Transforms are unnormalised; the 1/(n1 n2 n3) factor is folded into the
// multiplier. 1D FFTs are Stockham autosort, radix 4 (one radix-2 stage for
// odd log2 N), each stage staged through registers so that a single LDS
// buffer suffices. Twiddles come from a float table built on the host in
// double precision.

#include "internal.h"

#include <cmath>
#include <vector>

namespace claire {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxTw = 1024;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by i
__device__ __forceinline__ float2 times_i(float2 a) { return make_float2(-a.y, a.x); }

// exp(DIR * 2 pi i q / T) read from the forward table tw[q] = exp(-2 pi i q / T)
template <int DIR>
__device__ __forceinline__ float2 twiddle(const float2* tw, int q) {
    float2 t = tw[q];
    return DIR < 0 ? t : cconj(t);
}

// One Stockham stage of radix R over nb sequences of length N = 2^logN held
// in LDS. Element e of sequence b sits at buf[b*bs + e*es]. E bounds the
// elements per thread (nb*N <= kThreads*E). BMAJOR: consecutive threads take
// consecutive sequences (column tiles) instead of consecutive butterflies.
template <int R, int DIR, int E, bool BMAJOR>
__device__ __forceinline__ void stockham_stage(float2* buf, int logN, int nb, int bs, int es,
                                               int logNs, const float2* tw, int logT, int tid) {
    constexpr int B = E / R;                  // butterflies per thread
    constexpr int logR = (R == 2) ? 1 : 2;
    const int nbf = (1 << logN) >> logR;      // butterflies per sequence
    const int total = nb * nbf;
    const int Ns = 1 << logNs;
    const int tshift = logT - logNs - logR;
    float2 v[B][R];
    int dst[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const int t = tid + i * kThreads;
        if (t < total) {
            int b, j;
            if (BMAJOR) { b = t % nb; j = t / nb; }
            else        { j = t & (nbf - 1); b = t >> (logN - logR); }
            const int k = j & (Ns - 1);
            const float2* src = buf + b * bs;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = src[(j + r * nbf) * es];
#pragma unroll
            for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], twiddle<DIR>(tw, (r * k) << tshift));
            if (R == 2) {
                const float2 a = v[i][0], c = v[i][1];
                v[i][0] = cadd(a, c);
                v[i][1] = csub(a, c);
            } else {
                const float2 b0 = cadd(v[i][0], v[i][2]);
                const float2 b1 = csub(v[i][0], v[i][2]);
                const float2 b2 = cadd(v[i][1], v[i][3]);
                float2 b3 = csub(v[i][1], v[i][3]);
                // forward: multiply b3 by -i; inverse: by +i
                b3 = (DIR < 0) ? make_float2(b3.y, -b3.x) : make_float2(-b3.y, b3.x);
                v[i][0] = cadd(b0, b2);
                v[i][1] = cadd(b1, b3);
                v[i][2] = csub(b0, b2);
                v[i][3] = csub(b1, b3);
            }
            dst[i] = b * bs + ((j - k) * R + k) * es;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const int t = tid + i * kThreads;
        if (t < total) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[dst[i] + r * Ns * es] = v[i][r];
        }
    }
    __syncthreads();
}

template <int DIR, int E, bool BMAJOR>
__device__ void lds_fft(float2* buf, int logN, int nb, int bs, int es, const float2* tw, int logT,
                        int tid) {
    int logNs = 0;
    if (logN & 1) {
        stockham_stage<2, DIR, E, BMAJOR>(buf, logN, nb, bs, es, 0, tw, logT, tid);
        logNs = 1;
    }
    for (; logNs < logN; logNs += 2)
        stockham_stage<4, DIR, E, BMAJOR>(buf, logN, nb, bs, es, logNs, tw, logT, tid);
}

__device__ __forceinline__ void load_twiddles(float2* tw_s, const float2* __restrict__ tw, int T,
                                              int tid) {
    for (int q = tid; q < T; q += kThreads) tw_s[q] = tw[q];
}

// ---------------------------------------------------------------- pass 1
// rows: n1*n2 rows of n3 reals -> rows of nh bins. Grid (rows/RB, ncomp).
template <int E>
__global__ __launch_bounds__(kThreads) void k_r2c_x3(const float* __restrict__ in,
                                                     float2* __restrict__ out, int l3, int RB,
                                                     long long n, long long nspec,
                                                     const float2* __restrict__ tw, int logT) {
    extern __shared__ float2 smem[];
    float2* tw_s = smem;
    float2* buf = smem + (1 << logT);
    const int tid = threadIdx.x;
    const int n3 = 1 << l3, M = n3 >> 1, nh = M + 1;
    const long long row0 = (long long)blockIdx.x * RB;
    const float2* src = reinterpret_cast<const float2*>(in + blockIdx.y * n) + row0 * M;
    float2* dst = out + blockIdx.y * nspec + row0 * nh;
    load_twiddles(tw_s, tw, 1 << logT, tid);
    for (int e = tid; e < RB * M; e += kThreads) buf[e] = src[e];
    __syncthreads();
    lds_fft<-1, E, false>(buf, l3 - 1, RB, M, 1, tw_s, logT, tid);
    // X[k] = (Z[k] + conj Z[M-k])/2 - (i/2) w^k (Z[k] - conj Z[M-k]), w = exp(-2 pi i / n3)
    const int tsh = logT - l3;
    for (int e = tid; e < RB * nh; e += kThreads) {
        const int r = e / nh, k = e - r * nh;
        const float2* z = buf + r * M;
        const float2 zk = z[k & (M - 1)];
        const float2 zc = cconj(z[(M - k) & (M - 1)]);
        const float2 ev = cscale(cadd(zk, zc), 0.5f);
        const float2 od = cscale(csub(zk, zc), 0.5f);
        const float2 w = tw_s[k << tsh];
        // -(i) * w * od
        const float2 wo = cmul(w, od);
        dst[e] = make_float2(ev.x + wo.y, ev.y - wo.x);
    }
}

// ---------------------------------------------------------------- pass 5
// rows of nh bins -> rows of n3 reals (x n3, unnormalised), + optional add.
template <int E>
__global__ __launch_bounds__(kThreads) void k_c2r_x3(const float2* __restrict__ in,
                                                     float* __restrict__ out,
                                                     const float* __restrict__ add, int l3,
                                                     int RB, long long n, long long nspec,
                                                     const float2* __restrict__ tw, int logT) {
    extern __shared__ float2 smem[];
    float2* tw_s = smem;
    float2* buf = smem + (1 << logT);
    const int tid = threadIdx.x;
    const int n3 = 1 << l3, M = n3 >> 1, nh = M + 1;
    const long long row0 = (long long)blockIdx.x * RB;
    const float2* src = in + blockIdx.y * nspec + row0 * nh;
    load_twiddles(tw_s, tw, 1 << logT, tid);
    __syncthreads();
    // Z[k] = (X[k] + conj X[M-k]) + i conj(w^k) (X[k] - conj X[M-k]); the
    // imaginary parts of the DC and Nyquist bins are ignored (real signal).
    const int tsh = logT - l3;
    for (int e = tid; e < RB * M; e += kThreads) {
        const int r = e >> (l3 - 1), k = e & (M - 1);
        const float2* x = src + (long long)r * nh;
        float2 xk = x[k];
        float2 xm = x[M - k];
        if (k == 0) { xk.y = 0.f; xm.y = 0.f; }
        const float2 xc = cconj(xm);
        const float2 s = cadd(xk, xc);
        const float2 d = csub(xk, xc);
        const float2 w = cconj(tw_s[k << tsh]);
        buf[e] = cadd(s, times_i(cmul(w, d)));
    }
    __syncthreads();
    lds_fft<+1, E, false>(buf, l3 - 1, RB, M, 1, tw_s, logT, tid);
    float2* dst = reinterpret_cast<float2*>(out + blockIdx.y * n) + row0 * M;
    const float2* ad = add ? reinterpret_cast<const float2*>(add + blockIdx.y * n) + row0 * M : nullptr;
    for (int e = tid; e < RB * M; e += kThreads) {
        float2 val = buf[e];
        if (ad) { const float2 a = ad[e]; val.x += a.x; val.y += a.y; }
        dst[e] = val;
    }
}

// ------------------------------------------------------- passes 2 and 4
// Column tiles: element (r, c) of a tile at data[blockIdx.y*ystride + r*stride
// + c0 + c], r < 2^logN, c < C, c0 + c < nh. Grid (ceil(nh/C), outer, ncomp).
template <int DIR, int E>
__global__ __launch_bounds__(kThreads) void k_c2c_cols(float2* __restrict__ data, int logN, int C,
                                                       long long stride, long long ystride,
                                                       int nh, long long nspec,
                                                       const float2* __restrict__ tw, int logT) {
    extern __shared__ float2 smem[];
    float2* tw_s = smem;
    float2* buf = smem + (1 << logT);
    const int tid = threadIdx.x;
    const int N = 1 << logN;
    const int c0 = blockIdx.x * C;
    const int cw = min(C, nh - c0);
    float2* base = data + blockIdx.z * nspec + blockIdx.y * ystride + c0;
    load_twiddles(tw_s, tw, 1 << logT, tid);
    for (int e = tid; e < N * C; e += kThreads) {
        const int r = e / C, c = e - r * C;
        buf[e] = (c < cw) ? base[r * stride + c] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    lds_fft<DIR, E, true>(buf, logN, C, 1, C, tw_s, logT, tid);
    for (int e = tid; e < N * C; e += kThreads) {
        const int r = e / C, c = e - r * C;
        if (c < cw) base[r * stride + c] = buf[e];
    }
}

// ---------------------------------------------------------------- pass 3
struct Mult {
    int n1, n2, n3;
    float alpha;   // regularisation weight
    int p;         // power of |k|^2
    float norm;    // 1 / (n1 n2 n3)
};

__device__ __forceinline__ int signed_k(int i, int n) { return i < (n >> 1) ? i : i - n; }

// i k_a with the Nyquist wavenumber of that axis removed, times norm
__device__ __forceinline__ float deriv_k(int i, int n) {
    return (i == (n >> 1)) ? 0.f : (float)signed_k(i, n);
}

__device__ __forceinline__ float reg_symbol(const Mult& m, int k1, int k2, int k3) {
    const float kk = (float)(k1 * k1 + k2 * k2) + (float)(k3 * k3);
    return m.p == 1 ? kk : kk * kk;
}

// MODE: SPEC_REG / SPEC_REG_INV (per component, grid z = component),
// SPEC_GRAD (1 -> 3), SPEC_DIV (3 -> 1). Column tiles along x1 for fixed k2.
template <int MODE, int E>
__global__ __launch_bounds__(kThreads) void k_x1_fused(const float2* __restrict__ in,
                                                       float2* __restrict__ out, int l1, int C,
                                                       int nh, long long nspec, Mult m,
                                                       const float2* __restrict__ tw, int logT) {
    extern __shared__ float2 smem[];
    float2* tw_s = smem;
    float2* A = smem + (1 << logT);
    float2* B = A + ((MODE == SPEC_GRAD || MODE == SPEC_DIV) ? (1 << l1) * C : 0);
    const int tid = threadIdx.x;
    const int N = 1 << l1;
    const int k2i = blockIdx.y;
    const int c0 = blockIdx.x * C;
    const int cw = min(C, nh - c0);
    const long long stride = (long long)m.n2 * nh;
    const long long off = (long long)k2i * nh + c0;
    const int k2 = signed_k(k2i, m.n2);
    load_twiddles(tw_s, tw, 1 << logT, tid);

    auto load_tile = [&](float2* dstb, const float2* src) {
        for (int e = tid; e < N * C; e += kThreads) {
            const int r = e / C, c = e - r * C;
            dstb[e] = (c < cw) ? src[off + r * stride + c] : make_float2(0.f, 0.f);
        }
    };
    auto store_tile = [&](const float2* srcb, float2* dstp) {
        for (int e = tid; e < N * C; e += kThreads) {
            const int r = e / C, c = e - r * C;
            if (c < cw) dstp[off + r * stride + c] = srcb[e];
        }
    };

    if (MODE == SPEC_REG || MODE == SPEC_REG_INV) {
        const int comp = blockIdx.z;
        load_tile(A, in + comp * nspec);
        __syncthreads();
        lds_fft<-1, E, true>(A, l1, C, 1, C, tw_s, logT, tid);
        for (int e = tid; e < N * C; e += kThreads) {
            const int r = e / C, c = e - r * C;
            const float sym = reg_symbol(m, signed_k(r, m.n1), k2, c0 + c);
            float f;
            if (MODE == SPEC_REG) f = m.norm * m.alpha * sym;
            else f = (sym == 0.f) ? m.norm : m.norm / (m.alpha * sym);
            A[e] = cscale(A[e], f);
        }
        __syncthreads();
        lds_fft<+1, E, true>(A, l1, C, 1, C, tw_s, logT, tid);
        store_tile(A, out + comp * nspec);
    } else if (MODE == SPEC_GRAD) {
        load_tile(A, in);
        __syncthreads();
        lds_fft<-1, E, true>(A, l1, C, 1, C, tw_s, logT, tid);
        const float kd2 = deriv_k(k2i, m.n2);
        for (int a = 0; a < 3; ++a) {
            for (int e = tid; e < N * C; e += kThreads) {
                const int r = e / C, c = e - r * C;
                float ka;
                if (a == 0) ka = deriv_k(r, m.n1);
                else if (a == 1) ka = kd2;
                else ka = deriv_k(c0 + c, m.n3);
                B[e] = cscale(times_i(A[e]), ka * m.norm);
            }
            __syncthreads();
            lds_fft<+1, E, true>(B, l1, C, 1, C, tw_s, logT, tid);
            store_tile(B, out + a * nspec);
            __syncthreads();
        }
    } else {  // SPEC_DIV
        const float kd2 = deriv_k(k2i, m.n2);
        for (int a = 0; a < 3; ++a) {
            load_tile(B, in + a * nspec);
            __syncthreads();
            lds_fft<-1, E, true>(B, l1, C, 1, C, tw_s, logT, tid);
            for (int e = tid; e < N * C; e += kThreads) {
                const int r = e / C, c = e - r * C;
                float ka;
                if (a == 0) ka = deriv_k(r, m.n1);
                else if (a == 1) ka = kd2;
                else ka = deriv_k(c0 + c, m.n3);
                const float2 t = cscale(times_i(B[e]), ka * m.norm);
                A[e] = (a == 0) ? t : cadd(A[e], t);
            }
            __syncthreads();
        }
        lds_fft<+1, E, true>(A, l1, C, 1, C, tw_s, logT, tid);
        store_tile(A, out);
    }
}

// ------------------------------------------------------------- host side
// Kernels whose dynamic LDS exceeds the 64 KiB default opt in to the larger
// gfx950 allocation (160 KiB per CU).
template <typename K>
int allow_lds(K kernel, size_t bytes) {
    if (bytes > 65536)
        CL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return 0;
}

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Column tile width and elements per thread for a transform of length N.
struct TileCfg { int C; int E; };
TileCfg tile_cfg(int N, int nh) {
    TileCfg t;
    t.E = (N >= 512) ? 32 : 16;
    t.C = (kThreads * t.E) / N;
    if (t.C > 16) t.C = 16;
    if (t.C > nh) t.C = nh;
    if (t.C < 1) t.C = 1;
    return t;
}

int row_block(int n3, long long rows) {
    // rows per block for the x3 passes: RB * n3/2 <= kThreads * 16
    int M = n3 / 2;
    int RB = (kThreads * 16) / M;
    if (RB < 1) RB = 1;
    while (RB > 1 && rows % RB) RB >>= 1;
    return RB;
}

int fwd_x3(const Geo& g, const SpectralWork& w, const float* in, float2* spec, int ncomp,
           hipStream_t s) {
    const long long rows = (long long)g.n1 * g.n2;
    const int RB = row_block(g.n3, rows);
    const int logT = ilog2(w.tw_n);
    const size_t sh = sizeof(float2) * ((1 << logT) + RB * (g.n3 / 2));
    dim3 grid((unsigned)(rows / RB), ncomp);
    hipLaunchKernelGGL(k_r2c_x3<16>, grid, dim3(kThreads), sh, s, in, spec, g.l3, RB, g.n, g.nspec,
                       w.tw, logT);
    CL_LAUNCH_CHECK();
    return 0;
}

int inv_x3(const Geo& g, const SpectralWork& w, const float2* spec, float* out, const float* add,
           int ncomp, hipStream_t s) {
    const long long rows = (long long)g.n1 * g.n2;
    const int RB = row_block(g.n3, rows);
    const int logT = ilog2(w.tw_n);
    const size_t sh = sizeof(float2) * ((1 << logT) + RB * (g.n3 / 2));
    dim3 grid((unsigned)(rows / RB), ncomp);
    hipLaunchKernelGGL(k_c2r_x3<16>, grid, dim3(kThreads), sh, s, spec, out, add, g.l3, RB, g.n,
                       g.nspec, w.tw, logT);
    CL_LAUNCH_CHECK();
    return 0;
}

template <int DIR>
int cols_x2(const Geo& g, const SpectralWork& w, float2* spec, int ncomp, hipStream_t s) {
    const TileCfg t = tile_cfg(g.n2, g.nh);
    const int logT = ilog2(w.tw_n);
    const size_t sh = sizeof(float2) * ((1 << logT) + (size_t)g.n2 * t.C);
    dim3 grid((g.nh + t.C - 1) / t.C, g.n1, ncomp);
    const long long stride = g.nh, ystride = (long long)g.n2 * g.nh;
    if (t.E == 16) {
        CL_TRY(allow_lds(k_c2c_cols<DIR, 16>, sh));
        hipLaunchKernelGGL((k_c2c_cols<DIR, 16>), grid, dim3(kThreads), sh, s, spec, g.l2, t.C,
                           stride, ystride, g.nh, g.nspec, w.tw, logT);
    } else {
        CL_TRY(allow_lds(k_c2c_cols<DIR, 32>, sh));
        hipLaunchKernelGGL((k_c2c_cols<DIR, 32>), grid, dim3(kThreads), sh, s, spec, g.l2, t.C,
                           stride, ystride, g.nh, g.nspec, w.tw, logT);
    }
    CL_LAUNCH_CHECK();
    return 0;
}

template <int MODE>
int fused_x1(const Geo& g, const SpectralWork& w, const float2* in, float2* out, Mult m,
             int ncomp, hipStream_t s) {
    const TileCfg t = tile_cfg(g.n1, g.nh);
    const int logT = ilog2(w.tw_n);
    const int tiles = (MODE == SPEC_GRAD || MODE == SPEC_DIV) ? 2 : 1;
    const size_t sh = sizeof(float2) * ((1 << logT) + (size_t)tiles * g.n1 * t.C);
    dim3 grid((g.nh + t.C - 1) / t.C, g.n2, ncomp);
    if (t.E == 16) {
        CL_TRY(allow_lds(k_x1_fused<MODE, 16>, sh));
        hipLaunchKernelGGL((k_x1_fused<MODE, 16>), grid, dim3(kThreads), sh, s, in, out, g.l1, t.C,
                           g.nh, g.nspec, m, w.tw, logT);
    } else {
        CL_TRY(allow_lds(k_x1_fused<MODE, 32>, sh));
        hipLaunchKernelGGL((k_x1_fused<MODE, 32>), grid, dim3(kThreads), sh, s, in, out, g.l1, t.C,
                           g.nh, g.nspec, m, w.tw, logT);
    }
    CL_LAUNCH_CHECK();
    return 0;
}

}  // namespace

int spectral_init(SpectralWork& w, const Geo& g) {
    int T = g.n1;
    if (g.n2 > T) T = g.n2;
    if (g.n3 > T) T = g.n3;
    if (T > kMaxTw) {
        set_error("grid extent %d exceeds the FFT limit %d", T, kMaxTw);
        return CLAIRE_EINVAL;
    }
    w.tw_n = T;
    std::vector<float2> h(T);
    for (int q = 0; q < T; ++q) {
        const double a = -2.0 * M_PI * (double)q / (double)T;
        h[q] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    CL_HIP(hipMalloc(&w.tw, sizeof(float2) * T));
    CL_HIP(hipMemcpy(w.tw, h.data(), sizeof(float2) * T, hipMemcpyHostToDevice));
    CL_HIP(hipMalloc(&w.spec, sizeof(float2) * 3 * g.nspec));
    return 0;
}

void spectral_free(SpectralWork& w) {
    if (w.tw) (void)hipFree(w.tw);
    if (w.spec) (void)hipFree(w.spec);
    w.tw = nullptr;
    w.spec = nullptr;
}

int spectral_apply(const Geo& g, SpectralWork& w, SpecMode mode, const float* in, float* out,
                   double alpha, int p, hipStream_t s, const float* add) {
    Mult m;
    m.n1 = g.n1;
    m.n2 = g.n2;
    m.n3 = g.n3;
    m.alpha = (float)alpha;
    m.p = p;
    m.norm = (float)(1.0 / ((double)g.n1 * g.n2 * g.n3));
    float2* S = w.spec;
    switch (mode) {
    case SPEC_GRAD:
        CL_TRY(fwd_x3(g, w, in, S, 1, s));
        CL_TRY(cols_x2<-1>(g, w, S, 1, s));
        // output a = 0 overwrites the input tile only after it was loaded
        CL_TRY(fused_x1<SPEC_GRAD>(g, w, S, S, m, 1, s));
        CL_TRY(cols_x2<+1>(g, w, S, 3, s));
        CL_TRY(inv_x3(g, w, S, out, add, 3, s));
        break;
    case SPEC_DIV:
        CL_TRY(fwd_x3(g, w, in, S, 3, s));
        CL_TRY(cols_x2<-1>(g, w, S, 3, s));
        CL_TRY(fused_x1<SPEC_DIV>(g, w, S, S, m, 1, s));
        CL_TRY(cols_x2<+1>(g, w, S, 1, s));
        CL_TRY(inv_x3(g, w, S, out, add, 1, s));
        break;
    case SPEC_REG:
        CL_TRY(fwd_x3(g, w, in, S, 3, s));
        CL_TRY(cols_x2<-1>(g, w, S, 3, s));
        CL_TRY(fused_x1<SPEC_REG>(g, w, S, S, m, 3, s));
        CL_TRY(cols_x2<+1>(g, w, S, 3, s));
        CL_TRY(inv_x3(g, w, S, out, add, 3, s));
        break;
    case SPEC_REG_INV:
        CL_TRY(fwd_x3(g, w, in, S, 3, s));
        CL_TRY(cols_x2<-1>(g, w, S, 3, s));
        CL_TRY(fused_x1<SPEC_REG_INV>(g, w, S, S, m, 3, s));
        CL_TRY(cols_x2<+1>(g, w, S, 3, s));
        CL_TRY(inv_x3(g, w, S, out, add, 3, s));
        break;
    default:
        set_error("unknown spectral mode %d", (int)mode);
        return CLAIRE_EINVAL;
    }
    return 0;
}

}  // namespace claire
