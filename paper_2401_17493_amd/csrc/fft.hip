// 3D real FFTs and the pseudo-spectral operators built on them
// (Section 2.5.3: Fourier differentiation; Section 2.2: L = (-Laplacian)^p;
// Sections 2.5.5-2.5.6: (alpha L)^{-1}).
//
// Layout: real fields [n1][n2][n3] (x3 contiguous); spectra are half-complex
// [n1][n2][hp], nh = n3/2 + 1 bins per row padded to a pitch hp of whole
// 128-byte lines (16 complex), so that the column passes' row segments are
// line-aligned.
//
// A spectral operator is five passes over HBM:
//   1. x3 R2C: rows of n3 reals read as n3/2 complex (even + i odd), an
//      n3/2-point complex FFT in LDS, then the split into n3/2 + 1 bins;
//   2. x2 C2C forward on [n2][C] column tiles (C consecutive k3 bins);
//   3. x1: forward C2C, pointwise multiplier, inverse C2C, all on one tile in
//      LDS (the x1 transform completes the 3D spectrum, so the multiplier is
//      applied there without another round trip);
//   4. x2 C2C inverse;
//   5. x3 C2R: the inverse split, an n3/2-point inverse FFT, interleaved
//      real output, with an optional fused addend.
// Transforms are unnormalised; 1/(n1 n2 n3) is folded into the multiplier.
// 1D FFTs are Stockham autosort, radix 4 (one radix-2 stage for odd log2 N);
// each stage goes through registers so a single LDS buffer suffices.
// Twiddles come from tables built on the host in double precision.
//
// General extents (n1, n2 even products of 2, 3 and 5; n3 a power of two):
// the x3 passes are the same; the x2 and x1 column transforms are
// mixed-radix Stockham stages (radix 4, 2, 3, 5) between two LDS buffers, and
// the multiplier is a separate pointwise pass over the full spectrum.
//
// Precision. The multiplier alpha |k|^{2p} of L amplifies the forward
// transform's round-off at high wavenumbers by up to (k_max/k_data)^{2p}; in
// float32 that reaches 1e-4..1e-2 of the result for smooth fields. The
// forward half of L (passes 1-2 and the forward part of pass 3, and the
// multiplication) therefore runs in float64; the inverse half, whose
// round-off is not amplified, stays float32. Gradient, divergence and
// (alpha L)^{-1} (multipliers |k|, |k|, |k|^{-2p}) are float32 throughout.

#include "internal.h"

#include <cmath>
#include <vector>

namespace claire {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxTw = 1024;

// ----------------------------------------------------- complex arithmetic
template <typename C> struct RealOf;
template <> struct RealOf<float2> { using T = float; };
template <> struct RealOf<double2> { using T = double; };

template <typename C>
__device__ __forceinline__ C cx(typename RealOf<C>::T x, typename RealOf<C>::T y) {
    C r;
    r.x = x;
    r.y = y;
    return r;
}
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    return cx<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return cx<C>(a.x + b.x, a.y + b.y); }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return cx<C>(a.x - b.x, a.y - b.y); }
template <typename C>
__device__ __forceinline__ C cconj(C a) { return cx<C>(a.x, -a.y); }
template <typename C>
__device__ __forceinline__ C cscale(C a, typename RealOf<C>::T s) { return cx<C>(a.x * s, a.y * s); }
template <typename C>
__device__ __forceinline__ C times_i(C a) { return cx<C>(-a.y, a.x); }

// exp(DIR * 2 pi i q / T) read from the forward table tw[q] = exp(-2 pi i q / T)
template <int DIR, typename C>
__device__ __forceinline__ C twiddle(const C* tw, int q) {
    const C t = tw[q];
    return DIR < 0 ? t : cconj(t);
}

// One Stockham stage of radix R over nb sequences of length N = 2^logN held
// in LDS. Element e of sequence b sits at buf[b*bs + e*es]. E bounds the
// elements per thread (nb*N <= kThreads*E). BMAJOR: consecutive threads take
// consecutive sequences (column tiles) instead of consecutive butterflies.
template <int R, int DIR, int E, bool BMAJOR, typename C>
__device__ __forceinline__ void stockham_stage(C* buf, int logN, int nb, int bs, int es, int logNs,
                                               const C* tw, int logT, int tid) {
    constexpr int B = E / R;                  // butterflies per thread
    constexpr int logR = (R == 2) ? 1 : 2;
    const int nbf = (1 << logN) >> logR;      // butterflies per sequence
    const int total = nb * nbf;
    const int Ns = 1 << logNs;
    const int tshift = logT - logNs - logR;
    C v[B][R];
    int dst[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const int t = tid + i * kThreads;
        if (t < total) {
            int b, j;
            // B-major batches (column tiles) come in powers of two
            if (BMAJOR) { b = t & (nb - 1); j = t >> (31 - __clz(nb)); }
            else        { j = t & (nbf - 1); b = t >> (logN - logR); }
            const int k = j & (Ns - 1);
            const C* src = buf + b * bs;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = src[(j + r * nbf) * es];
#pragma unroll
            for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], twiddle<DIR>(tw, (r * k) << tshift));
            if (R == 2) {
                const C a = v[i][0], c = v[i][1];
                v[i][0] = cadd(a, c);
                v[i][1] = csub(a, c);
            } else {
                const C b0 = cadd(v[i][0], v[i][2]);
                const C b1 = csub(v[i][0], v[i][2]);
                const C b2 = cadd(v[i][1], v[i][3]);
                C b3 = csub(v[i][1], v[i][3]);
                // forward: multiply b3 by -i; inverse: by +i
                b3 = (DIR < 0) ? cx<C>(b3.y, -b3.x) : cx<C>(-b3.y, b3.x);
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

template <int DIR, int E, bool BMAJOR, typename C>
__device__ __forceinline__ void lds_fft(C* buf, int logN, int nb, int bs, int es, const C* tw, int logT, int tid) {
    int logNs = 0;
    if (logN & 1) {
        stockham_stage<2, DIR, E, BMAJOR>(buf, logN, nb, bs, es, 0, tw, logT, tid);
        logNs = 1;
    }
    for (; logNs < logN; logNs += 2)
        stockham_stage<4, DIR, E, BMAJOR>(buf, logN, nb, bs, es, logNs, tw, logT, tid);
}

template <typename C>
__device__ __forceinline__ void load_twiddles(C* tw_s, const C* __restrict__ tw, int T, int tid) {
    for (int q = tid; q < T; q += kThreads) tw_s[q] = tw[q];
}

// Copy `total` (<= kThreads*E) values into LDS: all of a thread's loads are
// issued before any store, so their latencies overlap.
template <int E, typename C, typename F>
__device__ __forceinline__ void stage(C* buf, int total, int tid, F load) {
    C tmp[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int e = tid + i * kThreads;
        if (e < total) tmp[i] = load(e);
    }
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int e = tid + i * kThreads;
        if (e < total) buf[e] = tmp[i];
    }
}

// ---------------------------------------------------------------- pass 1
// n1*n2 rows of n3 reals -> rows of nh bins in precision C. Grid (rows/RB, ncomp).
template <int E, typename C>
__global__ __launch_bounds__(kThreads) void k_r2c_x3(const float* __restrict__ in,
                                                     C* __restrict__ out, int l3, int RB,
                                                     long long n, long long nspec,
                                                     const C* __restrict__ tw, int logT) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* tw_s = reinterpret_cast<C*>(smem_raw);
    C* buf = tw_s + (1 << logT);
    using R = typename RealOf<C>::T;
    const int tid = threadIdx.x;
    const int n3 = 1 << l3, M = n3 >> 1, nh = M + 1, hp = spec_pitch(nh);
    const long long row0 = (long long)blockIdx.x * RB;
    const float2* src = reinterpret_cast<const float2*>(in + blockIdx.y * n) + row0 * M;
    C* dst = out + blockIdx.y * nspec + row0 * hp;
    load_twiddles(tw_s, tw, 1 << logT, tid);
    stage<E>(buf, RB * M, tid, [&](int e) {
        const float2 x = src[e];
        return cx<C>((R)x.x, (R)x.y);
    });
    __syncthreads();
    lds_fft<-1, E, false>(buf, l3 - 1, RB, M, 1, tw_s, logT, tid);
    // X[k] = (Z[k] + conj Z[M-k])/2 - (i/2) w^k (Z[k] - conj Z[M-k]), w = exp(-2 pi i / n3)
    const int tsh = logT - l3;
    const float inv_nh = quot_inv(nh);   // RB nh < 2^14 and nh <= 513
    for (int e = tid; e < RB * nh; e += kThreads) {
        int k;
        const int r = quot(e, nh, inv_nh, k);
        const C* z = buf + r * M;
        const C zk = z[k & (M - 1)];
        const C zc = cconj(z[(M - k) & (M - 1)]);
        const C ev = cscale(cadd(zk, zc), (R)0.5);
        const C od = cscale(csub(zk, zc), (R)0.5);
        const C wo = cmul(tw_s[k << tsh], od);
        dst[r * hp + k] = cx<C>(ev.x + wo.y, ev.y - wo.x);   // ev - i * wo
    }
}

// ---------------------------------------------------------------- pass 5
// rows of nh bins -> rows of n3 reals (x n3, unnormalised). AUX = 0: plain;
// AUX = 1: + aux (addend); AUX = 2: also the block's share of <out, aux> in
// float64 -> partial[block]. A thread's aux loads are all issued before its
// first store.
template <int E, int AUX>
__global__ __launch_bounds__(kThreads) void k_c2r_x3(const float2* __restrict__ in,
                                                     float* __restrict__ out,
                                                     const float* __restrict__ aux, int l3,
                                                     int RB, long long n, long long nspec,
                                                     const float2* __restrict__ tw, int logT,
                                                     double* __restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* tw_s = reinterpret_cast<float2*>(smem_raw);
    float2* buf = tw_s + (1 << logT);
    const int tid = threadIdx.x;
    const int n3 = 1 << l3, M = n3 >> 1, hp = spec_pitch(M + 1);
    const long long row0 = (long long)blockIdx.x * RB;
    const float2* src = in + blockIdx.y * nspec + row0 * hp;
    load_twiddles(tw_s, tw, 1 << logT, tid);
    __syncthreads();
    // Z[k] = (X[k] + conj X[M-k]) + i conj(w^k) (X[k] - conj X[M-k]); the
    // imaginary parts of the DC and Nyquist bins are ignored (real signal).
    // A thread takes the pair (k, M-k), 0 < k < M/2, from one load of each
    // bin; k = 0 also takes Z[0] (from X[0], X[M]) and Z[M/2]. All of a
    // thread's loads are issued before its first LDS store.
    const int tsh = logT - l3;
    const int half = M >> 1, lh = l3 - 2;
    auto zval = [&](float2 xk, float2 xm, int k) {
        const float2 xc = cconj(xm);
        const float2 sm = cadd(xk, xc);
        const float2 df = csub(xk, xc);
        const float2 w = cconj(tw_s[k << tsh]);
        return cadd(sm, times_i(cmul(w, df)));
    };
    {
        constexpr int EH = E / 2;
        const int npair = RB * half;
        float2 xa[EH], xb[EH], xh[EH];
#pragma unroll
        for (int i = 0; i < EH; ++i) {
            const int e = tid + i * kThreads;
            if (e < npair) {
                const int r = e >> lh, k = e & (half - 1);
                const float2* x = src + (long long)r * hp;
                xa[i] = x[k];
                xb[i] = x[M - k];
                if (k == 0) xh[i] = x[half];
            }
        }
#pragma unroll
        for (int i = 0; i < EH; ++i) {
            const int e = tid + i * kThreads;
            if (e < npair) {
                const int r = e >> lh, k = e & (half - 1);
                float2* z = buf + r * M;
                if (k == 0) {
                    float2 x0 = xa[i], xn = xb[i];
                    x0.y = 0.f; xn.y = 0.f;
                    z[0] = zval(x0, xn, 0);
                    z[half] = zval(xh[i], xh[i], half);
                } else {
                    z[k] = zval(xa[i], xb[i], k);
                    z[M - k] = zval(xb[i], xa[i], M - k);
                }
            }
        }
    }
    __syncthreads();
    lds_fft<+1, E, false>(buf, l3 - 1, RB, M, 1, tw_s, logT, tid);
    // output rows as 16-byte stores (two complex values of buf each)
    float4* dst = reinterpret_cast<float4*>(out + blockIdx.y * n) + row0 * (M >> 1);
    const float4* b4 = reinterpret_cast<const float4*>(buf);
    const int nq = (RB * M) >> 1;
    double dot = 0.0;
    if (AUX == 0) {
        for (int e = tid; e < nq; e += kThreads) dst[e] = b4[e];
    } else {
        // all of this thread's aux loads in flight at once
        constexpr int EQ = E / 2;
        const float4* ax = reinterpret_cast<const float4*>(aux + blockIdx.y * n) + row0 * (M >> 1);
        float4 pre[EQ];
#pragma unroll
        for (int i = 0; i < EQ; ++i) {
            const int e = tid + i * kThreads;
            if (e < nq) pre[i] = ax[e];
        }
#pragma unroll
        for (int i = 0; i < EQ; ++i) {
            const int e = tid + i * kThreads;
            if (e < nq) {
                float4 val = b4[e];
                if (AUX == 1) {
                    val.x += pre[i].x; val.y += pre[i].y; val.z += pre[i].z; val.w += pre[i].w;
                }
                dst[e] = val;
                if (AUX == 2)
                    dot += ((double)val.x * pre[i].x + (double)val.y * pre[i].y) +
                           ((double)val.z * pre[i].z + (double)val.w * pre[i].w);
            }
        }
    }
    if (AUX == 2) {
        __shared__ double sh[4];
        const double t = block_sum_256(dot, sh);
        if (tid == 0) partial[(long long)blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
}

// ------------------------------------------------------- passes 2 and 4
// Column tiles: element (r, c) of a tile at data[blockIdx.y*ystride + r*stride
// + c0 + c], r < 2^logN, c < C, c0 + c < nh. Grid (ceil(nh/C), outer, ncomp).
template <int DIR, int E, typename C>
__global__ __launch_bounds__(kThreads) void k_c2c_cols(C* __restrict__ data, int logN, int CW,
                                                       long long stride, long long ystride,
                                                       int nh, long long nspec,
                                                       const C* __restrict__ tw, int logT) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* tw_s = reinterpret_cast<C*>(smem_raw);
    C* buf = tw_s + (1 << logT);
    const int tid = threadIdx.x;
    const int lcw = 31 - __clz(CW);   // CW is a power of two
    const int N = 1 << logN;
    const int c0 = blockIdx.x * CW;
    const int cw = min(CW, nh - c0);
    C* base = data + blockIdx.z * nspec + blockIdx.y * ystride + c0;
    load_twiddles(tw_s, tw, 1 << logT, tid);
    stage<E>(buf, N * CW, tid, [&](int e) {
        const int r = e >> lcw, c = e & (CW - 1);
        return (c < cw) ? base[r * stride + c] : cx<C>(0, 0);
    });
    __syncthreads();
    lds_fft<DIR, E, true>(buf, logN, CW, 1, CW, tw_s, logT, tid);
    for (int e = tid; e < N * CW; e += kThreads) {
        const int r = e >> lcw, c = e & (CW - 1);
        if (c < cw) base[r * stride + c] = buf[e];
    }
}

// ---------------------------------------------------------------- pass 3
struct Mult {
    int n1, n2, n3;
    double alpha;   // regularisation weight
    int p;          // power of |k|^2
    double norm;    // 1 / (n1 n2 n3)
    int hp;         // row pitch of the spectrum
};

__device__ __forceinline__ int signed_k(int i, int n) { return i < (n >> 1) ? i : i - n; }

// Block coordinates of an x1 column-tile launch, grid (column blocks, n2,
// components), reordered so that each of the 8 XCDs (which receive workgroups
// round-robin in dispatch order) sweeps one contiguous range of (column block,
// row, component): the two 8-column tiles that share each 128-byte line of a
// spectrum row then run on the same XCD, close in time, and the line is
// fetched from HBM once instead of once per L2. Grids whose size is not a
// multiple of 8 keep the plain order.
struct TileXYZ { int x, y, z; };
__device__ __forceinline__ TileXYZ xcd_tile() {
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned total = gx * gy * gridDim.z;
    unsigned w = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    if ((total & 7u) == 0) w = (w & 7u) * (total >> 3) + (w >> 3);
    TileXYZ t;
    const unsigned q = w / gx;
    t.x = (int)(w - q * gx);
    t.z = (int)(q / gy);
    t.y = (int)(q - (unsigned)t.z * gy);
    return t;
}

// wavenumber of an odd derivative: the Nyquist index of the axis maps to 0
__device__ __forceinline__ float deriv_k(int i, int n) {
    return (i == (n >> 1)) ? 0.f : (float)signed_k(i, n);
}

__device__ __forceinline__ double reg_symbol(int p, int k1, int k2, int k3) {
    const double kk = (double)(k1 * k1 + k2 * k2 + k3 * k3);
    return p == 1 ? kk : kk * kk;
}

// alpha L in float64: the forward transform along x1 and the multiplier in
// double, then the tile is narrowed to float for the inverse transform.
// Input double spectrum (3 components, grid z), output float spectrum.
template <int E>
__global__ __launch_bounds__(kThreads) void k_x1_reg64(const double2* __restrict__ in,
                                                       float2* __restrict__ out, int l1, int CW,
                                                       int nh, long long nspec, Mult m,
                                                       const double2* __restrict__ tw64,
                                                       const float2* __restrict__ tw32, int logT) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double2* tw_d = reinterpret_cast<double2*>(smem_raw);
    float2* tw_f = reinterpret_cast<float2*>(tw_d + (1 << logT));
    double2* A = reinterpret_cast<double2*>(tw_f + (1 << logT));
    float2* Af = reinterpret_cast<float2*>(A);   // same storage, narrowed in place
    const int tid = threadIdx.x;
    const int lcw = 31 - __clz(CW);   // CW is a power of two
    const int N = 1 << l1;
    const TileXYZ bt = xcd_tile();
    const int c0 = bt.x * CW;
    const int cw = min(CW, nh - c0);
    const long long stride = (long long)m.n2 * m.hp;
    const long long off = bt.z * nspec + (long long)bt.y * m.hp + c0;
    const int k2 = signed_k(bt.y, m.n2);
    load_twiddles(tw_d, tw64, 1 << logT, tid);
    load_twiddles(tw_f, tw32, 1 << logT, tid);
    stage<E>(A, N * CW, tid, [&](int e) {
        const int r = e >> lcw, c = e & (CW - 1);
        return (c < cw) ? in[off + r * stride + c] : make_double2(0.0, 0.0);
    });
    __syncthreads();
    lds_fft<-1, E, true>(A, l1, CW, 1, CW, tw_d, logT, tid);
    // multiply in double, narrow to float: read all, barrier, write all
    constexpr int PER = E;
    float2 keep[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = tid + i * kThreads;
        if (e < N * CW) {
            const int r = e >> lcw, c = e & (CW - 1);
            const double f = m.norm * m.alpha * reg_symbol(m.p, signed_k(r, m.n1), k2, c0 + c);
            const double2 a = A[e];
            keep[i] = make_float2((float)(a.x * f), (float)(a.y * f));
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = tid + i * kThreads;
        if (e < N * CW) Af[e] = keep[i];
    }
    __syncthreads();
    lds_fft<+1, E, true>(Af, l1, CW, 1, CW, tw_f, logT, tid);
    for (int e = tid; e < N * CW; e += kThreads) {
        const int r = e >> lcw, c = e & (CW - 1);
        if (c < cw) out[off + r * stride + c] = Af[e];
    }
}

// float32 multipliers: SPEC_REG_INV, SPEC_REG_ISQRT and SPEC_REG32 (per
// component, grid z = component), SPEC_GRAD (1 -> 3), SPEC_DIV (3 -> 1). Column tiles along x1 for fixed k2.
template <int MODE, int E>
__global__ __launch_bounds__(kThreads) void k_x1_fused(const float2* __restrict__ in,
                                                       float2* __restrict__ out, int l1, int CW,
                                                       int nh, long long nspec, Mult m,
                                                       const float2* __restrict__ tw, int logT) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* tw_s = reinterpret_cast<float2*>(smem_raw);
    float2* A = tw_s + (1 << logT);
    float2* B = A + ((MODE == SPEC_GRAD || MODE == SPEC_DIV) ? (1 << l1) * CW : 0);
    const int tid = threadIdx.x;
    const int lcw = 31 - __clz(CW);   // CW is a power of two
    const int N = 1 << l1;
    const TileXYZ bt = xcd_tile();
    const int k2i = bt.y;
    const int c0 = bt.x * CW;
    const int cw = min(CW, nh - c0);
    const long long stride = (long long)m.n2 * m.hp;
    const long long off = (long long)k2i * m.hp + c0;
    const int k2 = signed_k(k2i, m.n2);
    const float norm = (float)m.norm;
    load_twiddles(tw_s, tw, 1 << logT, tid);

    auto load_tile = [&](float2* dstb, const float2* src) {
        stage<E>(dstb, N * CW, tid, [&](int e) {
            const int r = e >> lcw, c = e & (CW - 1);
            return (c < cw) ? src[off + r * stride + c] : make_float2(0.f, 0.f);
        });
    };
    auto store_tile = [&](const float2* srcb, float2* dstp) {
        for (int e = tid; e < N * CW; e += kThreads) {
            const int r = e >> lcw, c = e & (CW - 1);
            if (c < cw) dstp[off + r * stride + c] = srcb[e];
        }
    };

    if (MODE == SPEC_REG_INV || MODE == SPEC_REG_ISQRT || MODE == SPEC_REG32) {
        const int comp = bt.z;
        load_tile(A, in + comp * nspec);
        __syncthreads();
        lds_fft<-1, E, true>(A, l1, CW, 1, CW, tw_s, logT, tid);
        const float alpha = (float)m.alpha;
        for (int e = tid; e < N * CW; e += kThreads) {
            const int r = e >> lcw, c = e & (CW - 1);
            const float sym = (float)reg_symbol(m.p, signed_k(r, m.n1), k2, c0 + c);
            float f;
            if (MODE == SPEC_REG32) f = norm * alpha * sym;
            else
                f = (sym == 0.f) ? norm
                                 : (MODE == SPEC_REG_INV ? norm / (alpha * sym)
                                                         : norm / sqrtf(alpha * sym));
            A[e] = cscale(A[e], f);
        }
        __syncthreads();
        lds_fft<+1, E, true>(A, l1, CW, 1, CW, tw_s, logT, tid);
        store_tile(A, out + comp * nspec);
    } else if (MODE == SPEC_GRAD) {
        load_tile(A, in);
        __syncthreads();
        lds_fft<-1, E, true>(A, l1, CW, 1, CW, tw_s, logT, tid);
        const float kd2 = deriv_k(k2i, m.n2);
        for (int a = 0; a < 3; ++a) {
            for (int e = tid; e < N * CW; e += kThreads) {
                const int r = e >> lcw, c = e & (CW - 1);
                float ka;
                if (a == 0) ka = deriv_k(r, m.n1);
                else if (a == 1) ka = kd2;
                else ka = deriv_k(c0 + c, m.n3);
                B[e] = cscale(times_i(A[e]), ka * norm);
            }
            __syncthreads();
            lds_fft<+1, E, true>(B, l1, CW, 1, CW, tw_s, logT, tid);
            store_tile(B, out + a * nspec);
            __syncthreads();
        }
    } else {  // SPEC_DIV
        const float kd2 = deriv_k(k2i, m.n2);
        for (int a = 0; a < 3; ++a) {
            load_tile(B, in + a * nspec);
            __syncthreads();
            lds_fft<-1, E, true>(B, l1, CW, 1, CW, tw_s, logT, tid);
            for (int e = tid; e < N * CW; e += kThreads) {
                const int r = e >> lcw, c = e & (CW - 1);
                float ka;
                if (a == 0) ka = deriv_k(r, m.n1);
                else if (a == 1) ka = kd2;
                else ka = deriv_k(c0 + c, m.n3);
                const float2 t = cscale(times_i(B[e]), ka * norm);
                A[e] = (a == 0) ? t : cadd(A[e], t);
            }
            __syncthreads();
        }
        lds_fft<+1, E, true>(A, l1, CW, 1, CW, tw_s, logT, tid);
        store_tile(A, out);
    }
}

// Coupled multipliers of the near-incompressible model (3 -> 3): the three
// component tiles of one x1 column block sit in LDS together, so each mode
// mixes its components in one pass. With q = k_d . F (k_d the odd-derivative
// wavenumbers, Nyquist 0; |k|^2 the full symbol):
//   NI_PROJECT: F - M k_d q / |k|^2, M = beta a / (alpha + beta a),
//               a = 1/|k|^2 + 1 (grad M Delta^{-1} div subtracted);
//   NI_PENALTY: beta a k_d q (the operator -grad beta (-Delta^{-1} + id) div);
// both 0 on the coupled part at k = 0.
template <int CM, int E>
__global__ __launch_bounds__(kThreads) void k_x1_coupled(float2* __restrict__ data, int l1,
                                                         int CW, int nh, long long nspec,
                                                         Mult m, float beta,
                                                         const float2* __restrict__ tw,
                                                         int logT) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* tw_s = reinterpret_cast<float2*>(smem_raw);
    float2* T = tw_s + (1 << logT);
    const int tid = threadIdx.x;
    const int lcw = 31 - __clz(CW);   // CW is a power of two
    const int N = 1 << l1;
    const int tile = N * CW;
    const TileXYZ bt = xcd_tile();
    const int k2i = bt.y;
    const int c0 = bt.x * CW;
    const int cw = min(CW, nh - c0);
    const long long stride = (long long)m.n2 * m.hp;
    const long long off = (long long)k2i * m.hp + c0;
    const float norm = (float)m.norm;
    const float alpha = (float)m.alpha;
    load_twiddles(tw_s, tw, 1 << logT, tid);
    for (int a = 0; a < 3; ++a) {
        const float2* src = data + a * nspec;
        stage<E>(T + a * tile, tile, tid, [&](int e) {
            const int r = e >> lcw, c = e & (CW - 1);
            return (c < cw) ? src[off + r * stride + c] : make_float2(0.f, 0.f);
        });
    }
    __syncthreads();
    for (int a = 0; a < 3; ++a) lds_fft<-1, E, true>(T + a * tile, l1, CW, 1, CW, tw_s, logT, tid);
    const int k2 = signed_k(k2i, m.n2);
    const float kd2 = deriv_k(k2i, m.n2);
    for (int e = tid; e < tile; e += kThreads) {
        const int r = e >> lcw, c = e & (CW - 1);
        const int k1 = signed_k(r, m.n1), k3 = c0 + c;
        const float kd1 = deriv_k(r, m.n1), kd3 = deriv_k(k3, m.n3);
        const float kk = (float)(k1 * k1 + k2 * k2 + k3 * k3);
        const float2 t0 = T[e], t1 = T[tile + e], t2 = T[2 * tile + e];
        const float2 q = make_float2(kd1 * t0.x + kd2 * t1.x + kd3 * t2.x,
                                     kd1 * t0.y + kd2 * t1.y + kd3 * t2.y);
        float s1, s2 = 0.f;
        if (CM == NI_PROJECT) {
            s1 = norm;
            if (kk > 0.f) {
                const float ba = beta * (1.f / kk + 1.f);
                s2 = -norm * (ba / (alpha + ba)) / kk;
            }
        } else {
            s1 = 0.f;
            if (kk > 0.f) s2 = norm * beta * (1.f / kk + 1.f);
        }
        T[e] = make_float2(s1 * t0.x + s2 * kd1 * q.x, s1 * t0.y + s2 * kd1 * q.y);
        T[tile + e] = make_float2(s1 * t1.x + s2 * kd2 * q.x, s1 * t1.y + s2 * kd2 * q.y);
        T[2 * tile + e] = make_float2(s1 * t2.x + s2 * kd3 * q.x, s1 * t2.y + s2 * kd3 * q.y);
    }
    __syncthreads();
    for (int a = 0; a < 3; ++a) {
        float2* buf = T + a * tile;
        lds_fft<+1, E, true>(buf, l1, CW, 1, CW, tw_s, logT, tid);
        float2* dst = data + a * nspec;
        for (int e = tid; e < tile; e += kThreads) {
            const int r = e >> lcw, c = e & (CW - 1);
            if (c < cw) dst[off + r * stride + c] = buf[e];
        }
    }
}

// ------------------------------------------------------- general extents
// Radices of a mixed-radix transform in stage order.
struct RadixPlan {
    int N;
    int ns;
    int R[16];
};

// Radix-R DFT y_m = sum_r x_r exp(DIR 2 pi i r m / R) of registers x, R in
// {2, 3, 4, 5}.
template <int R, int DIR, typename C>
__device__ __forceinline__ void small_dft(const C* x, C* y) {
    using T = typename RealOf<C>::T;
    if constexpr (R == 2) {
        y[0] = cadd(x[0], x[1]);
        y[1] = csub(x[0], x[1]);
    } else if constexpr (R == 4) {
        const C b0 = cadd(x[0], x[2]), b1 = csub(x[0], x[2]);
        const C b2 = cadd(x[1], x[3]);
        C b3 = csub(x[1], x[3]);
        b3 = (DIR < 0) ? cx<C>(b3.y, -b3.x) : cx<C>(-b3.y, b3.x);
        y[0] = cadd(b0, b2);
        y[1] = cadd(b1, b3);
        y[2] = csub(b0, b2);
        y[3] = csub(b1, b3);
    } else {
        // cos/sin of 2 pi q / R for q < R
        T cs[R], sn[R];
        if constexpr (R == 3) {
            cs[0] = T(1); sn[0] = T(0);
            cs[1] = T(-0.5); sn[1] = T(0.86602540378443864676);
            cs[2] = T(-0.5); sn[2] = T(-0.86602540378443864676);
        } else {
            cs[0] = T(1); sn[0] = T(0);
            cs[1] = T(0.30901699437494742410); sn[1] = T(0.95105651629515357212);
            cs[2] = T(-0.80901699437494742410); sn[2] = T(0.58778525229247312917);
            cs[3] = T(-0.80901699437494742410); sn[3] = T(-0.58778525229247312917);
            cs[4] = T(0.30901699437494742410); sn[4] = T(-0.95105651629515357212);
        }
#pragma unroll
        for (int m = 0; m < R; ++m) {
            C acc = x[0];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int q = (r * m) % R;
                const C w = cx<C>(cs[q], DIR < 0 ? -sn[q] : sn[q]);
                acc = cadd(acc, cmul(x[r], w));
            }
            y[m] = acc;
        }
    }
}

// One Stockham stage on CW columns: butterfly j (of N/R per column) reads
// src[j + r N/R], twiddles by exp(DIR 2 pi i r k / (Ns R)), k = j mod Ns, and
// writes dst[(j - k) R + k + m Ns]. Element e of row q is at q CW + column.
template <int R, int DIR, typename C>
__device__ __forceinline__ void stage_gen(const C* src, C* dst, int N, int CW, int Ns,
                                          const C* tw, int tid) {
    const int M = N / R;
    const int tstep = N / (Ns * R);
    const int lcw = 31 - __clz(CW);        // CW is a power of two
    const float inv_ns = quot_inv(Ns);     // j < N <= 1024, Ns <= 1024
    for (int t = tid; t < M * CW; t += kThreads) {
        const int j = t >> lcw, col = t & (CW - 1);
        int k;
        (void)quot(j, Ns, inv_ns, k);      // k = j mod Ns
        C x[R], y[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            C v = src[(j + r * M) * CW + col];
            if (r > 0) {
                C w = tw[r * k * tstep];
                if (DIR > 0) w.y = -w.y;
                v = cmul(v, w);
            }
            x[r] = v;
        }
        small_dft<R, DIR>(x, y);
        const int o = (j - k) * R + k;
#pragma unroll
        for (int m = 0; m < R; ++m) dst[(o + m * Ns) * CW + col] = y[m];
    }
}

// Multiplier applied inside an x1 column pass (general grids): 0 none,
// 1 (alpha |k|^{2p})^{-1}, 2 (alpha |k|^{2p})^{-1/2}, both 1 at k = 0, times norm.
struct ColMult {
    int n2;            // x2 extent (blockIdx.y is the x2 index)
    double alpha, norm;
    int p;
};

template <int DIR, typename C, int MULT>
__device__ __forceinline__ void stages_gen(C*& src, C*& dst, int N, int CW, const C* tw_s,
                                           const RadixPlan& plan, int tid) {
    int Ns = 1;
    for (int st = 0; st < plan.ns; ++st) {
        const int R = plan.R[st];
        if (R == 4) stage_gen<4, DIR>(src, dst, N, CW, Ns, tw_s, tid);
        else if (R == 2) stage_gen<2, DIR>(src, dst, N, CW, Ns, tw_s, tid);
        else if (R == 3) stage_gen<3, DIR>(src, dst, N, CW, Ns, tw_s, tid);
        else stage_gen<5, DIR>(src, dst, N, CW, Ns, tw_s, tid);
        __syncthreads();
        C* t = src;
        src = dst;
        dst = t;
        Ns *= R;
    }
}

// Column transforms of length N = plan.N along an axis with element stride
// `stride`; tiles of CW consecutive half-complex x3 bins, one tile row per
// blockIdx.y (ystride apart), component blockIdx.z. With MULT (x1 axis,
// float only) the tile is transformed forward, multiplied and transformed
// back in LDS.
template <int DIR, typename C, int MULT>
__global__ __launch_bounds__(kThreads) void k_cols_gen(C* __restrict__ data, int CW,
                                                       long long stride, long long ystride,
                                                       int nh, long long nspec,
                                                       const C* __restrict__ tw,
                                                       RadixPlan plan, ColMult cm) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int N = plan.N;
    C* tw_s = reinterpret_cast<C*>(smem_raw);
    C* A = tw_s + N;
    C* B = A + N * CW;
    const int tid = threadIdx.x;
    const int lcw = 31 - __clz(CW);   // CW is a power of two
    const TileXYZ bt = xcd_tile();
    const int c0 = bt.x * CW;
    const int cw = min(CW, nh - c0);
    C* base = data + bt.z * nspec + bt.y * ystride + c0;
    for (int q = tid; q < N; q += kThreads) tw_s[q] = tw[q];
    for (int e = tid; e < N * CW; e += kThreads) {
        const int r = e >> lcw, c = e & (CW - 1);
        A[e] = (c < cw) ? base[r * stride + c] : cx<C>(0, 0);
    }
    __syncthreads();
    C* src = A;
    C* dst = B;
    if constexpr (MULT == 0) {
        stages_gen<DIR, C, 0>(src, dst, N, CW, tw_s, plan, tid);
    } else {
        stages_gen<-1, C, 0>(src, dst, N, CW, tw_s, plan, tid);
        const int k2 = signed_k(bt.y, cm.n2);
        const float alpha = (float)cm.alpha, norm = (float)cm.norm;
        for (int e = tid; e < N * CW; e += kThreads) {
            const int r = e >> lcw, c = e & (CW - 1);
            // in float, as in the power-of-two x1 pass
            const float sym = alpha * (float)reg_symbol(cm.p, signed_k(r, N), k2, c0 + c);
            const float f = (sym == 0.f) ? norm
                            : (MULT == 1 ? norm / sym : norm / sqrtf(sym));
            src[e] = cscale(src[e], f);
        }
        __syncthreads();
        stages_gen<+1, C, 0>(src, dst, N, CW, tw_s, plan, tid);
    }
    for (int e = tid; e < N * CW; e += kThreads) {
        const int r = e >> lcw, c = e & (CW - 1);
        if (c < cw) base[r * stride + c] = src[e];
    }
}

// Pointwise multiplier on a full spectrum (general grids): GRAD 1 -> 3,
// DIV 3 -> 1, REG (from the double spectrum) and the coupled
// near-incompressible modes; in place on S. (alpha L)^{-1} and its square
// root are fused into the x1 column pass instead.
enum GenMult { GM_GRAD, GM_DIV, GM_REG, GM_REG_INV, GM_REG_ISQRT, GM_NI_PROJECT, GM_NI_PENALTY };

template <int MODE>
__global__ __launch_bounds__(kThreads) void k_mult_gen(float2* __restrict__ S,
                                                       const double2* __restrict__ S64,
                                                       int n1, int n2, int n3, int nh,
                                                       long long nspec, double alpha, int p,
                                                       double beta, double norm) {
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= nspec) return;
    const unsigned hp = (unsigned)spec_pitch(nh);
    // nspec < 2^32 (extents <= 1024): 32-bit index arithmetic
    const unsigned u = (unsigned)idx;
    const unsigned r = u / hp;
    const int i3 = (int)(u - r * hp);
    if (i3 >= nh) return;   // row padding
    const unsigned r1 = r / (unsigned)n2;
    const int i2 = (int)(r - r1 * (unsigned)n2);
    const int i1 = (int)r1;
    const int k1 = signed_k(i1, n1), k2 = signed_k(i2, n2), k3 = i3;
    const float kd[3] = {deriv_k(i1, n1), deriv_k(i2, n2), deriv_k(i3, n3)};
    const float nf = (float)norm;
    if (MODE == GM_GRAD) {
        const float2 a = S[idx];
#pragma unroll
        for (int c = 0; c < 3; ++c) S[c * nspec + idx] = cscale(times_i(a), kd[c] * nf);
    } else if (MODE == GM_DIV) {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int c = 0; c < 3; ++c) acc = cadd(acc, cscale(times_i(S[c * nspec + idx]), kd[c] * nf));
        S[idx] = acc;
    } else if (MODE == GM_REG) {
        const double f = norm * alpha * reg_symbol(p, k1, k2, k3);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double2 a = S64[c * nspec + idx];
            S[c * nspec + idx] = make_float2((float)(a.x * f), (float)(a.y * f));
        }
    } else {
        const double kk = (double)k1 * k1 + (double)k2 * k2 + (double)k3 * k3;
        float2 t[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) t[c] = S[c * nspec + idx];
        const float2 q = make_float2(kd[0] * t[0].x + kd[1] * t[1].x + kd[2] * t[2].x,
                                     kd[0] * t[0].y + kd[1] * t[1].y + kd[2] * t[2].y);
        float s1, s2 = 0.f;
        if (MODE == GM_NI_PROJECT) {
            s1 = nf;
            if (kk > 0.0) {
                const double ba = beta * (1.0 / kk + 1.0);
                s2 = (float)(-norm * (ba / (alpha + ba)) / kk);
            }
        } else {
            s1 = 0.f;
            if (kk > 0.0) s2 = (float)(norm * beta * (1.0 / kk + 1.0));
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
            S[c * nspec + idx] = make_float2(s1 * t[c].x + s2 * kd[c] * q.x,
                                             s1 * t[c].y + s2 * kd[c] * q.y);
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

// Column tile width for a transform of length N with `elems` complex values
// per tile (E = elems / kThreads per thread).
// The width is a power of two: the column-tile kernels index their tiles
// with shifts and masks.
int tile_cols(int N, int nh, int elems) {
    int C = elems / N;
    if (C > 16) C = 16;
    if (C > nh) C = nh;
    if (C < 1) C = 1;
    while (C & (C - 1)) C &= C - 1;   // round down to a power of two
    return C;
}

int row_block(int n3, long long rows, int elems) {
    // rows per block for the x3 passes: RB * n3/2 <= elems
    const int M = n3 / 2;
    int RB = elems / M;
    if (RB < 1) RB = 1;
    while (RB > 1 && rows % RB) RB >>= 1;
    return RB;
}

// double spectra use half-size tiles (same LDS bytes as float tiles) so that
// several workgroups still fit on a CU
template <typename C>
constexpr int tile_elems() { return sizeof(C) == 8 ? 4096 : 2048; }

template <typename C>
int fwd_x3(const Geo& g, const C* tw, int T, const float* in, C* spec, int ncomp, hipStream_t s) {
    const long long rows = (long long)g.n1 * g.n2;
    const int RB = row_block(g.n3, rows, 2048);
    const int logT = ilog2(T);
    const size_t sh = sizeof(C) * ((1 << logT) + RB * (g.n3 / 2));
    dim3 grid((unsigned)(rows / RB), ncomp);
    if (sizeof(C) == 8) {
        CL_TRY(allow_lds(k_r2c_x3<8, C>, sh));
        hipLaunchKernelGGL((k_r2c_x3<8, C>), grid, dim3(kThreads), sh, s, in, spec, g.l3, RB,
                           g.n, g.nspec, tw, logT);
    } else {
        CL_TRY(allow_lds(k_r2c_x3<8, C>, sh));
        hipLaunchKernelGGL((k_r2c_x3<8, C>), grid, dim3(kThreads), sh, s, in, spec, g.l3, RB,
                           g.n, g.nspec, tw, logT);
    }
    CL_LAUNCH_CHECK();
    return 0;
}

int inv_x3(const Geo& g, const SpectralWork& w, const float2* spec, float* out, const float* add,
           int ncomp, hipStream_t s, const float* dot_with = nullptr, Reducer* red = nullptr,
           int slot = 0) {
    // half-size row blocks (2048 complex values): twice the workgroups in
    // flight, which covers the loads of the addend or dot operand
    const long long rows = (long long)g.n1 * g.n2;
    const int RB = row_block(g.n3, rows, 2048);
    const int logT = ilog2(w.tw_n);
    const size_t sh = sizeof(float2) * ((1 << logT) + RB * (g.n3 / 2));
    dim3 grid((unsigned)(rows / RB), ncomp);
    if (dot_with) {
        CL_TRY(allow_lds(k_c2r_x3<8, 2>, sh));
        hipLaunchKernelGGL((k_c2r_x3<8, 2>), grid, dim3(kThreads), sh, s, spec, out, dot_with,
                           g.l3, RB, g.n, g.nspec, w.tw, logT, red->partial);
        CL_LAUNCH_CHECK();
        return red_fold_sum(*red, (int)(grid.x * grid.y), 1, 0, slot, s);
    }
    if (add) {
        CL_TRY(allow_lds(k_c2r_x3<8, 1>, sh));
        hipLaunchKernelGGL((k_c2r_x3<8, 1>), grid, dim3(kThreads), sh, s, spec, out, add, g.l3,
                           RB, g.n, g.nspec, w.tw, logT, nullptr);
    } else {
        CL_TRY(allow_lds(k_c2r_x3<8, 0>, sh));
        hipLaunchKernelGGL((k_c2r_x3<8, 0>), grid, dim3(kThreads), sh, s, spec, out, nullptr,
                           g.l3, RB, g.n, g.nspec, w.tw, logT, nullptr);
    }
    CL_LAUNCH_CHECK();
    return 0;
}

template <int DIR, int E, typename C>
int cols_launch(const Geo& g, const C* tw, int logT, C* spec, int CW, size_t sh, dim3 grid,
                hipStream_t s) {
    CL_TRY(allow_lds(k_c2c_cols<DIR, E, C>, sh));
    hipLaunchKernelGGL((k_c2c_cols<DIR, E, C>), grid, dim3(kThreads), sh, s, spec, g.l2, CW,
                       (long long)g.hp, (long long)g.n2 * g.hp, g.nh, g.nspec, tw, logT);
    CL_LAUNCH_CHECK();
    return 0;
}

// Column-tile budgets (complex values per workgroup tile) of the x2 pass and
// the fused x1 pass in float: the tile width is budget / n; the elements per
// thread (and so the registers, and the occupancy) follow from it.
#ifndef CLAIRE_FFT_COL_ELEMS
#define CLAIRE_FFT_COL_ELEMS 8192
#endif
#ifndef CLAIRE_FFT_X1_ELEMS
#define CLAIRE_FFT_X1_ELEMS 2048
#endif

template <int DIR, typename C>
int cols_x2(const Geo& g, const C* tw, int T, C* spec, int ncomp, hipStream_t s) {
    // float tiles hold up to CLAIRE_FFT_COL_ELEMS values, double tiles 2048
    constexpr int elems = sizeof(C) == 8 ? CLAIRE_FFT_COL_ELEMS : 2048;
    const int CW = tile_cols(g.n2, g.nh, elems);
    const int logT = ilog2(T);
    const size_t sh = sizeof(C) * ((1 << logT) + (size_t)g.n2 * CW);
    dim3 grid((g.nh + CW - 1) / CW, g.n1, ncomp);
    const int per = (g.n2 * CW + kThreads - 1) / kThreads;
    if (per <= 8) return cols_launch<DIR, 8>(g, tw, logT, spec, CW, sh, grid, s);
    if (per <= 16) return cols_launch<DIR, 16>(g, tw, logT, spec, CW, sh, grid, s);
    return cols_launch<DIR, 32>(g, tw, logT, spec, CW, sh, grid, s);
}

template <int MODE>
int fused_x1(const Geo& g, const float2* tw, int T, const float2* in, float2* out, Mult m,
             int ncomp, hipStream_t s) {
    const int CW = tile_cols(g.n1, g.nh, CLAIRE_FFT_X1_ELEMS);
    const int logT = ilog2(T);
    const int tiles = (MODE == SPEC_GRAD || MODE == SPEC_DIV) ? 2 : 1;
    const size_t sh = sizeof(float2) * ((1 << logT) + (size_t)tiles * g.n1 * CW);
    dim3 grid((g.nh + CW - 1) / CW, g.n2, ncomp);
    if (g.n1 * CW <= 8 * kThreads) {
        CL_TRY(allow_lds(k_x1_fused<MODE, 8>, sh));
        hipLaunchKernelGGL((k_x1_fused<MODE, 8>), grid, dim3(kThreads), sh, s, in, out, g.l1, CW,
                           g.nh, g.nspec, m, tw, logT);
    } else if (g.n1 * CW <= 16 * kThreads) {
        CL_TRY(allow_lds(k_x1_fused<MODE, 16>, sh));
        hipLaunchKernelGGL((k_x1_fused<MODE, 16>), grid, dim3(kThreads), sh, s, in, out, g.l1, CW,
                           g.nh, g.nspec, m, tw, logT);
    } else {
        CL_TRY(allow_lds(k_x1_fused<MODE, 32>, sh));
        hipLaunchKernelGGL((k_x1_fused<MODE, 32>), grid, dim3(kThreads), sh, s, in, out, g.l1, CW,
                           g.nh, g.nspec, m, tw, logT);
    }
    CL_LAUNCH_CHECK();
    return 0;
}

RadixPlan make_plan(int N) {
    RadixPlan p;
    p.N = N;
    p.ns = 0;
    int m = N;
    while (m % 4 == 0) { p.R[p.ns++] = 4; m /= 4; }
    while (m % 2 == 0) { p.R[p.ns++] = 2; m /= 2; }
    while (m % 3 == 0) { p.R[p.ns++] = 3; m /= 3; }
    while (m % 5 == 0) { p.R[p.ns++] = 5; m /= 5; }
    return p;   // m == 1 for extents accepted by make_geo's caller
}

// General-grid column transform along x2 (axis 2) or x1 (axis 1); MULT > 0
// (x1 only): forward, multiplier, inverse in one pass
template <int DIR, typename C, int MULT = 0>
int cols_gen(const Geo& g, int axis, const C* tw, C* spec, int ncomp, hipStream_t s,
             double alpha = 0.0, int p = 1) {
    const int N = axis == 1 ? g.n1 : g.n2;
    // two tiles and the twiddle table within 64 KiB of LDS
    int CW = (int)((65536 / sizeof(C) - N) / (2 * N));
    if (CW > 16) CW = 16;
    if (CW > g.nh) CW = g.nh;
    if (CW < 1) {
        set_error("column length %d exceeds the general-grid FFT tile", N);
        return CLAIRE_EINVAL;
    }
    while (CW & (CW - 1)) CW &= CW - 1;   // a power of two: shift indexing
    const size_t sh = sizeof(C) * ((size_t)N + 2 * (size_t)N * CW);
    const long long stride = axis == 1 ? (long long)g.n2 * g.hp : g.hp;
    const long long ystride = axis == 1 ? g.hp : (long long)g.n2 * g.hp;
    dim3 grid((g.nh + CW - 1) / CW, axis == 1 ? g.n2 : g.n1, ncomp);
    ColMult cm;
    cm.n2 = g.n2;
    cm.alpha = alpha;
    cm.norm = 1.0 / ((double)g.n1 * g.n2 * g.n3);
    cm.p = p;
    hipLaunchKernelGGL((k_cols_gen<DIR, C, MULT>), grid, dim3(kThreads), sh, s, spec, CW, stride,
                       ystride, g.nh, g.nspec, tw, make_plan(N), cm);
    CL_LAUNCH_CHECK();
    return 0;
}

template <int MODE>
int mult_gen(const Geo& g, SpectralWork& w, double alpha, int p, double beta, hipStream_t s) {
    hipLaunchKernelGGL(k_mult_gen<MODE>, dim3((unsigned)((g.nspec + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, w.spec, w.spec64, g.n1, g.n2, g.n3, g.nh, g.nspec,
                       alpha, p, beta, 1.0 / ((double)g.n1 * g.n2 * g.n3));
    CL_LAUNCH_CHECK();
    return 0;
}

// Spectral operator on a general grid: x3 R2C, x2 and x1 forward columns,
// pointwise multiplier, x1 and x2 inverse columns, x3 C2R (with the addend
// or the fused dot product); for (alpha L)^{-1} and (alpha L)^{-1/2} the x1
// forward, multiplier and x1 inverse are one pass.
template <int DIR>
int cols_x1(const Geo& g, const float2* tw, int T, float2* spec, int ncomp, hipStream_t s);

// Column passes of a general grid: an axis whose extent is a power of two
// takes the power-of-two column kernels (with that axis's own twiddle table),
// the others the mixed-radix ones.
template <int DIR>
int gen_x1(const Geo& g, const SpectralWork& w, float2* S, int ncomp, hipStream_t s) {
    if ((1 << g.l1) == g.n1) return cols_x1<DIR>(g, w.tw1, g.n1, S, ncomp, s);
    return cols_gen<DIR>(g, 1, w.tw1, S, ncomp, s);
}
template <int DIR, typename C>
int gen_x2(const Geo& g, const C* tw2, C* S, int ncomp, hipStream_t s) {
    if ((1 << g.l2) == g.n2) return cols_x2<DIR>(g, tw2, g.n2, S, ncomp, s);
    return cols_gen<DIR>(g, 2, tw2, S, ncomp, s);
}

int spectral_gen(const Geo& g, SpectralWork& w, int mode, const float* in, float* out,
                 double alpha, int p, double beta, hipStream_t s, const float* add,
                 const float* dot_with, Reducer* red, int slot) {
    const int nin = mode == GM_GRAD ? 1 : 3;
    const int nout = mode == GM_DIV ? 1 : 3;
    float2* S = w.spec;
    if (mode == GM_REG_INV || mode == GM_REG_ISQRT) {
        // the multiplier is fused into the x1 pass
        CL_TRY(fwd_x3(g, w.tw, w.tw_n, in, S, 3, s));
        CL_TRY(gen_x2<-1>(g, w.tw2, S, 3, s));
        if ((1 << g.l1) == g.n1) {
            Mult m;
            m.n1 = g.n1;
            m.n2 = g.n2;
            m.n3 = g.n3;
            m.alpha = alpha;
            m.p = p;
            m.norm = 1.0 / ((double)g.n1 * g.n2 * g.n3);
            m.hp = g.hp;
            if (mode == GM_REG_INV)
                CL_TRY(fused_x1<SPEC_REG_INV>(g, w.tw1, g.n1, S, S, m, 3, s));
            else
                CL_TRY(fused_x1<SPEC_REG_ISQRT>(g, w.tw1, g.n1, S, S, m, 3, s));
        } else if (mode == GM_REG_INV) {
            CL_TRY((cols_gen<-1, float2, 1>(g, 1, w.tw1, S, 3, s, alpha, p)));
        } else {
            CL_TRY((cols_gen<-1, float2, 2>(g, 1, w.tw1, S, 3, s, alpha, p)));
        }
        CL_TRY(gen_x2<+1>(g, w.tw2, S, 3, s));
        return inv_x3(g, w, S, out, add, 3, s, dot_with, red, slot);
    }
    if (mode == GM_REG) {
        CL_TRY(fwd_x3(g, w.tw64, w.tw_n, in, w.spec64, 3, s));
        CL_TRY(gen_x2<-1>(g, w.tw2_64, w.spec64, 3, s));
        CL_TRY(cols_gen<-1>(g, 1, w.tw1_64, w.spec64, 3, s));
    } else {
        CL_TRY(fwd_x3(g, w.tw, w.tw_n, in, S, nin, s));
        CL_TRY(gen_x2<-1>(g, w.tw2, S, nin, s));
        CL_TRY(gen_x1<-1>(g, w, S, nin, s));
    }
    switch (mode) {
    case GM_GRAD: CL_TRY(mult_gen<GM_GRAD>(g, w, alpha, p, beta, s)); break;
    case GM_DIV: CL_TRY(mult_gen<GM_DIV>(g, w, alpha, p, beta, s)); break;
    case GM_REG: CL_TRY(mult_gen<GM_REG>(g, w, alpha, p, beta, s)); break;
    case GM_NI_PROJECT: CL_TRY(mult_gen<GM_NI_PROJECT>(g, w, alpha, p, beta, s)); break;
    default: CL_TRY(mult_gen<GM_NI_PENALTY>(g, w, alpha, p, beta, s)); break;
    }
    CL_TRY(gen_x1<+1>(g, w, S, nout, s));
    CL_TRY(gen_x2<+1>(g, w.tw2, S, nout, s));
    return inv_x3(g, w, S, out, add, nout, s, dot_with, red, slot);
}

template <int CM>
int coupled_x1(const Geo& g, const SpectralWork& w, float2* spec, Mult m, double beta,
               hipStream_t s) {
    const int CW = tile_cols(g.n1, g.nh, CLAIRE_FFT_X1_ELEMS);
    const int logT = ilog2(w.tw_n);
    const size_t sh = sizeof(float2) * ((1 << logT) + (size_t)3 * g.n1 * CW);
    dim3 grid((g.nh + CW - 1) / CW, g.n2, 1);
    auto go = [&](auto kern) -> int {
        CL_TRY(allow_lds(kern, sh));
        hipLaunchKernelGGL(kern, grid, dim3(kThreads), sh, s, spec, g.l1, CW, g.nh, g.nspec, m,
                           (float)beta, w.tw, logT);
        CL_LAUNCH_CHECK();
        return 0;
    };
    if (g.n1 * CW <= 8 * kThreads) return go(k_x1_coupled<CM, 8>);
    if (g.n1 * CW <= 16 * kThreads) return go(k_x1_coupled<CM, 16>);
    return go(k_x1_coupled<CM, 32>);
}

int reg_x1(const Geo& g, const SpectralWork& w, const double2* in, float2* out, Mult m,
           hipStream_t s) {
    const int CW = tile_cols(g.n1, g.nh, 2048);
    const int logT = ilog2(w.tw_n);
    const size_t sh = (sizeof(double2) + sizeof(float2)) * (1 << logT) +
                      sizeof(double2) * (size_t)g.n1 * CW;
    dim3 grid((g.nh + CW - 1) / CW, g.n2, 3);
    CL_TRY(allow_lds(k_x1_reg64<8>, sh));
    hipLaunchKernelGGL(k_x1_reg64<8>, grid, dim3(kThreads), sh, s, in, out, g.l1, CW, g.nh,
                       g.nspec, m, w.tw64, w.tw, logT);
    CL_LAUNCH_CHECK();
    return 0;
}

// x1 column pass (rows spaced n2 nh apart, one tile row per x2 index)
template <int DIR>
int cols_x1(const Geo& g, const float2* tw, int T, float2* spec, int ncomp, hipStream_t s) {
    const int CW = tile_cols(g.n1, g.nh, CLAIRE_FFT_COL_ELEMS);
    const int logT = ilog2(T);
    const size_t sh = sizeof(float2) * ((1 << logT) + (size_t)g.n1 * CW);
    dim3 grid((g.nh + CW - 1) / CW, g.n2, ncomp);
    const int per = (g.n1 * CW + kThreads - 1) / kThreads;
    const long long stride = (long long)g.n2 * g.hp, ystride = g.hp;
    auto go = [&](auto kern) -> int {
        CL_TRY(allow_lds(kern, sh));
        hipLaunchKernelGGL(kern, grid, dim3(kThreads), sh, s, spec, g.l1, CW, stride, ystride,
                           g.nh, g.nspec, tw, logT);
        CL_LAUNCH_CHECK();
        return 0;
    };
    if (per <= 8) return go(k_c2c_cols<DIR, 8, float2>);
    if (per <= 16) return go(k_c2c_cols<DIR, 16, float2>);
    return go(k_c2c_cols<DIR, 32, float2>);
}

__device__ __forceinline__ float isqrt_symbol(double alpha, int p, int k1, int k2, int k3) {
    const double sym = alpha * reg_symbol(p, k1, k2, k3);
    return sym == 0.0 ? 1.f : (float)(1.0 / sqrt(sym));
}

// kept by the cut-off filter: |k_a| < n_a^c / 2 on every axis (k3 >= 0)
__device__ __forceinline__ bool kept(int k1, int k2, int k3, int c1, int c2, int c3) {
    return abs(k1) < (c1 >> 1) && abs(k2) < (c2 >> 1) && k3 < (c3 >> 1);
}

__global__ __launch_bounds__(kThreads) void k_spec_restrict(const float2* __restrict__ F,
                                                            float2* __restrict__ C, int f1,
                                                            int f2, int fh, long long fspec,
                                                            int c1, int c2, int c3, int ch,
                                                            long long cspec, int ncomp,
                                                            double alpha, int p, int isqrt,
                                                            float inv_nf) {
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= cspec * ncomp) return;
    const int comp = (int)(idx / cspec);
    const long long e = idx - comp * cspec;
    const int chp = spec_pitch(ch), fhp = spec_pitch(fh);
    const int i3 = (int)(e % chp);
    const int i2 = (int)((e / chp) % c2);
    const int i1 = (int)(e / ((long long)chp * c2));
    const int k1 = signed_k(i1, c1), k2 = signed_k(i2, c2), k3 = i3;
    float2 out = make_float2(0.f, 0.f);
    if (i3 < ch && kept(k1, k2, k3, c1, c2, c3)) {
        const int j1 = (k1 + f1) % f1, j2 = (k2 + f2) % f2;
        const float2 v = F[comp * fspec + ((long long)j1 * f2 + j2) * fhp + k3];
        const float sg = (isqrt ? isqrt_symbol(alpha, p, k1, k2, k3) : 1.f) * inv_nf;
        out = make_float2(v.x * sg, v.y * sg);
    }
    C[idx] = out;
}

__global__ __launch_bounds__(kThreads) void k_spec_combine(float2* __restrict__ F,
                                                           const float2* __restrict__ S, int f1,
                                                           int f2, int fh, long long fspec,
                                                           int c1, int c2, int c3, int ch,
                                                           long long cspec, int ncomp,
                                                           double alpha, int p, float inv_nf,
                                                           float inv_nc) {
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= fspec * ncomp) return;
    const int comp = (int)(idx / fspec);
    const long long e = idx - comp * fspec;
    const int chp = spec_pitch(ch), fhp = spec_pitch(fh);
    const int i3 = (int)(e % fhp);
    if (i3 >= fh) return;   // row padding
    const int i2 = (int)((e / fhp) % f2);
    const int i1 = (int)(e / ((long long)fhp * f2));
    const int k1 = signed_k(i1, f1), k2 = signed_k(i2, f2), k3 = i3;
    const float sg = isqrt_symbol(alpha, p, k1, k2, k3);
    float2 out;
    if (kept(k1, k2, k3, c1, c2, c3)) {
        const int j1 = (k1 + c1) % c1, j2 = (k2 + c2) % c2;
        const float2 v = S[comp * cspec + ((long long)j1 * c2 + j2) * chp + k3];
        out = make_float2(v.x * sg * inv_nc, v.y * sg * inv_nc);
    } else {
        const float2 v = F[idx];
        const float f = sg * sg * inv_nf;
        out = make_float2(v.x * f, v.y * f);
    }
    F[idx] = out;
}

}  // namespace

// exp(-2 pi i q / N), q < N, in float and double
int make_table(int N, float2** tf, double2** td) {
    std::vector<float2> h(N);
    std::vector<double2> hd(N);
    for (int q = 0; q < N; ++q) {
        const double a = -2.0 * M_PI * (double)q / (double)N;
        hd[q] = make_double2(std::cos(a), std::sin(a));
        h[q] = make_float2((float)hd[q].x, (float)hd[q].y);
    }
    CL_HIP(hipMalloc(tf, sizeof(float2) * N));
    CL_HIP(hipMemcpy(*tf, h.data(), sizeof(float2) * N, hipMemcpyHostToDevice));
    CL_HIP(hipMalloc(td, sizeof(double2) * N));
    CL_HIP(hipMemcpy(*td, hd.data(), sizeof(double2) * N, hipMemcpyHostToDevice));
    return 0;
}

int spectral_init(SpectralWork& w, const Geo& g) {
    int T = g.n1;
    if (g.n2 > T) T = g.n2;
    if (g.n3 > T) T = g.n3;
    if (T > kMaxTw) {
        set_error("grid extent %d exceeds the FFT limit %d", T, kMaxTw);
        return CLAIRE_EINVAL;
    }
    if (!g.pow2) {
        // x3 passes index a power-of-two table by shifts; x1 and x2 columns
        // use tables of their own lengths
        T = g.n3;
        CL_TRY(make_table(g.n1, &w.tw1, &w.tw1_64));
        CL_TRY(make_table(g.n2, &w.tw2, &w.tw2_64));
    }
    w.tw_n = T;
    std::vector<float2> h(T);
    std::vector<double2> hd(T);
    for (int q = 0; q < T; ++q) {
        const double a = -2.0 * M_PI * (double)q / (double)T;
        hd[q] = make_double2(std::cos(a), std::sin(a));
        h[q] = make_float2((float)hd[q].x, (float)hd[q].y);
    }
    CL_HIP(hipMalloc(&w.tw, sizeof(float2) * T));
    CL_HIP(hipMemcpy(w.tw, h.data(), sizeof(float2) * T, hipMemcpyHostToDevice));
    CL_HIP(hipMalloc(&w.tw64, sizeof(double2) * T));
    CL_HIP(hipMemcpy(w.tw64, hd.data(), sizeof(double2) * T, hipMemcpyHostToDevice));
    CL_HIP(hipMalloc(&w.spec, sizeof(float2) * 3 * g.nspec));
    CL_HIP(hipMalloc(&w.spec64, sizeof(double2) * 3 * g.nspec));
    return 0;
}

void spectral_free(SpectralWork& w) {
    if (w.tw) (void)hipFree(w.tw);
    if (w.tw64) (void)hipFree(w.tw64);
    if (w.tw1) (void)hipFree(w.tw1);
    if (w.tw1_64) (void)hipFree(w.tw1_64);
    if (w.tw2) (void)hipFree(w.tw2);
    if (w.tw2_64) (void)hipFree(w.tw2_64);
    if (w.spec) (void)hipFree(w.spec);
    if (w.spec64) (void)hipFree(w.spec64);
    w = SpectralWork();
}

int spectral_apply(const Geo& g, SpectralWork& w, SpecMode mode, const float* in, float* out,
                   double alpha, int p, hipStream_t s, const float* add, const float* dot_with,
                   Reducer* red, int slot) {
    if (dot_with && (mode != SPEC_REG_INV || !red || add)) {
        set_error("fused dot product only with SPEC_REG_INV, a reducer and no addend");
        return CLAIRE_EINVAL;
    }
    if (!g.pow2) {
        static const int gm[] = {GM_GRAD, GM_DIV, GM_REG, GM_REG_INV, GM_REG_ISQRT, GM_REG};
        if ((int)mode < 0 || (int)mode > 5) {
            set_error("unknown spectral mode %d", (int)mode);
            return CLAIRE_EINVAL;
        }
        return spectral_gen(g, w, gm[mode], in, out, alpha, p, 0.0, s, add, dot_with, red, slot);
    }
    Mult m;
    m.n1 = g.n1;
    m.n2 = g.n2;
    m.n3 = g.n3;
    m.alpha = alpha;
    m.p = p;
    m.norm = 1.0 / ((double)g.n1 * g.n2 * g.n3);
    m.hp = g.hp;
    float2* S = w.spec;
    switch (mode) {
    case SPEC_GRAD:
        CL_TRY(fwd_x3(g, w.tw, w.tw_n, in, S, 1, s));
        CL_TRY(cols_x2<-1>(g, w.tw, w.tw_n, S, 1, s));
        // output a = 0 overwrites the input tile only after it was loaded
        CL_TRY(fused_x1<SPEC_GRAD>(g, w.tw, w.tw_n, S, S, m, 1, s));
        CL_TRY(cols_x2<+1>(g, w.tw, w.tw_n, S, 3, s));
        CL_TRY(inv_x3(g, w, S, out, add, 3, s));
        break;
    case SPEC_DIV:
        CL_TRY(fwd_x3(g, w.tw, w.tw_n, in, S, 3, s));
        CL_TRY(cols_x2<-1>(g, w.tw, w.tw_n, S, 3, s));
        CL_TRY(fused_x1<SPEC_DIV>(g, w.tw, w.tw_n, S, S, m, 1, s));
        CL_TRY(cols_x2<+1>(g, w.tw, w.tw_n, S, 1, s));
        CL_TRY(inv_x3(g, w, S, out, add, 1, s));
        break;
    case SPEC_REG:
        CL_TRY(fwd_x3(g, w.tw64, w.tw_n, in, w.spec64, 3, s));
        CL_TRY(cols_x2<-1>(g, w.tw64, w.tw_n, w.spec64, 3, s));
        CL_TRY(reg_x1(g, w, w.spec64, S, m, s));
        CL_TRY(cols_x2<+1>(g, w.tw, w.tw_n, S, 3, s));
        CL_TRY(inv_x3(g, w, S, out, add, 3, s));
        break;
    case SPEC_REG32:
        CL_TRY(fwd_x3(g, w.tw, w.tw_n, in, S, 3, s));
        CL_TRY(cols_x2<-1>(g, w.tw, w.tw_n, S, 3, s));
        CL_TRY(fused_x1<SPEC_REG32>(g, w.tw, w.tw_n, S, S, m, 3, s));
        CL_TRY(cols_x2<+1>(g, w.tw, w.tw_n, S, 3, s));
        CL_TRY(inv_x3(g, w, S, out, add, 3, s));
        break;
    case SPEC_REG_INV:
        CL_TRY(fwd_x3(g, w.tw, w.tw_n, in, S, 3, s));
        CL_TRY(cols_x2<-1>(g, w.tw, w.tw_n, S, 3, s));
        CL_TRY(fused_x1<SPEC_REG_INV>(g, w.tw, w.tw_n, S, S, m, 3, s));
        CL_TRY(cols_x2<+1>(g, w.tw, w.tw_n, S, 3, s));
        CL_TRY(inv_x3(g, w, S, out, add, 3, s, dot_with, red, slot));
        break;
    case SPEC_REG_ISQRT:
        CL_TRY(fwd_x3(g, w.tw, w.tw_n, in, S, 3, s));
        CL_TRY(cols_x2<-1>(g, w.tw, w.tw_n, S, 3, s));
        CL_TRY(fused_x1<SPEC_REG_ISQRT>(g, w.tw, w.tw_n, S, S, m, 3, s));
        CL_TRY(cols_x2<+1>(g, w.tw, w.tw_n, S, 3, s));
        CL_TRY(inv_x3(g, w, S, out, add, 3, s));
        break;
    default:
        set_error("unknown spectral mode %d", (int)mode);
        return CLAIRE_EINVAL;
    }
    return 0;
}

int spectral_ni(const Geo& g, SpectralWork& w, NiMode mode, const float* in, float* out,
                double alpha, double beta, hipStream_t s, const float* add,
                const float* dot_with, Reducer* red, int slot) {
    if (dot_with && (!red || add)) {
        set_error("fused dot product needs a reducer and no addend");
        return CLAIRE_EINVAL;
    }
    if (!(beta > 0.0)) {
        set_error("the near-incompressible operators need beta > 0");
        return CLAIRE_EINVAL;
    }
    if (!g.pow2)
        return spectral_gen(g, w, mode == NI_PROJECT ? GM_NI_PROJECT : GM_NI_PENALTY, in, out,
                            alpha, 1, beta, s, add, dot_with, red, slot);
    Mult m;
    m.n1 = g.n1;
    m.n2 = g.n2;
    m.n3 = g.n3;
    m.alpha = alpha;
    m.p = 1;
    m.norm = 1.0 / ((double)g.n1 * g.n2 * g.n3);
    m.hp = g.hp;
    float2* S = w.spec;
    CL_TRY(fwd_x3(g, w.tw, w.tw_n, in, S, 3, s));
    CL_TRY(cols_x2<-1>(g, w.tw, w.tw_n, S, 3, s));
    if (mode == NI_PROJECT) CL_TRY(coupled_x1<NI_PROJECT>(g, w, S, m, beta, s));
    else CL_TRY(coupled_x1<NI_PENALTY>(g, w, S, m, beta, s));
    CL_TRY(cols_x2<+1>(g, w.tw, w.tw_n, S, 3, s));
    return inv_x3(g, w, S, out, add, 3, s, dot_with, red, slot);
}

int spectral_forward(const Geo& g, const SpectralWork& w, const float* in, float2* spec,
                     int ncomp, hipStream_t s) {
    CL_TRY(fwd_x3(g, w.tw, w.tw_n, in, spec, ncomp, s));
    if (!g.pow2) {
        CL_TRY(cols_gen<-1>(g, 2, w.tw2, spec, ncomp, s));
        return cols_gen<-1>(g, 1, w.tw1, spec, ncomp, s);
    }
    CL_TRY(cols_x2<-1>(g, w.tw, w.tw_n, spec, ncomp, s));
    return cols_x1<-1>(g, w.tw, w.tw_n, spec, ncomp, s);
}

int spectral_inverse(const Geo& g, const SpectralWork& w, float2* spec, float* out, int ncomp,
                     hipStream_t s) {
    if (!g.pow2) {
        CL_TRY(cols_gen<+1>(g, 1, w.tw1, spec, ncomp, s));
        CL_TRY(cols_gen<+1>(g, 2, w.tw2, spec, ncomp, s));
    } else {
        CL_TRY(cols_x1<+1>(g, w.tw, w.tw_n, spec, ncomp, s));
        CL_TRY(cols_x2<+1>(g, w.tw, w.tw_n, spec, ncomp, s));
    }
    return inv_x3(g, w, spec, out, nullptr, ncomp, s);
}

int spectral_restrict_modes(const Geo& gf, const Geo& gc, const float2* F, float2* C, int ncomp,
                            double alpha, int p, bool isqrt, hipStream_t s) {
    const long long total = gc.nspec * ncomp;
    hipLaunchKernelGGL(k_spec_restrict, dim3((unsigned)((total + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, F, C, gf.n1, gf.n2, gf.nh, gf.nspec, gc.n1, gc.n2,
                       gc.n3, gc.nh, gc.nspec, ncomp, alpha, p, isqrt ? 1 : 0,
                       (float)(1.0 / (double)gf.n));
    CL_LAUNCH_CHECK();
    return 0;
}

int spectral_combine_modes(const Geo& gf, const Geo& gc, float2* F, const float2* S, int ncomp,
                           double alpha, int p, hipStream_t s) {
    const long long total = gf.nspec * ncomp;
    hipLaunchKernelGGL(k_spec_combine, dim3((unsigned)((total + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, F, S, gf.n1, gf.n2, gf.nh, gf.nspec, gc.n1, gc.n2,
                       gc.n3, gc.nh, gc.nspec, ncomp, alpha, p, (float)(1.0 / (double)gf.n),
                       (float)(1.0 / (double)gc.n));
    CL_LAUNCH_CHECK();
    return 0;
}

}  // namespace claire
