// Learned warm start: a periodic 3D convolutional encoder--decoder trained
// and evaluated on the matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Every 3x3x3 convolution is an implicit GEMM: rows are voxels (M), columns
// output channels (N), the reduction runs over k = t cin + ci (27 taps times
// the input channels, padded to a multiple of 32). Operands are bfloat16,
// accumulation float32. The same kernel runs the backward-data pass with the
// weights flipped in t and transposed in (co, ci); the weight gradient is a
// second GEMM whose reduction runs over voxels, split across workgroups into
// deterministic partial sums. Activations are channels last, batch first.
//
// MFMA 16x16x32 operand layout (lane l, g = l / 16): A row l % 16 holds
// k = 8 g .. 8 g + 7; B column l % 16 holds the same k; the 4 results of a
// lane are rows 4 g + r, column l % 16.

#include "internal.h"

#include "claire_net.h"

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

namespace claire {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr float kLeak = 0.1f;
constexpr int kInC = 8;        // input feature channels
constexpr int kOutC = 3;       // velocity components
constexpr int kLayers = 15;

__device__ __forceinline__ float slope(bf16 y) { return (float)y > 0.f ? 1.f : kLeak; }

// Voxel index of (b, j1, j2, j3) on a 2^l grid.
__device__ __forceinline__ long long vox(int b, int j1, int j2, int j3, int l) {
    return ((long long)b << (3 * l)) | ((long long)j1 << (2 * l)) | ((long long)j2 << l) | j3;
}

// Convolution input: channels [0, ca) from `a` (stored at half resolution
// and read nearest-upsampled when a_up), channels [ca, ca + cb) from `b`.
struct ConvIn {
    const bf16* a;
    int ca, a_up;
    const bf16* b;
    int cb;
};

// Element (voxel (bb, j1, j2, j3) at level l, channel ci) of the input view.
__device__ __forceinline__ const bf16* in_ptr(const ConvIn& in, int l, int bb, int j1, int j2,
                                              int j3, int ci) {
    if (ci < in.ca) {
        if (in.a_up) return in.a + vox(bb, j1 >> 1, j2 >> 1, j3 >> 1, l - 1) * in.ca + ci;
        return in.a + vox(bb, j1, j2, j3, l) * in.ca + ci;
    }
    return in.b + vox(bb, j1, j2, j3, l) * in.cb + (ci - in.ca);
}

enum ConvEpi {
    EPI_ACT = 0,        // y16 = bf16(leaky(acc + bias))
    EPI_LINEAR = 1,     // y32 = acc + bias
    EPI_DGRAD_ACT = 2,  // y16 = bf16(acc * slope(yprev))
    EPI_DGRAD_RAW = 3,  // y32 (channels < csplit) / y32b (the rest) = acc
    EPI_ACT32 = 4,      // y32 = leaky(acc + bias)
};

struct ConvOut {
    bf16* y16;
    float* y32;
    float* y32b;
    int csplit;
    const bf16* yprev;
    const float* bias;
};

// Reduction range of split z of gridDim.z over kpad (multiples of 32), and
// this lane's first (tap, channel) pair k = t cin + ci in it.
__device__ __forceinline__ void conv_krange(int kpad, int cin, int g, int& kc0, int& kc1, int& t,
                                            int& ci) {
    const int ks = kpad >> 5, per = (ks + (int)gridDim.z - 1) / (int)gridDim.z;
    kc0 = min(ks, (int)blockIdx.z * per) << 5;
    kc1 = min(ks, ((int)blockIdx.z + 1) * per) << 5;
    const int k0 = kc0 + 8 * g;
    t = k0 / cin;
    ci = k0 - t * cin;
}

// Implicit-GEMM convolution: each wave computes 16 voxels x 64 output
// channels (4 MFMA tiles), a workgroup 64 voxels; grid (ceil(mtot/64),
// ceil(nrows/64), splits). wt: [nrows][kpad] bfloat16, zero beyond cout rows
// and 27 cin columns; cin = ca + cb and both multiples of 8. With more than
// one split (grids too small to fill the chip) split z sums its share of the
// reduction into part[z][m][nrows] and k_conv_reduce applies the epilogue.
template <int EPI>
__global__ __launch_bounds__(256) void k_conv(ConvIn in, const bf16* __restrict__ wt, int kpad,
                                              int nrows, int cout, int l, int mtot,
                                              ConvOut out, float* __restrict__ part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, li = lane & 15;
    const int mask = (1 << l) - 1;
    const int mbase = (blockIdx.x * 4 + wave) * 16;
    const int n0 = blockIdx.y * 64;
    const int cin = in.ca + in.cb;
    const int m = mbase + li;
    const bool mval = m < mtot;
    const int i3 = m & mask, i2 = (m >> l) & mask, i1 = (m >> (2 * l)) & mask, bb = m >> (3 * l);
    int kc0, kc1, t, ci;
    conv_krange(kpad, cin, g, kc0, kc1, t, ci);
    floatx4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int kc = kc0; kc < kc1; kc += 32) {
        bf16x8 av = {};
        if (mval && t < 27) {
            const int o1 = t / 9 - 1, o2 = (t / 3) % 3 - 1, o3 = t % 3 - 1;
            av = *reinterpret_cast<const bf16x8*>(
                in_ptr(in, l, bb, (i1 + o1) & mask, (i2 + o2) & mask, (i3 + o3) & mask, ci));
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int r0 = n0 + nt * 16;
            if (r0 < nrows) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8*>(
                    wt + (size_t)(r0 + li) * kpad + kc + 8 * g);
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nt], 0, 0, 0);
            }
        }
        ci += 32;
        while (ci >= cin) { ci -= cin; ++t; }
    }
    if (gridDim.z > 1) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int co = n0 + nt * 16 + li;
            if (n0 + nt * 16 >= nrows) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int mo = mbase + 4 * g + r;
                if (mo < mtot)
                    part[((size_t)blockIdx.z * mtot + mo) * nrows + co] = acc[nt][r];
            }
        }
        return;
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int co = n0 + nt * 16 + li;
        if (n0 + nt * 16 >= nrows || co >= cout) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int mo = mbase + 4 * g + r;
            if (mo >= mtot) continue;
            const float a = acc[nt][r];
            if (EPI == EPI_ACT) {
                const float z = a + (out.bias ? out.bias[co] : 0.f);
                out.y16[(size_t)mo * cout + co] = (bf16)(z > 0.f ? z : kLeak * z);
            } else if (EPI == EPI_LINEAR) {
                out.y32[(size_t)mo * cout + co] = a + (out.bias ? out.bias[co] : 0.f);
            } else if (EPI == EPI_ACT32) {
                const float z = a + (out.bias ? out.bias[co] : 0.f);
                out.y32[(size_t)mo * cout + co] = z > 0.f ? z : kLeak * z;
            } else if (EPI == EPI_DGRAD_ACT) {
                out.y16[(size_t)mo * cout + co] = (bf16)(a * slope(out.yprev[(size_t)mo * cout + co]));
            } else {
                if (co < out.csplit) out.y32[(size_t)mo * out.csplit + co] = a;
                else out.y32b[(size_t)mo * (cout - out.csplit) + (co - out.csplit)] = a;
            }
        }
    }
}

// Output element of a convolution tile (shared by both convolution kernels).
template <int EPI>
__device__ __forceinline__ void conv_store(const ConvOut& out, int cout, long long mo, int co,
                                           float a) {
    if (EPI == EPI_ACT) {
        const float z = a + (out.bias ? out.bias[co] : 0.f);
        out.y16[(size_t)mo * cout + co] = (bf16)(z > 0.f ? z : kLeak * z);
    } else if (EPI == EPI_LINEAR) {
        out.y32[(size_t)mo * cout + co] = a + (out.bias ? out.bias[co] : 0.f);
    } else if (EPI == EPI_ACT32) {
        const float z = a + (out.bias ? out.bias[co] : 0.f);
        out.y32[(size_t)mo * cout + co] = z > 0.f ? z : kLeak * z;
    } else if (EPI == EPI_DGRAD_ACT) {
        out.y16[(size_t)mo * cout + co] = (bf16)(a * slope(out.yprev[(size_t)mo * cout + co]));
    } else {
        if (co < out.csplit) out.y32[(size_t)mo * out.csplit + co] = a;
        else out.y32b[(size_t)mo * (cout - out.csplit) + (co - out.csplit)] = a;
    }
}

// Halo-staged implicit GEMM for grids of at least 4^3: a workgroup owns a
// 4 x 4 x 4 brick of one batch item (64 voxels, 16 per wave) and 64 output
// channels. The brick's periodic 6 x 6 x 6 neighbourhood with all cin input
// channels is copied into LDS once (16-byte loads through the same input
// view as k_conv: concatenation and nearest upsampling), and the A
// fragments of all 27 taps are read from there: each input value is fetched
// from global memory ~3.4 times per brick instead of 27 times per voxel.
// Same K order (k = t cin + ci), MFMA and epilogues as k_conv.
constexpr int kHaloPos = 216;
constexpr int kHaloMaxC = 144;                 // input channels the LDS tile may hold (62 KB)
template <int EPI>
__global__ __launch_bounds__(256) void k_conv_halo(ConvIn in, const bf16* __restrict__ wt,
                                                   int kpad, int nrows, int cout, int l,
                                                   ConvOut out, float* __restrict__ part) {
    extern __shared__ __align__(16) bf16 halo[];   // [216][cin]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, li = lane & 15;
    const int mask = (1 << l) - 1;
    const int lb = l - 2;                      // log2 of bricks per axis
    const int bid = blockIdx.x;
    const int o3 = (bid & ((1 << lb) - 1)) << 2;
    const int o2 = ((bid >> lb) & ((1 << lb) - 1)) << 2;
    const int o1 = ((bid >> (2 * lb)) & ((1 << lb) - 1)) << 2;
    const int bb = bid >> (3 * lb);
    const int n0 = blockIdx.y * 64;
    const int cin = in.ca + in.cb;
    const int c8 = cin >> 3;                   // 16-byte channel groups per voxel
    // stage the neighbourhood: position p = (a, b, c) in 6^3, voxel o + (a, b, c) - 1
    for (int e = threadIdx.x; e < kHaloPos * c8; e += 256) {
        const int p = e / c8, cg = e - p * c8;
        const int a = p / 36, b = (p / 6) % 6, c = p % 6;
        const bf16x8 v = *reinterpret_cast<const bf16x8*>(
            in_ptr(in, l, bb, (o1 + a - 1) & mask, (o2 + b - 1) & mask, (o3 + c - 1) & mask,
                   8 * cg));
        *reinterpret_cast<bf16x8*>(halo + p * cin + 8 * cg) = v;
    }
    __syncthreads();
    // this lane's A row: brick voxel (wave, li / 4, li % 4)
    const int prow = wave * 36 + (li >> 2) * 6 + (li & 3);
    int kc0, kc1, t, ci;
    conv_krange(kpad, cin, g, kc0, kc1, t, ci);
    floatx4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int kc = kc0; kc < kc1; kc += 32) {
        bf16x8 av = {};
        if (t < 27) {
            const int pt = (t / 9) * 36 + ((t / 3) % 3) * 6 + t % 3;
            av = *reinterpret_cast<const bf16x8*>(halo + (prow + pt) * cin + ci);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int r0 = n0 + nt * 16;
            if (r0 < nrows) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8*>(
                    wt + (size_t)(r0 + li) * kpad + kc + 8 * g);
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nt], 0, 0, 0);
            }
        }
        ci += 32;
        while (ci >= cin) { ci -= cin; ++t; }
    }
    // results: rows 4 g + r of the wave's 16 voxels = brick voxel (wave, g, r)
    if (gridDim.z > 1) {
        const long long mtot = (long long)gridDim.x << 6;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int co = n0 + nt * 16 + li;
            if (n0 + nt * 16 >= nrows) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                part[((size_t)blockIdx.z * mtot + vox(bb, o1 + wave, o2 + g, o3 + r, l)) * nrows +
                     co] = acc[nt][r];
        }
        return;
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int co = n0 + nt * 16 + li;
        if (n0 + nt * 16 >= nrows || co >= cout) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            conv_store<EPI>(out, cout, vox(bb, o1 + wave, o2 + g, o3 + r, l), co, acc[nt][r]);
    }
}

// Narrow layers (at most 16 x NG output columns, NG <= 6, e.g. the 16-channel layers at
// the network's finest level): a workgroup owns a 4x4x16 voxel brick; wave w
// takes its x1 plane w as four rows of 16 x3 voxels, four MFMA tiles along
// the voxels that share each weight fragment, so one 16-byte weight load
// feeds four MFMAs instead of one, and each A fragment read from LDS feeds
// the NG column groups. The 6x6x18 neighbourhood of all input channels is
// staged in LDS once. Same fragments and summation order per output as
// k_conv_halo.
constexpr int kNarrowPos = 6 * 6 * 18;
constexpr int kNarrowMaxC = 48;                // input channels staged at a time (62 KB)
constexpr int kNarrowMaxNG = 6;                // column groups of 16
template <int EPI, int NG>
__global__ __launch_bounds__(256) void k_conv_narrow(ConvIn in, const bf16* __restrict__ wt,
                                                     int kpad, int cout, int l, ConvOut out,
                                                     int cst) {
    extern __shared__ __align__(16) bf16 halo[];   // [648][cst]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, li = lane & 15;
    const int mask = (1 << l) - 1;
    const int lb = l - 2, lb3 = l - 4;             // log2 of bricks along x1, x2 and along x3
    int bid = blockIdx.x;
    const int o3 = (bid & ((1 << lb3) - 1)) << 4;
    bid >>= lb3;
    const int o2 = (bid & ((1 << lb) - 1)) << 2;
    bid >>= lb;
    const int o1 = (bid & ((1 << lb) - 1)) << 2;
    const int bb = bid >> lb;
    const int cin = in.ca + in.cb;
    // cst channels are staged at a time (a divisor of cin, a multiple of 8);
    // with cst < cin the reduction runs chunk by chunk, each over its taps
    // and channels
    const int c8 = cst >> 3;                       // 16-byte channel groups per voxel
    const int ksc = (27 * cst + 31) & ~31;         // reduction steps of a chunk x 32
    floatx4 acc[NG][4];
#pragma unroll
    for (int gi = 0; gi < NG; ++gi)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[gi][mt] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int q0 = 0; q0 < cin; q0 += cst) {
        if (q0) __syncthreads();   // the previous chunk's fragments have been read
        // stage the neighbourhood: position p = (a, b, c) in 6 x 6 x 18, voxel
        // o + (a, b, c) - 1, channels q0 .. q0 + cst - 1
        for (int e = threadIdx.x; e < kNarrowPos * c8; e += 256) {
            const int p = e / c8, cg = e - p * c8;
            const int a = p / 108, b = (p / 18) % 6, c = p % 18;
            const bf16x8 v = *reinterpret_cast<const bf16x8*>(
                in_ptr(in, l, bb, (o1 + a - 1) & mask, (o2 + b - 1) & mask,
                       (o3 + c - 1) & mask, q0 + 8 * cg));
            *reinterpret_cast<bf16x8*>(halo + p * cst + 8 * cg) = v;
        }
        __syncthreads();
        // this lane's A rows: voxels (wave, mt, li) of the brick, mt = 0..3
        int t = 0, ci = 8 * g;
        while (ci >= cst) { ci -= cst; ++t; }
        for (int kc = 0; kc < ksc; kc += 32) {
            bf16x8 bv[NG];
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                bv[gi] = bf16x8{};
                if (t < 27)
                    bv[gi] = *reinterpret_cast<const bf16x8*>(
                        wt + (size_t)(gi * 16 + li) * kpad + t * cin + q0 + ci);
            }
            const int pt = t < 27 ? (t / 9) * 108 + ((t / 3) % 3) * 18 + t % 3 : 0;
            const bf16* base = halo + (wave * 108 + li + pt) * cst + ci;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                bf16x8 av = {};
                if (t < 27) av = *reinterpret_cast<const bf16x8*>(base + mt * 18 * cst);
#pragma unroll
                for (int gi = 0; gi < NG; ++gi)
                    acc[gi][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[gi],
                                                                          acc[gi][mt], 0, 0, 0);
            }
            ci += 32;
            while (ci >= cst) { ci -= cst; ++t; }
        }
    }
    // results: rows 4 g + r of tile mt = brick voxel (wave, mt, 4 g + r), column 16 gi + li
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
        const int co = gi * 16 + li;
        if (co >= cout) continue;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                conv_store<EPI>(out, cout, vox(bb, o1 + wave, o2 + mt, o3 + 4 * g + r, l), co,
                                acc[gi][mt][r]);
    }
}

// Sum of the reduction splits of a convolution in split order, then the
// epilogue: y[m][co] for co < cout from part[z][m][nrows].
template <int EPI>
__global__ __launch_bounds__(256) void k_conv_reduce(const float* __restrict__ part, int nsplit,
                                                     long long mtot, int nrows, int cout,
                                                     ConvOut out) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= mtot * cout) return;
    const long long mo = idx / cout;
    const int co = (int)(idx - mo * cout);
    float a = 0.f;
    for (int z = 0; z < nsplit; ++z) a += part[((size_t)z * mtot + mo) * nrows + co];
    conv_store<EPI>(out, cout, mo, co, a);
}

// Weight-gradient GEMM: partial[s][row][k] = sum over the voxels of split s
// of dz[m][row] x(m + o_t)[ci], k = t cin + ci. A workgroup covers 16 rows x
// 256 columns (64 per wave, 4 MFMA tiles), grid (rowtiles * ktiles, splits);
// voxels advance 32 per MFMA. chunk is a multiple of 32.
__global__ __launch_bounds__(256) void k_wgrad(ConvIn in, const bf16* __restrict__ dz, int cdz,
                                               int l, int mtot, int kpad, int ktiles,
                                               int chunk, float* __restrict__ partial,
                                               int nrows) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, li = lane & 15;
    const int mask = (1 << l) - 1;
    const int row0 = (blockIdx.x / ktiles) * 16;
    const int kcol0 = (blockIdx.x % ktiles) * 256 + wave * 64;
    const int split = blockIdx.y;
    const int mstart = split * chunk;
    const int mend = min(mtot, mstart + chunk);
    const int cin = in.ca + in.cb;
    int tt[4], cc[4];
    bool kv[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int k = kcol0 + nt * 16 + li;
        kv[nt] = k < 27 * cin;
        tt[nt] = k / cin;
        cc[nt] = k - tt[nt] * cin;
    }
    const int co = row0 + li;
    const bool cov = co < cdz;
    floatx4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int mc = mstart; mc < mend; mc += 32) {
        bf16x8 av = {};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int mm = mc + 8 * g + j;
            if (cov && mm < mend) av[j] = dz[(size_t)mm * cdz + co];
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            if (kcol0 + nt * 16 >= kpad) continue;
            bf16x8 bv = {};
            if (kv[nt]) {
                const int t = tt[nt];
                const int o1 = t / 9 - 1, o2 = (t / 3) % 3 - 1, o3 = t % 3 - 1;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int mm = mc + 8 * g + j;
                    if (mm < mend) {
                        const int i3 = mm & mask, i2 = (mm >> l) & mask, i1 = (mm >> (2 * l)) & mask;
                        const int bb = mm >> (3 * l);
                        bv[j] = *in_ptr(in, l, bb, (i1 + o1) & mask, (i2 + o2) & mask,
                                        (i3 + o3) & mask, cc[nt]);
                    }
                }
            }
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int k = kcol0 + nt * 16 + li;
        if (kcol0 + nt * 16 >= kpad) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            partial[((size_t)split * nrows + row0 + 4 * g + r) * kpad + k] = acc[nt][r];
    }
}

// The same weight-gradient GEMM with both operands staged through LDS: per
// step of 32 voxels, the workgroup copies dz^T (16 output channels x 32
// voxels) and the transposed im2col block (its 256 k-columns x 32 voxels,
// one 16-byte load of 8 channels per voxel and k-group) into LDS, so every
// MFMA fragment is one 16-byte LDS read instead of eight 2-byte global
// loads. Same grid, partial-sum layout and summation order per lane as
// k_wgrad. Needs both input channel counts and cdz to be multiples of 8.
// With pb, the workgroups of the first k-tile also sum the staged dz^T rows
// into the bias partial pb[split][co] (in place of k_bias_partial).
__global__ __launch_bounds__(256) void k_wgrad_lds(ConvIn in, const bf16* __restrict__ dz,
                                                   int cdz, int l, int mtot, int kpad,
                                                   int ktiles, int chunk,
                                                   float* __restrict__ partial, int nrows,
                                                   float* __restrict__ pb) {
    __shared__ __align__(16) bf16 sa[16 * 32];     // [co][m]
    __shared__ __align__(16) bf16 sb[256 * 32];    // [k][m]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, li = lane & 15;
    const int mask = (1 << l) - 1;
    const int row0 = (blockIdx.x / ktiles) * 16;
    const int kblk = (blockIdx.x % ktiles) * 256;
    const int split = blockIdx.y;
    const int mstart = split * chunk;
    const int mend = min(mtot, mstart + chunk);
    const int cin = in.ca + in.cb;
    const int ktot = 27 * cin;
    // this thread's staging items: voxel lane mloc, k-groups kg = tid/32 + 8 q
    const int mloc = threadIdx.x & 31;
    int tq[4], cq[4];
    bool kq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k0 = kblk + ((threadIdx.x >> 5) + 8 * q) * 8;
        kq[q] = k0 < ktot;
        tq[q] = kq[q] ? k0 / cin : 0;
        cq[q] = k0 - tq[q] * cin;
    }
    floatx4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bool bias = pb && kblk == 0;
    float bacc = 0.f;
    for (int mc = mstart; mc < mend; mc += 32) {
        const int mm = mc + mloc;
        const bool mv = mm < mend;
        if (threadIdx.x < 64) {
            const int m2 = mc + (threadIdx.x >> 1), cg = (threadIdx.x & 1) * 8;
            bf16x8 v = {};
            if (m2 < mend && row0 + cg < cdz)
                v = *reinterpret_cast<const bf16x8*>(dz + (size_t)m2 * cdz + row0 + cg);
#pragma unroll
            for (int j = 0; j < 8; ++j) sa[(cg + j) * 32 + (threadIdx.x >> 1)] = v[j];
        }
        const int i3 = mm & mask, i2 = (mm >> l) & mask, i1 = (mm >> (2 * l)) & mask;
        const int bb = mm >> (3 * l);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bf16x8 v = {};
            if (mv && kq[q]) {
                const int t = tq[q];
                const int o1 = t / 9 - 1, o2 = (t / 3) % 3 - 1, o3 = t % 3 - 1;
                v = *reinterpret_cast<const bf16x8*>(in_ptr(in, l, bb, (i1 + o1) & mask,
                                                            (i2 + o2) & mask, (i3 + o3) & mask,
                                                            cq[q]));
            }
            const int kr = ((threadIdx.x >> 5) + 8 * q) * 8;
#pragma unroll
            for (int j = 0; j < 8; ++j) sb[(kr + j) * 32 + mloc] = v[j];
        }
        __syncthreads();
        // the bias gradient: the first k-tile's workgroups sum the staged dz^T rows
        if (bias && threadIdx.x < 16) {
#pragma unroll
            for (int m = 0; m < 32; ++m) bacc += (float)sa[threadIdx.x * 32 + m];
        }
        const bf16x8 av = *reinterpret_cast<const bf16x8*>(sa + li * 32 + 8 * g);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            if (kblk + wave * 64 + nt * 16 >= kpad) continue;
            const bf16x8 bv =
                *reinterpret_cast<const bf16x8*>(sb + (wave * 64 + nt * 16 + li) * 32 + 8 * g);
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nt], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int kc = kblk + wave * 64 + nt * 16;
        if (kc >= kpad) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            partial[((size_t)split * nrows + row0 + 4 * g + r) * kpad + kc + li] = acc[nt][r];
    }
    if (bias && threadIdx.x < 16 && row0 + threadIdx.x < cdz)
        pb[(size_t)split * cdz + row0 + threadIdx.x] = bacc;
}

// Weight gradient on 4x4x16 voxel bricks; a workgroup takes the 16 output
// rows 16 blockIdx.y .. + 15 of dz's cdz (nrows = 16 gridDim.y) and the CT
// 16-channel tiles from 16 CT blockIdx.z of the input. Split s takes bricks
// [s bps, (s + 1) bps).
// Per brick, dz^T (16 outputs x 256 voxels) and, per 16-channel tile of the
// input, its 6x6x18 neighbourhood transposed to channel planes are staged in
// LDS; the neighbourhood is kept in three copies shifted by one x3 column, so
// the 8 consecutive x3 voxels of every tap's B fragment are one aligned
// 16-byte read. Every staged value then feeds all 27 taps instead of being
// re-staged per tap as an im2col block. Wave w accumulates taps w, w + 4, ...
// for all channel tiles over all its bricks; wave 0 also sums dz^T against a
// fragment of ones (the bias gradient). Partial-sum layout as k_wgrad:
// partial[s][co][t cin + ci]. Needs cin <= 16 CT gridDim.z, cin and cdz
// multiples of 8, cdz <= nrows and l >= 4.
constexpr int kWbPlane = 6 * 6 * 16 + 8;      // bf16 per channel plane of a shifted copy
constexpr int kWbRow = 256 + 8;               // bf16 per dz^T row
template <int CT>
__global__ __launch_bounds__(256) void k_wgrad_brick(ConvIn in, const bf16* __restrict__ dz,
                                                     int cdz, int l, int nbricks, int bps,
                                                     int kpad, float* __restrict__ partial,
                                                     float* __restrict__ pb) {
    __shared__ __align__(16) bf16 xs[3 * 16 * kWbPlane];   // [s3][c][a6 6 + b6][16]
    __shared__ __align__(16) bf16 dzt[16 * kWbRow];        // [co][a 64 + b 16 + j]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, li = lane & 15;
    const int mask = (1 << l) - 1;
    const int lb = l - 2, lb3 = l - 4;
    const int cin = in.ca + in.cb;
    const int split = blockIdx.x;
    const int b0 = split * bps, b1 = min(nbricks, b0 + bps);
    const int row0 = 16 * blockIdx.y, nrows = 16 * gridDim.y;
    const int rows = min(16, cdz - row0);       // valid rows of this tile, a multiple of 8
    // rows beyond cdz of dz^T stay zero
    for (int e = threadIdx.x; e < 16 * kWbRow; e += 256) dzt[e] = (bf16)0.f;
    floatx4 acc[7][CT], accb = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ti = 0; ti < 7; ++ti)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ti][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
    bf16x8 ones;
#pragma unroll
    for (int j = 0; j < 8; ++j) ones[j] = (bf16)1.f;
    // this lane's voxels in chunk c (32 voxels = rows (a, b0c), (a, b0c + 1)):
    // a = c / 2, b = 2 (c % 2) + g / 2, j = 8 (g % 2) .. + 7
    const int bg = g >> 1, jg = 8 * (g & 1);
    for (int br = b0; br < b1; ++br) {
        int bid = br;
        const int o3 = (bid & ((1 << lb3) - 1)) << 4;
        bid >>= lb3;
        const int o2 = (bid & ((1 << lb) - 1)) << 2;
        bid >>= lb;
        const int o1 = (bid & ((1 << lb) - 1)) << 2;
        const int bb = bid >> lb;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            __syncthreads();   // the previous tile's fragments have been read
            if (ct == 0) {
                // dz^T of the brick: voxel v = a 64 + b 16 + j, 8 channels per item
                for (int e = threadIdx.x; e < 256 * (rows >> 3); e += 256) {
                    const int v = e & 255, cg = e >> 8;
                    const int a = v >> 6, b = (v >> 4) & 3, j = v & 15;
                    const bf16x8 d = *reinterpret_cast<const bf16x8*>(
                        dz + vox(bb, o1 + a, o2 + b, o3 + j, l) * cdz + row0 + 8 * cg);
#pragma unroll
                    for (int i = 0; i < 8; ++i) dzt[(8 * cg + i) * kWbRow + v] = d[i];
                }
            }
            // the neighbourhood of channels 16 (CT z + ct) + 0..15: position
            // (a6, b6, jj) is voxel o + (a6, b6, jj) - 1, stored at column
            // jj - s3 of copy s3 (0 <= jj - s3 < 16)
            for (int e = threadIdx.x; e < 648 * 2; e += 256) {
                const int p = e >> 1, cg = e & 1;
                const int a6 = p / 108, b6 = (p / 18) % 6, jj = p % 18;
                const int c0 = 16 * (CT * (int)blockIdx.z + ct) + 8 * cg;
                bf16x8 v = {};
                if (c0 < cin)
                    v = *reinterpret_cast<const bf16x8*>(
                        in_ptr(in, l, bb, (o1 + a6 - 1) & mask, (o2 + b6 - 1) & mask,
                               (o3 + jj - 1) & mask, c0));
#pragma unroll
                for (int s3 = 0; s3 < 3; ++s3) {
                    const int j = jj - s3;
                    if (j < 0 || j > 15) continue;
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        xs[(s3 * 16 + 8 * cg + i) * kWbPlane + (a6 * 6 + b6) * 16 + j] = v[i];
                }
            }
            __syncthreads();
            for (int c = 0; c < 8; ++c) {
                const int a = c >> 1, b = 2 * (c & 1) + bg;
                const bf16x8 av =
                    *reinterpret_cast<const bf16x8*>(dzt + li * kWbRow + a * 64 + b * 16 + jg);
                if (ct == 0 && wave == 0)
                    accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, ones, accb, 0, 0, 0);
#pragma unroll
                for (int ti = 0; ti < 7; ++ti) {
                    const int t = wave + 4 * ti;
                    if (t < 27) {
                        const int s3 = t % 3, d1 = t / 9, d2 = (t / 3) % 3;
                        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(
                            xs + (s3 * 16 + li) * kWbPlane + ((a + d1) * 6 + b + d2) * 16 + jg);
                        acc[ti][ct] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[ti][ct], 0, 0, 0);
                    }
                }
            }
        }
    }
    // D[co = 4 g + r][ci = li] of tap t, channel tile ct
#pragma unroll
    for (int ti = 0; ti < 7; ++ti) {
        const int t = wave + 4 * ti;
        if (t >= 27) continue;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int ci = 16 * (CT * (int)blockIdx.z + ct) + li;
            if (ci >= cin) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                partial[((size_t)split * nrows + row0 + 4 * g + r) * kpad + t * cin + ci] =
                    acc[ti][ct][r];
        }
    }
    if (pb && blockIdx.z == 0 && wave == 0 && li == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (4 * g + r < rows) pb[(size_t)split * cdz + row0 + 4 * g + r] = accb[r];
    }
}

// pb[s][c] = sum over the voxels of split s of dz[m][c]: the 256 threads
// form (voxel lane, channel) pairs, channels fastest (coalesced rows), and
// the voxel lanes are folded in a fixed tree.
__global__ __launch_bounds__(256) void k_bias_partial(const bf16* __restrict__ dz, int cdz,
                                                      int mtot, int chunk,
                                                      float* __restrict__ pb) {
    __shared__ float sh[256];
    const int s = blockIdx.x;
    const int mstart = s * chunk, mend = min(mtot, mstart + chunk);
    if (cdz > 256) {                           // wider than a workgroup: one thread per channel
        for (int c = threadIdx.x; c < cdz; c += 256) {
            float acc = 0.f;
            for (int m = mstart; m < mend; ++m) acc += (float)dz[(size_t)m * cdz + c];
            pb[(size_t)s * cdz + c] = acc;
        }
        return;
    }
    int cp = 1;
    while (cp < cdz) cp <<= 1;                 // channel lanes
    const int rows = 256 / cp;
    const int c = threadIdx.x & (cp - 1), r = threadIdx.x / cp;
    float acc = 0.f;
    if (c < cdz)
        for (int m = mstart + r; m < mend; m += rows) acc += (float)dz[(size_t)m * cdz + c];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = rows >> 1; w > 0; w >>= 1) {
        if (r < w) sh[threadIdx.x] += sh[threadIdx.x + w * cp];
        __syncthreads();
    }
    if (r == 0 && c < cdz) pb[(size_t)s * cdz + c] = sh[c];
}

// gw[co][k] = sum_s partial[s][co][k] (co < cout, k < ktot), gb[co] = sum_s pb[s][co]:
// a workgroup takes kRedOut consecutive outputs and 256 / kRedOut groups of
// threads, group q summing every (256 / kRedOut)-th split from q; the group
// sums are then added pairwise in a fixed tree (float64 throughout). Many
// small groups keep enough workgroups in flight for the narrow layers, whose
// outputs are few and whose splits are many.
constexpr int kRedOut = 16;
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ partial,
                                                      const float* __restrict__ pb, int splits,
                                                      int nrows, int kpad, int cout, int ktot,
                                                      int cdz, float* __restrict__ gw,
                                                      float* __restrict__ gb) {
    constexpr int kGroups = 256 / kRedOut;
    __shared__ double sh[256];
    const long long idx = (long long)blockIdx.x * kRedOut + (threadIdx.x % kRedOut);
    const int sg = threadIdx.x / kRedOut;
    const long long nw = (long long)cout * ktot;
    double acc = 0.0;
    if (idx < nw) {
        const int co = (int)(idx / ktot), k = (int)(idx - (long long)co * ktot);
        for (int s = sg; s < splits; s += kGroups)
            acc += partial[((size_t)s * nrows + co) * kpad + k];
    } else if (idx < nw + cout) {
        const int co = (int)(idx - nw);
        for (int s = sg; s < splits; s += kGroups) acc += pb[(size_t)s * cdz + co];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kGroups / 2; w > 0; w >>= 1) {
        if (sg < w) sh[threadIdx.x] += sh[threadIdx.x + w * kRedOut];
        __syncthreads();
    }
    if (sg == 0) {
        if (idx < nw) gw[idx] = (float)sh[threadIdx.x];
        else if (idx < nw + cout) gb[idx - nw] = (float)sh[threadIdx.x];
    }
}

// x[m] = (m0, m1, m1 - m0, 0, 0, 0, 0, 0) in bfloat16; images [batch][R^3]
__global__ __launch_bounds__(256) void k_features(const float* __restrict__ m0,
                                                  const float* __restrict__ m1, int mtot,
                                                  bf16* __restrict__ x) {
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= mtot) return;
    const float a = m0[m], b = m1[m];
    bf16x8 v = {};
    v[0] = (bf16)a;
    v[1] = (bf16)b;
    v[2] = (bf16)(b - a);
    *reinterpret_cast<bf16x8*>(x + (size_t)m * kInC) = v;
}

// 2x2x2 mean (float sum in a fixed order), output level lo
__global__ __launch_bounds__(256) void k_pool(const bf16* __restrict__ x, int C, int lo,
                                              int mtot_out, bf16* __restrict__ y) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long long)mtot_out * C) return;
    const int m = (int)(idx / C), c = (int)(idx - (long long)m * C);
    const int mask = (1 << lo) - 1;
    const int i3 = m & mask, i2 = (m >> lo) & mask, i1 = (m >> (2 * lo)) & mask, bb = m >> (3 * lo);
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b2 = 0; b2 < 2; ++b2)
            for (int d = 0; d < 2; ++d)
                s += (float)x[vox(bb, 2 * i1 + a, 2 * i2 + b2, 2 * i3 + d, lo + 1) * C + c];
    y[idx] = (bf16)(0.125f * s);
}

// dz (coarse, level lc) = bf16(slope(y) * sum of the 8 fine children of dxa)
__global__ __launch_bounds__(256) void k_up_adjoint_slope(const float* __restrict__ dxa,
                                                          const bf16* __restrict__ y, int C,
                                                          int lc, int mtot_c,
                                                          bf16* __restrict__ dz) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long long)mtot_c * C) return;
    const int m = (int)(idx / C), c = (int)(idx - (long long)m * C);
    const int mask = (1 << lc) - 1;
    const int i3 = m & mask, i2 = (m >> lc) & mask, i1 = (m >> (2 * lc)) & mask, bb = m >> (3 * lc);
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b2 = 0; b2 < 2; ++b2)
            for (int d = 0; d < 2; ++d)
                s += dxa[vox(bb, 2 * i1 + a, 2 * i2 + b2, 2 * i3 + d, lc + 1) * C + c];
    dz[idx] = (bf16)(s * slope(y[idx]));
}

// dz (fine, level lf) = bf16(slope(y) (dxp(parent) / 8 + dskip))
__global__ __launch_bounds__(256) void k_pool_adjoint_slope(const float* __restrict__ dxp,
                                                            const float* __restrict__ dskip,
                                                            const bf16* __restrict__ y, int C,
                                                            int lf, int mtot_f,
                                                            bf16* __restrict__ dz) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long long)mtot_f * C) return;
    const int m = (int)(idx / C), c = (int)(idx - (long long)m * C);
    const int mask = (1 << lf) - 1;
    const int i3 = m & mask, i2 = (m >> lf) & mask, i1 = (m >> (2 * lf)) & mask, bb = m >> (3 * lf);
    const float s = dxp[vox(bb, i1 >> 1, i2 >> 1, i3 >> 1, lf - 1) * C + c] / 8.f + dskip[idx];
    dz[idx] = (bf16)(s * slope(y[idx]));
}

// Mean squared error against target [batch][3][R^3]: dz = bf16(scale (v - t))
// in channels 0..2 of [m][8] (zero elsewhere), per-block sums of squares.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ v,
                                             const float* __restrict__ target, int l, int mtot,
                                             float scale, bf16* __restrict__ dz,
                                             double* __restrict__ partial) {
    __shared__ double sh[4];
    const int m = blockIdx.x * 256 + threadIdx.x;
    double ss = 0.0;
    if (m < mtot) {
        const int r3 = 3 * l;
        const int b = m >> r3, i = m & ((1 << r3) - 1);
        bf16x8 o = {};
#pragma unroll
        for (int c = 0; c < kOutC; ++c) {
            const float d = v[(size_t)m * kOutC + c] - target[(((size_t)b * kOutC + c) << r3) + i];
            ss += (double)d * d;
            o[c] = (bf16)(scale * d);
        }
        *reinterpret_cast<bf16x8*>(dz + (size_t)m * 8) = o;
    }
    const double t = block_sum_256(ss, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// [m][3] -> [batch][3][R^3]
__global__ __launch_bounds__(256) void k_out_transpose(const float* __restrict__ v, int l,
                                                       int mtot, float* __restrict__ out) {
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= mtot) return;
    const int r3 = 3 * l;
    const int b = m >> r3, i = m & ((1 << r3) - 1);
#pragma unroll
    for (int c = 0; c < kOutC; ++c) out[(((size_t)b * kOutC + c) << r3) + i] = v[(size_t)m * kOutC + c];
}

// Adam step (update != 0) and/or repacking of one layer's parameters into
// the bfloat16 GEMM operands: wt[co][k] (k = t cin + ci) and the
// backward-data operand wtT[ci][(26 - t) coutE + co].
__global__ __launch_bounds__(256) void k_adam_pack(float* __restrict__ p, float* __restrict__ mo,
                                                   float* __restrict__ ve,
                                                   const float* __restrict__ g, int nw, int nb,
                                                   int update, float lr, float b1, float b2,
                                                   float c1, float c2, float eps,
                                                   bf16* __restrict__ wt, int kpad, int ktot,
                                                   bf16* __restrict__ wtT, int kpadT, int cin,
                                                   int coutE) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= nw + nb) return;
    float w = p[idx];
    if (update) {
        const float gi = g[idx];
        const float m1 = b1 * mo[idx] + (1.f - b1) * gi;
        const float v1 = b2 * ve[idx] + (1.f - b2) * gi * gi;
        mo[idx] = m1;
        ve[idx] = v1;
        w -= lr * (m1 / c1) / (sqrtf(v1 / c2) + eps);
        p[idx] = w;
    }
    if (idx < nw) {
        const int co = idx / ktot, k = idx - co * ktot;
        const int t = k / cin, ci = k - t * cin;
        const bf16 h = (bf16)w;
        wt[(size_t)co * kpad + k] = h;
        wtT[(size_t)ci * kpadT + (26 - t) * coutE + co] = h;
    }
}

__global__ __launch_bounds__(256) void k_zero16(bf16* __restrict__ x, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = (bf16)0.f;
}

// float32 -> bfloat16 -> float32 (rounding of a conv operand for claire_conv3d)
__global__ __launch_bounds__(256) void k_round16(const float* __restrict__ x, long long n,
                                                 bf16* __restrict__ y) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = (bf16)x[i];
}

// ------------------------------------------------------------ grid transfer
// dst (2^(l-1))^3 = 2x2x2 block means of src (2^l)^3, per component
__global__ __launch_bounds__(256) void k_restrict2(const float* __restrict__ src, int l,
                                                   long long ndst, int ncomp,
                                                   float* __restrict__ dst) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= ndst * ncomp) return;
    const int c = (int)(idx / ndst);
    const long long m = idx - (long long)c * ndst;
    const int lo = l - 1, mask = (1 << lo) - 1;
    const int i3 = (int)(m & mask), i2 = (int)((m >> lo) & mask), i1 = (int)(m >> (2 * lo));
    const float* s = src + ((long long)c << (3 * l));
    float acc = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int d = 0; d < 2; ++d)
                acc += s[vox(0, 2 * i1 + a, 2 * i2 + b, 2 * i3 + d, l)];
    dst[idx] = 0.125f * acc;
}

// Refine axis `ax` (0: x1, 1: x2, 2: x3) of fields with extents e[3] by 2:
// even points copy, midpoints (-f(i-1) + 9 f(i) + 9 f(i+1) - f(i+2)) / 16.
__global__ __launch_bounds__(256) void k_prolong_axis(const float* __restrict__ src, int e1,
                                                      int e2, int e3, int ax, int ncomp,
                                                      float* __restrict__ dst) {
    const int d1 = ax == 0 ? 2 * e1 : e1, d2 = ax == 1 ? 2 * e2 : e2, d3 = ax == 2 ? 2 * e3 : e3;
    const long long nd = (long long)d1 * d2 * d3;
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= nd * ncomp) return;
    const int c = (int)(idx / nd);
    const long long m = idx - (long long)c * nd;
    int j3 = (int)(m % d3);
    int j2 = (int)((m / d3) % d2);
    int j1 = (int)(m / ((long long)d3 * d2));
    const float* s = src + (long long)c * e1 * e2 * e3;
    int* jj = ax == 0 ? &j1 : (ax == 1 ? &j2 : &j3);
    const int ea = ax == 0 ? e1 : (ax == 1 ? e2 : e3);
    const int i = *jj >> 1;
    auto at = [&](int q) {
        *jj = ((q % ea) + ea) % ea;
        return s[((long long)j1 * e2 + j2) * e3 + j3];
    };
    float r;
    if ((ax == 0 ? j1 : (ax == 1 ? j2 : j3)) & 1) {
        const float fm1 = at(i - 1), f0 = at(i), fp1 = at(i + 1), fp2 = at(i + 2);
        r = (-fm1 + 9.f * f0 + 9.f * fp1 - fp2) / 16.f;
    } else {
        r = at(i);
    }
    dst[idx] = r;
}

unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

int lg2(int v) { int l = 0; while ((1 << l) < v) ++l; return l; }

template <typename T>
int dalloc(T** p, long long count) {
    CL_HIP(hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)(count > 0 ? count : 1)));
    return 0;
}
void dfree(void* p) {
    if (p) (void)hipFree(p);
}

int zero16(bf16* x, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero16, dim3(nblk(n)), dim3(256), 0, s, x, n);
    CL_LAUNCH_CHECK();
    return 0;
}

int roundup(int v, int q) { return (v + q - 1) / q * q; }

// Resample [ncomp][n_src^3] -> [ncomp][n_dst^3] with two scratch buffers of
// ncomp * max(n)^3 floats.
int resample(const float* src, int ns, float* dst, int nd, int ncomp, float* t0, float* t1,
             hipStream_t s) {
    const float* cur = src;
    int n = ns;
    float* bufs[2] = {t0, t1};
    int which = 0;
    auto target = [&](bool last) { return last ? dst : bufs[which]; };
    if (n == nd) {
        CL_HIP(hipMemcpyAsync(dst, src, sizeof(float) * (size_t)ncomp * nd * nd * nd,
                              hipMemcpyDeviceToDevice, s));
        return 0;
    }
    while (n > nd) {
        const bool last = n / 2 == nd;
        float* out = target(last);
        const long long ndst = (long long)(n / 2) * (n / 2) * (n / 2);
        hipLaunchKernelGGL(k_restrict2, dim3(nblk(ndst * ncomp)), dim3(256), 0, s, cur, lg2(n),
                           ndst, ncomp, out);
        CL_LAUNCH_CHECK();
        cur = out;
        which ^= 1;
        n /= 2;
    }
    while (n < nd) {
        int e[3] = {n, n, n};
        for (int ax = 0; ax < 3; ++ax) {
            const bool last = (2 * n == nd) && ax == 2;
            float* out = target(last);
            const long long ndst = 2LL * e[0] * e[1] * e[2];
            hipLaunchKernelGGL(k_prolong_axis, dim3(nblk(ndst * ncomp)), dim3(256), 0, s, cur,
                               e[0], e[1], e[2], ax, ncomp, out);
            CL_LAUNCH_CHECK();
            e[ax] *= 2;
            cur = out;
            which ^= 1;
        }
        n *= 2;
    }
    return 0;
}

uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

}  // namespace

// One convolution layer's geometry and GEMM operands.
struct NetLayer {
    int cin, cout, coutE;   // coutE: cout rounded up to 8 (channels of its dz)
    int ktot, kpad, nrows;  // forward GEMM: [nrows][kpad]
    int kpadT, nrowsT;      // backward-data GEMM: [nrowsT][kpadT]
    long long off;          // parameter offset
    bf16* wt = nullptr;
    bf16* wtT = nullptr;
};

}  // namespace claire

using namespace claire;

struct claire_net {
    int R = 0, l = 0, c[4] = {0, 0, 0, 0}, max_batch = 0;
    hipStream_t s = nullptr;
    NetLayer L[kLayers];
    long long nparam = 0;
    float *p = nullptr, *mo = nullptr, *ve = nullptr, *g = nullptr;
    int adam_t = 0;
    // activations (bfloat16, channels last)
    bf16 *x0 = nullptr, *e1a = nullptr, *s1 = nullptr, *p1 = nullptr, *e2a = nullptr,
         *s2 = nullptr, *p2 = nullptr, *e3a = nullptr, *s3 = nullptr, *p3 = nullptr,
         *ba = nullptr, *bt = nullptr, *d3a = nullptr, *d3 = nullptr, *d2a = nullptr,
         *d2 = nullptr, *d1a = nullptr, *d1 = nullptr;
    float* vout = nullptr;   // [m][3]
    // backward
    bf16* dzh = nullptr;                    // [m1][8]
    bf16 *dzA[4] = {}, *dzB[4] = {};        // per level ping-pong, [m_l][max(c_l, 8)]
    float *dxA = nullptr, *dxp = nullptr;
    float *dskip[3] = {};
    float *partial = nullptr, *pb = nullptr;
    long long partial_cap = 0, pb_cap = 0;
    Reducer red;
    bool have_grads = false;
    // warm-start scratch, grown on demand: restricted images, velocity at
    // the working resolution, two transfer buffers of 3 n^3 floats
    float *ws_a = nullptr, *ws_b = nullptr, *ws_v = nullptr, *ws_t0 = nullptr, *ws_t1 = nullptr;
    long long ws_cap = 0;
};

namespace claire {
namespace {

enum { ENC1A, ENC1B, ENC2A, ENC2B, ENC3A, ENC3B, BOTA, BOTB, DEC3A, DEC3B, DEC2A, DEC2B, DEC1A,
       DEC1B, HEAD };

long long vox_level(const claire_net* n, int level, int batch) {
    const int lv = n->l - level;
    return (long long)batch << (3 * lv);
}

// splits of the voxel reduction in the weight gradient and the chunk size
void wgrad_split(long long mtot, int& splits, int& chunk) {
    long long sp = (mtot + 511) / 512;
    if (sp > 1024) sp = 1024;
    if (sp < 1) sp = 1;
    long long ch = (mtot + sp - 1) / sp;
    ch = (ch + 31) / 32 * 32;
    splits = (int)((mtot + ch - 1) / ch);
    chunk = (int)ch;
}

// Reduction splits of a convolution whose 64 x 64 tiles alone would leave
// most of the chip idle (the coarse levels): enough splits for about 768
// workgroups, each keeping at least 8 of the kpad / 32 reduction steps.
int conv_splits(long long mtot, int nrows, int kpad) {
    const long long tiles = ((mtot + 63) / 64) * ((nrows + 63) / 64);
    if (tiles >= 384) return 1;
    long long sp = (768 + tiles - 1) / tiles;
    const long long smax = (kpad / 32) / 8;
    if (sp > smax) sp = smax;
    return sp < 1 ? 1 : (int)sp;
}

int net_alloc(claire_net* n) {
    const int c1 = n->c[0], c2 = n->c[1], c3 = n->c[2], c4 = n->c[3];
    const int dims[kLayers][2] = {
        {kInC, c1}, {c1, c1}, {c1, c2}, {c2, c2}, {c2, c3}, {c3, c3}, {c3, c4}, {c4, c4},
        {c4 + c3, c3}, {c3, c3}, {c3 + c2, c2}, {c2, c2}, {c2 + c1, c1}, {c1, c1}, {c1, kOutC}};
    long long off = 0;
    for (int i = 0; i < kLayers; ++i) {
        NetLayer& L = n->L[i];
        L.cin = dims[i][0];
        L.cout = dims[i][1];
        L.coutE = roundup(L.cout, 8);
        L.ktot = 27 * L.cin;
        L.kpad = roundup(L.ktot, 32);
        L.nrows = roundup(L.cout, 16);
        L.kpadT = roundup(27 * L.coutE, 32);
        L.nrowsT = roundup(L.cin, 16);
        L.off = off;
        off += (long long)L.cout * L.ktot + L.cout;
        CL_TRY(dalloc(&L.wt, (long long)L.nrows * L.kpad));
        CL_TRY(dalloc(&L.wtT, (long long)L.nrowsT * L.kpadT));
        CL_TRY(zero16(L.wt, (long long)L.nrows * L.kpad, n->s));
        CL_TRY(zero16(L.wtT, (long long)L.nrowsT * L.kpadT, n->s));
    }
    n->nparam = off;
    CL_TRY(dalloc(&n->p, off));
    CL_TRY(dalloc(&n->mo, off));
    CL_TRY(dalloc(&n->ve, off));
    CL_TRY(dalloc(&n->g, off));
    const int B = n->max_batch;
    const long long m1 = vox_level(n, 0, B), m2 = vox_level(n, 1, B), m3 = vox_level(n, 2, B),
                    m4 = vox_level(n, 3, B);
    CL_TRY(dalloc(&n->x0, m1 * kInC));
    CL_TRY(dalloc(&n->e1a, m1 * c1));
    CL_TRY(dalloc(&n->s1, m1 * c1));
    CL_TRY(dalloc(&n->p1, m2 * c1));
    CL_TRY(dalloc(&n->e2a, m2 * c2));
    CL_TRY(dalloc(&n->s2, m2 * c2));
    CL_TRY(dalloc(&n->p2, m3 * c2));
    CL_TRY(dalloc(&n->e3a, m3 * c3));
    CL_TRY(dalloc(&n->s3, m3 * c3));
    CL_TRY(dalloc(&n->p3, m4 * c3));
    CL_TRY(dalloc(&n->ba, m4 * c4));
    CL_TRY(dalloc(&n->bt, m4 * c4));
    CL_TRY(dalloc(&n->d3a, m3 * c3));
    CL_TRY(dalloc(&n->d3, m3 * c3));
    CL_TRY(dalloc(&n->d2a, m2 * c2));
    CL_TRY(dalloc(&n->d2, m2 * c2));
    CL_TRY(dalloc(&n->d1a, m1 * c1));
    CL_TRY(dalloc(&n->d1, m1 * c1));
    CL_TRY(dalloc(&n->vout, m1 * kOutC));
    CL_TRY(dalloc(&n->dzh, m1 * 8));
    const long long ml[4] = {m1, m2, m3, m4};
    for (int k = 0; k < 4; ++k) {
        const int ch = n->c[k] > 8 ? n->c[k] : 8;
        CL_TRY(dalloc(&n->dzA[k], ml[k] * ch));
        CL_TRY(dalloc(&n->dzB[k], ml[k] * ch));
    }
    long long dxa = m1 * c2;
    if (m2 * c3 > dxa) dxa = m2 * c3;
    if (m3 * c4 > dxa) dxa = m3 * c4;
    CL_TRY(dalloc(&n->dxA, dxa));
    long long dxp = m2 * c1;
    if (m3 * c2 > dxp) dxp = m3 * c2;
    if (m4 * c3 > dxp) dxp = m4 * c3;
    CL_TRY(dalloc(&n->dxp, dxp));
    CL_TRY(dalloc(&n->dskip[0], m1 * c1));
    CL_TRY(dalloc(&n->dskip[1], m2 * c2));
    CL_TRY(dalloc(&n->dskip[2], m3 * c3));
    // weight-gradient partial sums: the largest splits x nrows x kpad over layers
    const int lvl[kLayers] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0};
    for (int i = 0; i < kLayers; ++i) {
        int splits, chunk;
        wgrad_split(ml[lvl[i]], splits, chunk);
        const long long need = (long long)splits * n->L[i].nrows * n->L[i].kpad;
        if (need > n->partial_cap) n->partial_cap = need;
        const long long needb = (long long)splits * n->L[i].coutE;
        if (needb > n->pb_cap) n->pb_cap = needb;
        // the same buffer holds the reduction splits of the coarse-level
        // convolutions (forward and backward data), which run between
        // weight gradients on the same stream
        const NetLayer& L = n->L[i];
        const long long mt = ml[lvl[i]];
        const long long needf = (long long)conv_splits(mt, L.nrows, L.kpad) * mt * L.nrows;
        const long long needd = (long long)conv_splits(mt, L.nrowsT, L.kpadT) * mt * L.nrowsT;
        if (needf > n->partial_cap) n->partial_cap = needf;
        if (needd > n->partial_cap) n->partial_cap = needd;
    }
    CL_TRY(dalloc(&n->partial, n->partial_cap));
    CL_TRY(dalloc(&n->pb, n->pb_cap));
    CL_TRY(reducer_init(n->red, m1));
    return 0;
}

void net_release(claire_net* n) {
    for (auto& L : n->L) {
        dfree(L.wt);
        dfree(L.wtT);
    }
    void* bufs[] = {n->p, n->mo, n->ve, n->g, n->x0, n->e1a, n->s1, n->p1, n->e2a, n->s2,
                    n->p2, n->e3a, n->s3, n->p3, n->ba, n->bt, n->d3a, n->d3, n->d2a, n->d2,
                    n->d1a, n->d1, n->vout, n->dzh, n->dxA, n->dxp, n->partial, n->pb,
                    n->dskip[0], n->dskip[1], n->dskip[2], n->ws_a, n->ws_b, n->ws_v,
                    n->ws_t0, n->ws_t1};
    for (void* b : bufs) dfree(b);
    for (int k = 0; k < 4; ++k) {
        dfree(n->dzA[k]);
        dfree(n->dzB[k]);
    }
    reducer_free(n->red);
}

// Adam step (update) or repack of all layers' GEMM operands from n->p.
int net_pack(claire_net* n, bool update, double lr) {
    float c1 = 1.f, c2 = 1.f;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    if (update) {
        ++n->adam_t;
        c1 = (float)(1.0 - std::pow(0.9, n->adam_t));
        c2 = (float)(1.0 - std::pow(0.999, n->adam_t));
    }
    for (auto& L : n->L) {
        const int nw = L.cout * L.ktot, nb = L.cout;
        hipLaunchKernelGGL(k_adam_pack, dim3(nblk(nw + nb)), dim3(256), 0, n->s, n->p + L.off,
                           n->mo + L.off, n->ve + L.off, n->g + L.off, nw, nb, update ? 1 : 0,
                           (float)lr, b1, b2, c1, c2, eps, L.wt, L.kpad, L.ktot, L.wtT, L.kpadT,
                           L.cin, L.coutE);
        CL_LAUNCH_CHECK();
    }
    return 0;
}

int reset_adam(claire_net* n) {
    CL_TRY(launch_fill(n->mo, 0.f, n->nparam, n->s));
    CL_TRY(launch_fill(n->ve, 0.f, n->nparam, n->s));
    n->adam_t = 0;
    n->have_grads = false;
    return 0;
}

#ifndef CLAIRE_CONV_HALO
#define CLAIRE_CONV_HALO 1
#endif
#ifndef CLAIRE_CONV_NARROW
#define CLAIRE_CONV_NARROW 1
#endif
#ifndef CLAIRE_WGRAD_LDS
#define CLAIRE_WGRAD_LDS 1
#endif
constexpr bool kWgradLds = CLAIRE_WGRAD_LDS;

#ifndef CLAIRE_NARROW_SMALL_CHUNK
#define CLAIRE_NARROW_SMALL_CHUNK 1
#endif

template <int EPI>
int conv(const ConvIn& in, const bf16* wt, int kpad, int nrows, int cout, int l, long long mtot,
         const ConvOut& out, hipStream_t s, float* part = nullptr, long long part_cap = 0) {
    const int cin = in.ca + in.cb;
    // the halo kernels tile the grid by 4x4x4 or 4x4x16 bricks (mtot = batch 8^l);
    // the narrow kernel takes up to 6 column groups where its 256-voxel bricks
    // still give at least 256 workgroups
    const int ng = nrows / 16;
    const bool narrow = CLAIRE_CONV_NARROW && nrows <= 16 * kNarrowMaxNG && l >= 4 &&
                        (cin <= kNarrowMaxC || cin % kNarrowMaxC == 0) && (cin & 7) == 0 &&
                        (mtot & 255) == 0 && (ng == 1 || mtot >= 256LL * 256);
    // reduction splits: k_conv and k_conv_halo only
    int splits = part && !narrow ? conv_splits(mtot, nrows, kpad) : 1;
    if ((long long)splits * mtot * nrows > part_cap) splits = 1;
    const dim3 grid((unsigned)((mtot + 63) / 64), (unsigned)((nrows + 63) / 64),
                    (unsigned)splits);
    if (narrow) {
        // staged chunk: all channels up to kNarrowMaxC, else kNarrowMaxC; where
        // the summation order may change (part given: batches above one),
        // 24 or 16 channels, for more workgroups per CU
        int cst = cin <= kNarrowMaxC ? cin : kNarrowMaxC;
        if (part && CLAIRE_NARROW_SMALL_CHUNK)
            cst = (cin % 24 == 0) ? 24 : (cin % 16 == 0 ? 16 : cst);
        const size_t lds = sizeof(bf16) * kNarrowPos * cst;
        const dim3 ngrid((unsigned)(mtot / 256));
        if (ng == 1)
            hipLaunchKernelGGL((k_conv_narrow<EPI, 1>), ngrid, dim3(256), lds, s, in, wt, kpad,
                               cout, l, out, cst);
        else if (ng == 2)
            hipLaunchKernelGGL((k_conv_narrow<EPI, 2>), ngrid, dim3(256), lds, s, in, wt, kpad,
                               cout, l, out, cst);
        else if (ng == 3)
            hipLaunchKernelGGL((k_conv_narrow<EPI, 3>), ngrid, dim3(256), lds, s, in, wt, kpad,
                               cout, l, out, cst);
        else if (ng == 4)
            hipLaunchKernelGGL((k_conv_narrow<EPI, 4>), ngrid, dim3(256), lds, s, in, wt, kpad,
                               cout, l, out, cst);
        else if (ng == 5)
            hipLaunchKernelGGL((k_conv_narrow<EPI, 5>), ngrid, dim3(256), lds, s, in, wt, kpad,
                               cout, l, out, cst);
        else
            hipLaunchKernelGGL((k_conv_narrow<EPI, 6>), ngrid, dim3(256), lds, s, in, wt, kpad,
                               cout, l, out, cst);
    } else if (CLAIRE_CONV_HALO && l >= 2 && cin <= kHaloMaxC && (cin & 7) == 0 &&
               (mtot & 63) == 0) {
        const size_t lds = sizeof(bf16) * kHaloPos * cin;
        hipLaunchKernelGGL(k_conv_halo<EPI>, grid, dim3(256), lds, s, in, wt, kpad, nrows, cout,
                           l, out, part);
    } else {
        hipLaunchKernelGGL(k_conv<EPI>, grid, dim3(256), 0, s, in, wt, kpad, nrows, cout, l,
                           (int)mtot, out, part);
    }
    CL_LAUNCH_CHECK();
    if (splits > 1) {
        hipLaunchKernelGGL(k_conv_reduce<EPI>, dim3(nblk(mtot * cout)), dim3(256), 0, s, part,
                           splits, mtot, nrows, cout, out);
        CL_LAUNCH_CHECK();
    }
    return 0;
}

ConvIn one(const bf16* a, int ca) { return ConvIn{a, ca, 0, nullptr, 0}; }
ConvIn cat_up(const bf16* up, int cu, const bf16* skip, int cs) {
    return ConvIn{up, cu, 1, skip, cs};
}

// Split buffer for forward convolutions: batches of one (the warm start's
// inference) keep the single-pass reduction, so the initial guess the solver
// receives does not change with the training-side splitting.
float* fwd_part(claire_net* n, int batch) { return batch > 1 ? n->partial : nullptr; }

// forward layer with LeakyReLU into y (bfloat16)
int fwd(claire_net* n, int li, const ConvIn& in, int level, int batch, bf16* y) {
    const NetLayer& L = n->L[li];
    ConvOut o{};
    o.y16 = y;
    o.bias = n->p + L.off + (long long)L.cout * L.ktot;
    return conv<EPI_ACT>(in, L.wt, L.kpad, L.nrows, L.cout, n->l - level,
                         vox_level(n, level, batch), o, n->s, fwd_part(n, batch),
                         n->partial_cap);
}

int pool(claire_net* n, const bf16* x, int C, int level_out, int batch, bf16* y) {
    const long long mo = vox_level(n, level_out, batch);
    hipLaunchKernelGGL(k_pool, dim3(nblk(mo * C)), dim3(256), 0, n->s, x, C, n->l - level_out,
                       (int)mo, y);
    CL_LAUNCH_CHECK();
    return 0;
}

int net_forward(claire_net* n, const float* m0, const float* m1, int batch) {
    const int c1 = n->c[0], c2 = n->c[1], c3 = n->c[2], c4 = n->c[3];
    const long long mt = vox_level(n, 0, batch);
    hipLaunchKernelGGL(k_features, dim3(nblk(mt)), dim3(256), 0, n->s, m0, m1, (int)mt, n->x0);
    CL_LAUNCH_CHECK();
    CL_TRY(fwd(n, ENC1A, one(n->x0, kInC), 0, batch, n->e1a));
    CL_TRY(fwd(n, ENC1B, one(n->e1a, c1), 0, batch, n->s1));
    CL_TRY(pool(n, n->s1, c1, 1, batch, n->p1));
    CL_TRY(fwd(n, ENC2A, one(n->p1, c1), 1, batch, n->e2a));
    CL_TRY(fwd(n, ENC2B, one(n->e2a, c2), 1, batch, n->s2));
    CL_TRY(pool(n, n->s2, c2, 2, batch, n->p2));
    CL_TRY(fwd(n, ENC3A, one(n->p2, c2), 2, batch, n->e3a));
    CL_TRY(fwd(n, ENC3B, one(n->e3a, c3), 2, batch, n->s3));
    CL_TRY(pool(n, n->s3, c3, 3, batch, n->p3));
    CL_TRY(fwd(n, BOTA, one(n->p3, c3), 3, batch, n->ba));
    CL_TRY(fwd(n, BOTB, one(n->ba, c4), 3, batch, n->bt));
    CL_TRY(fwd(n, DEC3A, cat_up(n->bt, c4, n->s3, c3), 2, batch, n->d3a));
    CL_TRY(fwd(n, DEC3B, one(n->d3a, c3), 2, batch, n->d3));
    CL_TRY(fwd(n, DEC2A, cat_up(n->d3, c3, n->s2, c2), 1, batch, n->d2a));
    CL_TRY(fwd(n, DEC2B, one(n->d2a, c2), 1, batch, n->d2));
    CL_TRY(fwd(n, DEC1A, cat_up(n->d2, c2, n->s1, c1), 0, batch, n->d1a));
    CL_TRY(fwd(n, DEC1B, one(n->d1a, c1), 0, batch, n->d1));
    const NetLayer& H = n->L[HEAD];
    ConvOut o{};
    o.y32 = n->vout;
    o.bias = n->p + H.off + (long long)H.cout * H.ktot;
    return conv<EPI_LINEAR>(one(n->d1, c1), H.wt, H.kpad, H.nrows, H.cout, n->l, mt, o, n->s,
                            fwd_part(n, batch), n->partial_cap);
}

#ifndef CLAIRE_WGRAD_BRICK
#define CLAIRE_WGRAD_BRICK 1
#endif

// Launches k_wgrad_brick when the layer fits it (at most 64 outputs, at most
// 192 input channels, x3 extent >= 16); false if not.
constexpr int kBrickWgs = 512;   // two workgroups per CU in one round
bool wgrad_brick(const ConvIn& in, const bf16* dz, int cdz, int l, long long mt, int& splits,
                 int nrows, int kpad, float* partial, long long part_cap, float* pb,
                 long long pb_cap, hipStream_t s) {
    const int cin = in.ca + in.cb;
    if (!CLAIRE_WGRAD_BRICK || nrows > 64 || (nrows & 15) || cdz > nrows || (cdz & 7) ||
        (in.ca & 7) || (in.cb & 7) || cin > 192 || l < 4 || (mt & 255))
        return false;
    // channel tiles of 16, in groups of at most 3 per workgroup (the
    // accumulators of 7 taps x 3 tiles)
    const int tiles = (cin + 15) / 16, groups = (tiles + 2) / 3;
    const int ct = (tiles + groups - 1) / groups;
    // bricks per split: about kBrickWgs workgroups over splits, row tiles and
    // channel groups (fewer splits, fewer partial sums to write and reduce),
    // and no more splits than the partial buffers hold
    const int nbricks = (int)(mt / 256);
    int want = kBrickWgs / ((nrows / 16) * groups);
    if (want < 1) want = 1;
    int bps = (nbricks + want - 1) / want;
    auto nsplit = [&](int b) { return (long long)((nbricks + b - 1) / b); };
    while (nsplit(bps) * nrows * kpad > part_cap || nsplit(bps) * cdz > pb_cap) ++bps;
    splits = (int)nsplit(bps);
    const dim3 grid((unsigned)splits, (unsigned)(nrows / 16), (unsigned)groups), block(256);
    if (ct == 1)
        hipLaunchKernelGGL(k_wgrad_brick<1>, grid, block, 0, s, in, dz, cdz, l, nbricks, bps,
                           kpad, partial, pb);
    else if (ct == 2)
        hipLaunchKernelGGL(k_wgrad_brick<2>, grid, block, 0, s, in, dz, cdz, l, nbricks, bps,
                           kpad, partial, pb);
    else
        hipLaunchKernelGGL(k_wgrad_brick<3>, grid, block, 0, s, in, dz, cdz, l, nbricks, bps,
                           kpad, partial, pb);
    return true;
}

// weight and bias gradient of layer li from its input view and dz
int wgrad(claire_net* n, int li, const ConvIn& in, const bf16* dz, int level, int batch) {
    const NetLayer& L = n->L[li];
    const long long mt = vox_level(n, level, batch);
    int splits, chunk;
    wgrad_split(mt, splits, chunk);
    const int ktiles = (L.kpad + 255) / 256;
    const dim3 grid((unsigned)((L.nrows / 16) * ktiles), (unsigned)splits);
    if (wgrad_brick(in, dz, L.coutE, n->l - level, mt, splits, L.nrows, L.kpad, n->partial,
                    n->partial_cap, n->pb, n->pb_cap, n->s)) {
    } else if (kWgradLds && in.ca % 8 == 0 && in.cb % 8 == 0 && L.coutE % 8 == 0) {
        hipLaunchKernelGGL(k_wgrad_lds, grid, dim3(256), 0, n->s, in, dz, L.coutE, n->l - level,
                           (int)mt, L.kpad, ktiles, chunk, n->partial, L.nrows, n->pb);
    } else {
        hipLaunchKernelGGL(k_wgrad, grid, dim3(256), 0, n->s, in, dz, L.coutE, n->l - level,
                           (int)mt, L.kpad, ktiles, chunk, n->partial, L.nrows);
        CL_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_bias_partial, dim3(splits), dim3(256), 0, n->s, dz, L.coutE,
                           (int)mt, chunk, n->pb);
    }
    CL_LAUNCH_CHECK();
    const long long nw = (long long)L.cout * L.ktot;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((nw + L.cout + kRedOut - 1) / kRedOut)),
                       dim3(256), 0,
                       n->s, n->partial,
                       n->pb, splits, L.nrows, L.kpad, L.cout, L.ktot, L.coutE, n->g + L.off,
                       n->g + L.off + nw);
    CL_LAUNCH_CHECK();
    return 0;
}

// backward data through layer li: dz_prev = bf16(conv^T(dz) * slope(yprev))
int dgrad_act(claire_net* n, int li, const bf16* dz, const bf16* yprev, int level, int batch,
              bf16* dz_prev) {
    const NetLayer& L = n->L[li];
    ConvOut o{};
    o.y16 = dz_prev;
    o.yprev = yprev;
    return conv<EPI_DGRAD_ACT>(one(dz, L.coutE), L.wtT, L.kpadT, L.nrowsT, L.cin, n->l - level,
                               vox_level(n, level, batch), o, n->s, n->partial, n->partial_cap);
}

// backward data into float32, channels < csplit to a, the rest to b
int dgrad_raw(claire_net* n, int li, const bf16* dz, int level, int batch, int csplit, float* a,
              float* b) {
    const NetLayer& L = n->L[li];
    ConvOut o{};
    o.y32 = a;
    o.y32b = b;
    o.csplit = csplit;
    return conv<EPI_DGRAD_RAW>(one(dz, L.coutE), L.wtT, L.kpadT, L.nrowsT, L.cin, n->l - level,
                               vox_level(n, level, batch), o, n->s, n->partial, n->partial_cap);
}

int up_adjoint(claire_net* n, const float* dxa, const bf16* y, int C, int level_c, int batch,
               bf16* dz) {
    const long long mc = vox_level(n, level_c, batch);
    hipLaunchKernelGGL(k_up_adjoint_slope, dim3(nblk(mc * C)), dim3(256), 0, n->s, dxa, y, C,
                       n->l - level_c, (int)mc, dz);
    CL_LAUNCH_CHECK();
    return 0;
}

int pool_adjoint(claire_net* n, const float* dxp, const float* dskip, const bf16* y, int C,
                 int level_f, int batch, bf16* dz) {
    const long long mf = vox_level(n, level_f, batch);
    hipLaunchKernelGGL(k_pool_adjoint_slope, dim3(nblk(mf * C)), dim3(256), 0, n->s, dxp, dskip,
                       y, C, n->l - level_f, (int)mf, dz);
    CL_LAUNCH_CHECK();
    return 0;
}

int net_backward(claire_net* n, int batch) {
    const int c1 = n->c[0], c2 = n->c[1], c3 = n->c[2], c4 = n->c[3];
    bf16** A = n->dzA;
    bf16** B = n->dzB;
    CL_TRY(wgrad(n, HEAD, one(n->d1, c1), n->dzh, 0, batch));
    CL_TRY(dgrad_act(n, HEAD, n->dzh, n->d1, 0, batch, A[0]));
    CL_TRY(wgrad(n, DEC1B, one(n->d1a, c1), A[0], 0, batch));
    CL_TRY(dgrad_act(n, DEC1B, A[0], n->d1a, 0, batch, B[0]));
    CL_TRY(wgrad(n, DEC1A, cat_up(n->d2, c2, n->s1, c1), B[0], 0, batch));
    CL_TRY(dgrad_raw(n, DEC1A, B[0], 0, batch, c2, n->dxA, n->dskip[0]));
    CL_TRY(up_adjoint(n, n->dxA, n->d2, c2, 1, batch, A[1]));
    CL_TRY(wgrad(n, DEC2B, one(n->d2a, c2), A[1], 1, batch));
    CL_TRY(dgrad_act(n, DEC2B, A[1], n->d2a, 1, batch, B[1]));
    CL_TRY(wgrad(n, DEC2A, cat_up(n->d3, c3, n->s2, c2), B[1], 1, batch));
    CL_TRY(dgrad_raw(n, DEC2A, B[1], 1, batch, c3, n->dxA, n->dskip[1]));
    CL_TRY(up_adjoint(n, n->dxA, n->d3, c3, 2, batch, A[2]));
    CL_TRY(wgrad(n, DEC3B, one(n->d3a, c3), A[2], 2, batch));
    CL_TRY(dgrad_act(n, DEC3B, A[2], n->d3a, 2, batch, B[2]));
    CL_TRY(wgrad(n, DEC3A, cat_up(n->bt, c4, n->s3, c3), B[2], 2, batch));
    CL_TRY(dgrad_raw(n, DEC3A, B[2], 2, batch, c4, n->dxA, n->dskip[2]));
    CL_TRY(up_adjoint(n, n->dxA, n->bt, c4, 3, batch, A[3]));
    CL_TRY(wgrad(n, BOTB, one(n->ba, c4), A[3], 3, batch));
    CL_TRY(dgrad_act(n, BOTB, A[3], n->ba, 3, batch, B[3]));
    CL_TRY(wgrad(n, BOTA, one(n->p3, c3), B[3], 3, batch));
    CL_TRY(dgrad_raw(n, BOTA, B[3], 3, batch, c3, n->dxp, nullptr));
    CL_TRY(pool_adjoint(n, n->dxp, n->dskip[2], n->s3, c3, 2, batch, A[2]));
    CL_TRY(wgrad(n, ENC3B, one(n->e3a, c3), A[2], 2, batch));
    CL_TRY(dgrad_act(n, ENC3B, A[2], n->e3a, 2, batch, B[2]));
    CL_TRY(wgrad(n, ENC3A, one(n->p2, c2), B[2], 2, batch));
    CL_TRY(dgrad_raw(n, ENC3A, B[2], 2, batch, c2, n->dxp, nullptr));
    CL_TRY(pool_adjoint(n, n->dxp, n->dskip[1], n->s2, c2, 1, batch, A[1]));
    CL_TRY(wgrad(n, ENC2B, one(n->e2a, c2), A[1], 1, batch));
    CL_TRY(dgrad_act(n, ENC2B, A[1], n->e2a, 1, batch, B[1]));
    CL_TRY(wgrad(n, ENC2A, one(n->p1, c1), B[1], 1, batch));
    CL_TRY(dgrad_raw(n, ENC2A, B[1], 1, batch, c1, n->dxp, nullptr));
    CL_TRY(pool_adjoint(n, n->dxp, n->dskip[0], n->s1, c1, 0, batch, A[0]));
    CL_TRY(wgrad(n, ENC1B, one(n->e1a, c1), A[0], 0, batch));
    CL_TRY(dgrad_act(n, ENC1B, A[0], n->e1a, 0, batch, B[0]));
    CL_TRY(wgrad(n, ENC1A, one(n->x0, kInC), B[0], 0, batch));
    return 0;
}

int check_net(const claire_net* n) {
    if (!n) { set_error("net is NULL"); return CLAIRE_EINVAL; }
    return 0;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

int check_ptr(const void* p, const char* name) {
    if (!p) { set_error("%s is NULL", name); return CLAIRE_EINVAL; }
    if (!aligned16(p)) { set_error("%s is not 16-byte aligned", name); return CLAIRE_EINVAL; }
    return 0;
}

int check_batch(const claire_net* n, int batch) {
    if (batch < 1 || batch > n->max_batch) {
        set_error("batch %d out of range [1, %d]", batch, n->max_batch);
        return CLAIRE_EINVAL;
    }
    return 0;
}

// Operands of one stand-alone layer: bfloat16 copies of x (and dz) and the
// packed forward / backward-data weights.
struct LayerScratch {
    bf16 *x16 = nullptr, *dz16 = nullptr, *wt = nullptr, *wtT = nullptr;
    void release(hipStream_t s) {
        (void)hipStreamSynchronize(s);
        dfree(x16); dfree(dz16); dfree(wt); dfree(wtT);
    }
};

int layer_setup(LayerScratch& S, const NetLayer& L, const float* x, const float* w,
                const float* dz, long long mt, hipStream_t s) {
    CL_TRY(dalloc(&S.x16, mt * L.cin));
    CL_TRY(dalloc(&S.wt, (long long)L.nrows * L.kpad));
    CL_TRY(dalloc(&S.wtT, (long long)L.nrowsT * L.kpadT));
    CL_TRY(zero16(S.wt, (long long)L.nrows * L.kpad, s));
    CL_TRY(zero16(S.wtT, (long long)L.nrowsT * L.kpadT, s));
    hipLaunchKernelGGL(k_round16, dim3(nblk(mt * L.cin)), dim3(256), 0, s, x, mt * L.cin, S.x16);
    CL_LAUNCH_CHECK();
    const int nw = L.cout * L.ktot;
    hipLaunchKernelGGL(k_adam_pack, dim3(nblk(nw)), dim3(256), 0, s, const_cast<float*>(w),
                       nullptr, nullptr, nullptr, nw, 0, 0, 0.f, 0.f, 0.f, 1.f, 1.f, 0.f, S.wt,
                       L.kpad, L.ktot, S.wtT, L.kpadT, L.cin, L.coutE);
    CL_LAUNCH_CHECK();
    if (dz) {
        CL_TRY(dalloc(&S.dz16, mt * L.cout));
        hipLaunchKernelGGL(k_round16, dim3(nblk(mt * L.cout)), dim3(256), 0, s, dz,
                           mt * L.cout, S.dz16);
        CL_LAUNCH_CHECK();
    }
    return 0;
}

NetLayer layer_geometry(int cin, int cout) {
    NetLayer L;
    L.cin = cin;
    L.cout = cout;
    L.coutE = roundup(cout, 8);
    L.ktot = 27 * cin;
    L.kpad = roundup(L.ktot, 32);
    L.nrows = roundup(cout, 16);
    L.kpadT = roundup(27 * L.coutE, 32);
    L.nrowsT = roundup(cin, 16);
    L.off = 0;
    return L;
}

int check_layer_sizes(int batch, int res, int cin, int cout) {
    if (res < 1 || res > 256 || (res & (res - 1)) || batch < 1 || cin < 8 || cin % 8 ||
        cin > 512 || cout < 1 || cout > 512 || (long long)batch * res * res * res > (1LL << 24)) {
        set_error("bad convolution sizes");
        return CLAIRE_EINVAL;
    }
    return 0;
}

}  // namespace
}  // namespace claire

extern "C" {

int claire_net_create(claire_net** out, int res, const int channels[4], int max_batch,
                      unsigned long long seed, void* stream) {
    if (!out) { set_error("out is NULL"); return CLAIRE_EINVAL; }
    *out = nullptr;
    if (res < 8 || res > 256 || (res & (res - 1))) {
        set_error("res = %d: must be a power of two in [8, 256]", res);
        return CLAIRE_EINVAL;
    }
    if (!channels) { set_error("channels is NULL"); return CLAIRE_EINVAL; }
    for (int k = 0; k < 4; ++k)
        if (channels[k] < 8 || channels[k] > 256 || channels[k] % 8) {
            set_error("channels[%d] = %d: must be a multiple of 8 in [8, 256]", k, channels[k]);
            return CLAIRE_EINVAL;
        }
    if (max_batch < 1 || (long long)max_batch * res * res * res > (1LL << 26)) {
        set_error("max_batch = %d: need 1 <= max_batch and max_batch res^3 <= 2^26", max_batch);
        return CLAIRE_EINVAL;
    }
    claire_net* n = new (std::nothrow) claire_net();
    if (!n) { set_error("host allocation failed"); return CLAIRE_ENOMEM; }
    n->R = res;
    n->l = lg2(res);
    for (int k = 0; k < 4; ++k) n->c[k] = channels[k];
    n->max_batch = max_batch;
    n->s = reinterpret_cast<hipStream_t>(stream);
    int rc = net_alloc(n);
    if (rc < 0) {
        net_release(n);
        delete n;
        return rc;
    }
    // He-uniform weights (bound sqrt(6 / fan_in), a tenth of it for the
    // output layer), zero biases; splitmix64 stream from the seed
    std::vector<float> h((size_t)n->nparam, 0.f);
    uint64_t st = seed;
    for (int i = 0; i < kLayers; ++i) {
        const NetLayer& L = n->L[i];
        double a = std::sqrt(6.0 / L.ktot);
        if (i == HEAD) a *= 0.1;
        const long long nw = (long long)L.cout * L.ktot;
        for (long long k = 0; k < nw; ++k) {
            const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
            h[(size_t)(L.off + k)] = (float)((2.0 * u - 1.0) * a);
        }
    }
    hipError_t e = hipMemcpyAsync(n->p, h.data(), sizeof(float) * h.size(),
                                  hipMemcpyHostToDevice, n->s);
    if (e == hipSuccess) e = hipStreamSynchronize(n->s);
    if (e != hipSuccess) {
        hip_fail(e, "upload of initial weights", __FILE__, __LINE__);
        net_release(n);
        delete n;
        return CLAIRE_EDEVICE;
    }
    if ((rc = reset_adam(n)) < 0 || (rc = net_pack(n, false, 0.0)) < 0) {
        net_release(n);
        delete n;
        return rc;
    }
    *out = n;
    return 0;
}

int claire_net_destroy(claire_net* n) {
    if (!n) return 0;
    (void)hipStreamSynchronize(n->s);
    net_release(n);
    delete n;
    return 0;
}

long long claire_net_param_count(const claire_net* n) { return n ? n->nparam : -1; }

int claire_net_set_params(claire_net* n, const float* params) {
    CL_TRY(check_net(n));
    CL_TRY(check_ptr(params, "params"));
    CL_HIP(hipMemcpyAsync(n->p, params, sizeof(float) * (size_t)n->nparam,
                          hipMemcpyDeviceToDevice, n->s));
    CL_TRY(reset_adam(n));
    return net_pack(n, false, 0.0);
}

int claire_net_get_params(const claire_net* n, float* params) {
    CL_TRY(check_net(n));
    CL_TRY(check_ptr(params, "params"));
    CL_HIP(hipMemcpyAsync(params, n->p, sizeof(float) * (size_t)n->nparam,
                          hipMemcpyDeviceToDevice, n->s));
    return 0;
}

int claire_net_get_grads(const claire_net* n, float* grads) {
    CL_TRY(check_net(n));
    CL_TRY(check_ptr(grads, "grads"));
    if (!n->have_grads) { set_error("no gradient computed yet"); return CLAIRE_ESTATE; }
    CL_HIP(hipMemcpyAsync(grads, n->g, sizeof(float) * (size_t)n->nparam,
                          hipMemcpyDeviceToDevice, n->s));
    return 0;
}

int claire_net_set_grads(claire_net* n, const float* grads) {
    CL_TRY(check_net(n));
    CL_TRY(check_ptr(grads, "grads"));
    CL_HIP(hipMemcpyAsync(n->g, grads, sizeof(float) * (size_t)n->nparam,
                          hipMemcpyDeviceToDevice, n->s));
    n->have_grads = true;
    return 0;
}

int claire_net_forward(claire_net* n, const float* m0, const float* m1, int batch, float* v) {
    CL_TRY(check_net(n));
    CL_TRY(check_batch(n, batch));
    CL_TRY(check_ptr(m0, "m0"));
    CL_TRY(check_ptr(m1, "m1"));
    CL_TRY(check_ptr(v, "v"));
    CL_TRY(net_forward(n, m0, m1, batch));
    const long long mt = vox_level(n, 0, batch);
    hipLaunchKernelGGL(k_out_transpose, dim3(nblk(mt)), dim3(256), 0, n->s, n->vout, n->l,
                       (int)mt, v);
    CL_LAUNCH_CHECK();
    return 0;
}

int claire_net_loss_grad(claire_net* n, const float* m0, const float* m1, const float* v_target,
                         int batch, double* loss, float* v) {
    CL_TRY(check_net(n));
    CL_TRY(check_batch(n, batch));
    CL_TRY(check_ptr(m0, "m0"));
    CL_TRY(check_ptr(m1, "m1"));
    CL_TRY(check_ptr(v_target, "v_target"));
    if (v) CL_TRY(check_ptr(v, "v"));
    CL_TRY(net_forward(n, m0, m1, batch));
    const long long mt = vox_level(n, 0, batch);
    const double N = (double)mt * kOutC;
    hipLaunchKernelGGL(k_mse, dim3(nblk(mt)), dim3(256), 0, n->s, n->vout, v_target, n->l,
                       (int)mt, (float)(2.0 / N), n->dzh, n->red.partial);
    CL_LAUNCH_CHECK();
    CL_TRY(red_fold_sum(n->red, (int)nblk(mt), 1, 0, 0, n->s));
    if (v) {
        hipLaunchKernelGGL(k_out_transpose, dim3(nblk(mt)), dim3(256), 0, n->s, n->vout, n->l,
                           (int)mt, v);
        CL_LAUNCH_CHECK();
    }
    CL_TRY(net_backward(n, batch));
    n->have_grads = true;
    CL_TRY(red_fetch(n->red, n->s));
    if (loss) *loss = n->red.host[0] / N;
    return 0;
}

int claire_net_adam_step(claire_net* n, double lr) {
    CL_TRY(check_net(n));
    if (!n->have_grads) { set_error("no gradient computed yet"); return CLAIRE_ESTATE; }
    if (!(lr > 0.0)) { set_error("lr must be positive"); return CLAIRE_EINVAL; }
    return net_pack(n, true, lr);
}

int claire_net_train_step(claire_net* n, const float* m0, const float* m1, const float* v_target,
                          int batch, double lr, double* loss) {
    CL_TRY(claire_net_loss_grad(n, m0, m1, v_target, batch, loss, nullptr));
    return claire_net_adam_step(n, lr);
}

int claire_net_warm_start(claire_net* n, const float* m0, const float* m1, int nx, float* v0) {
    CL_TRY(check_net(n));
    CL_TRY(check_ptr(m0, "m0"));
    CL_TRY(check_ptr(m1, "m1"));
    CL_TRY(check_ptr(v0, "v0"));
    if (nx < n->R || nx > 1024 || (nx & (nx - 1))) {
        set_error("n = %d: must be a power of two in [%d, 1024]", nx, n->R);
        return CLAIRE_EINVAL;
    }
    const long long R3 = (long long)n->R * n->R * n->R;
    const long long big = 3LL * nx * nx * nx;
    if (big > n->ws_cap) {
        (void)hipStreamSynchronize(n->s);
        dfree(n->ws_a); dfree(n->ws_b); dfree(n->ws_v); dfree(n->ws_t0); dfree(n->ws_t1);
        n->ws_a = n->ws_b = n->ws_v = n->ws_t0 = n->ws_t1 = nullptr;
        n->ws_cap = 0;
        CL_TRY(dalloc(&n->ws_a, R3));
        CL_TRY(dalloc(&n->ws_b, R3));
        CL_TRY(dalloc(&n->ws_v, 3 * R3));
        CL_TRY(dalloc(&n->ws_t0, big));
        CL_TRY(dalloc(&n->ws_t1, big));
        n->ws_cap = big;
    }
    CL_TRY(resample(m0, nx, n->ws_a, n->R, 1, n->ws_t0, n->ws_t1, n->s));
    CL_TRY(resample(m1, nx, n->ws_b, n->R, 1, n->ws_t0, n->ws_t1, n->s));
    CL_TRY(claire_net_forward(n, n->ws_a, n->ws_b, 1, n->ws_v));
    return resample(n->ws_v, n->R, v0, nx, 3, n->ws_t0, n->ws_t1, n->s);
}

int claire_resample(const float* src, int n_src, float* dst, int n_dst, int ncomp, void* stream) {
    CL_TRY(check_ptr(src, "src"));
    CL_TRY(check_ptr(dst, "dst"));
    auto ok = [](int v) { return v >= 1 && v <= 1024 && (v & (v - 1)) == 0; };
    if (!ok(n_src) || !ok(n_dst)) {
        set_error("extents must be powers of two in [1, 1024]");
        return CLAIRE_EINVAL;
    }
    if (ncomp < 1 || ncomp > 16) { set_error("ncomp must be in [1, 16]"); return CLAIRE_EINVAL; }
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int nm = n_src > n_dst ? n_src : n_dst;
    const long long big = (long long)ncomp * nm * nm * nm;
    float *t0 = nullptr, *t1 = nullptr;
    int rc = 0;
    if ((rc = dalloc(&t0, big)) >= 0 && (rc = dalloc(&t1, big)) >= 0)
        rc = resample(src, n_src, dst, n_dst, ncomp, t0, t1, s);
    (void)hipStreamSynchronize(s);
    dfree(t0);
    dfree(t1);
    return rc < 0 ? rc : 0;
}

int claire_conv3d(const float* x, const float* w, const float* b, int batch, int res, int cin,
                  int cout, int act, float* y, void* stream) {
    CL_TRY(check_ptr(x, "x"));
    CL_TRY(check_ptr(w, "w"));
    CL_TRY(check_ptr(y, "y"));
    CL_TRY(check_layer_sizes(batch, res, cin, cout));
    if (act != 0 && act != 1) { set_error("act must be 0 or 1"); return CLAIRE_EINVAL; }
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const long long mt = (long long)batch * res * res * res;
    const NetLayer L = layer_geometry(cin, cout);
    LayerScratch S;
    float* part = nullptr;
    const long long part_cap = (long long)conv_splits(mt, L.nrows, L.kpad) * mt * L.nrows;
    int rc = layer_setup(S, L, x, w, nullptr, mt, s);
    if (rc >= 0) rc = dalloc(&part, part_cap);
    if (rc >= 0) {
        ConvOut o{};
        o.bias = b;
        o.y32 = y;
        rc = act ? conv<EPI_ACT32>(one(S.x16, cin), S.wt, L.kpad, L.nrows, cout, lg2(res), mt, o,
                                   s, part, part_cap)
                 : conv<EPI_LINEAR>(one(S.x16, cin), S.wt, L.kpad, L.nrows, cout, lg2(res), mt,
                                    o, s, part, part_cap);
    }
    S.release(s);
    dfree(part);
    return rc < 0 ? rc : 0;
}

int claire_conv3d_backward(const float* x, const float* w, const float* dz, int batch, int res,
                           int cin, int cout, float* dx, float* dw, float* db, void* stream) {
    CL_TRY(check_ptr(x, "x"));
    CL_TRY(check_ptr(w, "w"));
    CL_TRY(check_ptr(dz, "dz"));
    CL_TRY(check_ptr(dx, "dx"));
    CL_TRY(check_ptr(dw, "dw"));
    CL_TRY(check_ptr(db, "db"));
    CL_TRY(check_layer_sizes(batch, res, cin, cout));
    if (cout % 8) { set_error("cout must be a multiple of 8"); return CLAIRE_EINVAL; }
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const long long mt = (long long)batch * res * res * res;
    const int l = lg2(res);
    const NetLayer L = layer_geometry(cin, cout);
    LayerScratch S;
    float *partial = nullptr, *pb = nullptr;
    int splits, chunk;
    wgrad_split(mt, splits, chunk);
    // one buffer for the data gradient's reduction splits and, after it on
    // the same stream, the weight gradient's partial sums
    long long part_cap = (long long)splits * L.nrows * L.kpad;
    const long long dcap = (long long)conv_splits(mt, L.nrowsT, L.kpadT) * mt * L.nrowsT;
    if (dcap > part_cap) part_cap = dcap;
    int rc = layer_setup(S, L, x, w, dz, mt, s);
    if (rc >= 0) rc = dalloc(&partial, part_cap);
    if (rc >= 0) rc = dalloc(&pb, (long long)splits * L.coutE);
    if (rc >= 0) {
        ConvOut o{};
        o.y32 = dx;
        o.csplit = cin;
        rc = conv<EPI_DGRAD_RAW>(one(S.dz16, cout), S.wtT, L.kpadT, L.nrowsT, cin, l, mt, o, s,
                                 partial, part_cap);
    }
    if (rc >= 0) {
        const int ktiles = (L.kpad + 255) / 256;
        const dim3 wgrid((unsigned)((L.nrows / 16) * ktiles), (unsigned)splits);
        if (wgrad_brick(one(S.x16, cin), S.dz16, cout, l, mt, splits, L.nrows, L.kpad,
                        partial, part_cap, pb, (long long)splits * L.coutE, s)) {
        } else if (kWgradLds && cin % 8 == 0 && cout % 8 == 0) {
            hipLaunchKernelGGL(k_wgrad_lds, wgrid, dim3(256), 0, s, one(S.x16, cin), S.dz16,
                               cout, l, (int)mt, L.kpad, ktiles, chunk, partial, L.nrows, pb);
        } else {
            hipLaunchKernelGGL(k_wgrad, wgrid, dim3(256), 0, s, one(S.x16, cin), S.dz16, cout,
                               l, (int)mt, L.kpad, ktiles, chunk, partial, L.nrows);
            hipLaunchKernelGGL(k_bias_partial, dim3(splits), dim3(256), 0, s, S.dz16, cout,
                               (int)mt, chunk, pb);
        }
        const long long nw = (long long)cout * L.ktot;
        hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((nw + cout + kRedOut - 1) / kRedOut)),
                           dim3(256), 0,
                           s, partial, pb,
                           splits, L.nrows, L.kpad, cout, L.ktot, cout, dw, db);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = hip_fail(e, "weight gradient", __FILE__, __LINE__);
    }
    S.release(s);
    dfree(partial);
    dfree(pb);
    return rc < 0 ? rc : 0;
}

}  // extern "C"
