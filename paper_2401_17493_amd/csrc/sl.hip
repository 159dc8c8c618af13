// Semi-Lagrangian kernels (Section 2.5.2) with tricubic Lagrange
// interpolation (Section 2.5.4, p = 3).
//
// Departure points are stored as displacements in voxel units, d = (y - x)/h,
// so a query is (integer grid index) + (float displacement): the stencil
// origin floor(d) is exact and a zero displacement returns grid values
// bit-for-bit. Output voxels run x3 fastest across the wavefront (the
// LDS-staged gathers take two voxels per thread); the 4x4x4 stencil is read
// with wrapped indices: a mask when the extents are
// powers of two, a wrap by subtraction (box staging) or modulo (direct
// gathers) along x1 and x2 on grids with other extents. Single-field gathers
// and the backtrace are LDS-staged on every grid (ragged bricks on general
// ones); multi-field interpolation reads its stencils directly.

#include "internal.h"

#include <hip/hip_fp16.h>

namespace claire {
namespace {

constexpr int kThreads = 256;

struct G3 {
    int m1, m2, m3;     // extent - 1 (masks; m3 only on general grids)
    int l2, l3;         // shifts
    int s1;             // l2 + l3
    int n1, n2;         // extents (general grids: modulo wrap along x1, x2)
};

G3 make_g3(const Geo& g) {
    G3 r;
    r.m1 = g.n1 - 1;
    r.m2 = g.n2 - 1;
    r.m3 = g.n3 - 1;
    r.l2 = g.l2;
    r.l3 = g.l3;
    r.s1 = g.l2 + g.l3;
    r.n1 = g.n1;
    r.n2 = g.n2;
    return r;
}

__device__ __forceinline__ int wrapn(int x, int n) {
    const int r = x % n;
    return r < 0 ? r + n : r;
}

// Cubic Lagrange basis through nodes -1, 0, 1, 2 at fractional offset t.
__device__ __forceinline__ void cubic_basis(float t, float w[4]) {
    const float tp = t + 1.0f, tm = t - 1.0f, tmm = t - 2.0f;
    const float a = t * tm;             // t (t - 1)
    const float b = tp * tmm;           // (t + 1)(t - 2)
    w[0] = -(1.0f / 6.0f) * a * tmm;
    w[1] = 0.5f * b * tm;
    w[2] = -0.5f * b * t;
    w[3] = (1.0f / 6.0f) * a * tp;
}

// Stencil of the point (i1, i2, i3) + (d1, d2, d3).
struct Stencil {
    int o1[4], o2[4], o3[4];
    float w1[4], w2[4], w3[4];
};

template <bool GEN = false>
__device__ __forceinline__ void make_stencil(const G3& g, int i1, int i2, int i3, float d1,
                                             float d2, float d3, Stencil& st) {
    const float f1 = floorf(d1), f2 = floorf(d2), f3 = floorf(d3);
    const int b1 = i1 + (int)f1 - 1, b2 = i2 + (int)f2 - 1, b3 = i3 + (int)f3 - 1;
    cubic_basis(d1 - f1, st.w1);
    cubic_basis(d2 - f2, st.w2);
    cubic_basis(d3 - f3, st.w3);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if constexpr (GEN) {
            st.o1[q] = (wrapn(b1 + q, g.n1) * g.n2) << g.l3;
            st.o2[q] = wrapn(b2 + q, g.n2) << g.l3;
        } else {
            st.o1[q] = ((b1 + q) & g.m1) << g.s1;
            st.o2[q] = ((b2 + q) & g.m2) << g.l3;
        }
        st.o3[q] = (b3 + q) & g.m3;
    }
}

// element loads of float or half fields, widened to float
__device__ __forceinline__ float ldf(const float* p) { return *p; }
__device__ __forceinline__ float ldf(const __half* p) { return __half2float(*p); }

// Element i of a field with a uniform base pointer: the per-lane offset is a
// 32-bit byte offset (i < 2^30), so the load takes the scalar-base +
// vector-offset form with no 64-bit address arithmetic per lane.
__device__ __forceinline__ float ldi(const float* p, unsigned i) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(p) + (i << 2));
}
__device__ __forceinline__ float ldi(const __half* p, unsigned i) {
    return __half2float(
        *reinterpret_cast<const __half*>(reinterpret_cast<const char*>(p) + (i << 1)));
}
__device__ __forceinline__ float4 ldi4(const float* p, unsigned i) {
    return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(p) + (i << 2));
}
__device__ __forceinline__ void sti(float* p, unsigned i, float v) {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(p) + (i << 2)) = v;
}

template <int NF, typename T = float>
__device__ __forceinline__ void gather(const T* __restrict__ f, long long fstride,
                                       const Stencil& st, float out[NF]) {
#pragma unroll
    for (int k = 0; k < NF; ++k) out[k] = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int row = st.o1[a] + st.o2[b];
            const float wab = st.w1[a] * st.w2[b];
#pragma unroll
            for (int k = 0; k < NF; ++k) {
                const T* p = f + k * fstride + row;
                float t = st.w3[0] * ldf(p + st.o3[0]);
                t = fmaf(st.w3[1], ldf(p + st.o3[1]), t);
                t = fmaf(st.w3[2], ldf(p + st.o3[2]), t);
                t = fmaf(st.w3[3], ldf(p + st.o3[3]), t);
                out[k] = fmaf(wab, t, out[k]);
            }
        }
    }
}

__device__ __forceinline__ void coords(const G3& g, long long idx, int& i1, int& i2, int& i3) {
    i3 = (int)(idx & g.m3);
    i2 = (int)((idx >> g.l3) & g.m2);
    i1 = (int)(idx >> g.s1);
}

// ------------------------------------------------------------------------
// LDS-staged single-field gathers (the state, adjoint and incremental steps).
//
// A workgroup owns an output brick of 4 x 8 x 16 voxels. The bounding box of
// all the brick's 4x4x4 stencils comes from a per-brick table computed once
// per departure field (the departure points are fixed for a velocity and
// reused by every state, adjoint and incremental step) or, without a table,
// from a block reduction over the brick's displacements. The box of the
// source field is copied into LDS with row-contiguous loads and the values
// are interpolated from LDS: 64 LDS reads per voxel instead of 64 scattered
// global loads, which otherwise saturate the vector-memory address path long
// before HBM. With the table, the box, displacement and epilogue loads are
// all in flight together. A brick whose box exceeds the LDS budget (extreme
// local deformation) gathers directly from global memory instead. Bricks are
// handed out so that each XCD sweeps a contiguous slab of the grid, keeping
// the halo rows shared by neighbouring bricks in one L2.
// 5080 floats of box plus the reduction scratch: eight workgroups fill a
// CU's 160 KiB of LDS (the occupancy the kernels are compiled for). The
// boxes of strongly deformed velocities (local spread of the stencil origins
// of several voxels) still fit; a brick whose box does not gathers from
// global memory at several times the cost.
#ifndef CLAIRE_GATHER_BOXCAP
#define CLAIRE_GATHER_BOXCAP 5080
#endif
#ifndef CLAIRE_GATHER_VOX
#define CLAIRE_GATHER_VOX 2
#endif
constexpr int kBoxCap = CLAIRE_GATHER_BOXCAP;  // floats of LDS per workgroup
constexpr int kVox = CLAIRE_GATHER_VOX;        // voxels per thread: brick = 256 kVox voxels
constexpr int kLogVox = kVox == 1 ? 0 : (kVox == 2 ? 1 : 2);
#ifndef CLAIRE_GATHER_WAVES
#define CLAIRE_GATHER_WAVES 8
#endif
// waves per SIMD the gather kernels are compiled for (bounds their VGPRs)
constexpr int kGatherWaves = CLAIRE_GATHER_WAVES;
// The backtrace stages full-step departure boxes (larger) for three fields
// in turn: its own LDS budget and occupancy target.
constexpr int kBoxCapBT = 6144;
constexpr int kBacktraceWaves = 4;

struct Brick {
    int lb1, lb2, lb3;     // log2 of the brick extents
    int lnb2, lnb3;        // log2 of the bricks per axis along x2, x3
    int nbricks;
    int nb2, nb3;          // bricks along x2, x3 (general grids: the last ones ragged)
};

// brick 2^(1 + log2 kVox) x 8 x 16 (4 x 8 x 16 for kVox = 2), clipped to the grid
Brick make_brick(const Geo& g) {
    Brick b;
    if (!g.pow2) {
        // general grids (n1, n2 >= 8): full 2^(1+log2 kVox) x 8 x 16 bricks,
        // ragged along x1 and x2 at the high end
        b.lb1 = 1 + kLogVox;
        b.lb2 = 3;
        b.lb3 = g.l3 < 4 ? g.l3 : 4;
        b.nb2 = (g.n2 + 7) >> 3;
        b.nb3 = g.n3 >> b.lb3;
        b.lnb2 = b.lnb3 = 0;
        b.nbricks = ((g.n1 + (1 << b.lb1) - 1) >> b.lb1) * b.nb2 * b.nb3;
        return b;
    }
    b.lb1 = g.l1 < 1 + kLogVox ? g.l1 : 1 + kLogVox;
    b.lb2 = g.l2 < 3 ? g.l2 : 3;
    b.lb3 = g.l3 < 4 ? g.l3 : 4;
    b.lnb2 = g.l2 - b.lb2;
    b.lnb3 = g.l3 - b.lb3;
    b.nbricks = 1 << (g.l1 - b.lb1 + b.lnb2 + b.lnb3);
    b.nb2 = 1 << b.lnb2;
    b.nb3 = 1 << b.lnb3;
    return b;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Epilogues: combine the interpolated value u at voxel i with pointwise data.
// load() fetches the pointwise inputs early (before the box is staged) so
// their latency overlaps the staging; store() writes the result.
struct EpiStore {        // out = u
    float* out;
    struct Pre {};
    __device__ Pre load(unsigned) const { return Pre{}; }
    __device__ void store(unsigned i, float u, const Pre&) const { sti(out, i, u); }
};
struct EpiScale {        // out = A u  (continuity-equation step along -v)
    const float* A;
    float* out;
    struct Pre { float a; };
    __device__ Pre load(unsigned i) const { return Pre{ldi(A, i)}; }
    __device__ void store(unsigned i, float u, const Pre& p) const { sti(out, i, p.a * u); }
};
template <typename GT>      // GT: storage of grad m (float, or half in the mixed matvec)
struct EpiIncState {     // out = sign (u + coef f), f = -grad m . v~
    const GT* gm;
    const float* vt;
    float* out;
    long long n;
    float coef, sign;
    struct Pre { float f; };
    __device__ Pre load(unsigned i) const {
        return Pre{-(ldi(gm, i) * ldi(vt, i) + ldi(gm + n, i) * ldi(vt + n, i) +
                     ldi(gm + 2 * n, i) * ldi(vt + 2 * n, i))};
    }
    __device__ void store(unsigned i, float u, const Pre& p) const {
        sti(out, i, sign * (u + coef * p.f));
    }
};
struct EpiMakeA {        // out = 1 + (h_t/2)(D(y-) + D + h_t D(y-) D)
    const float* D;
    float* out;
    float ht;
    struct Pre { float dx; };
    __device__ Pre load(unsigned i) const { return Pre{ldi(D, i)}; }
    __device__ void store(unsigned i, float u, const Pre& p) const {
        sti(out, i, 1.0f + 0.5f * ht * (u + p.dx + ht * u * p.dx));
    }
};

// Brick owned by this workgroup (XCD-contiguous order) and its voxels.
struct BrickPos {
    int o1, o2, o3;    // first voxel
    int bvol;          // voxels in the brick
    int id;            // brick index (x3 fastest), independent of the launch order
};

template <bool GEN>
__device__ __forceinline__ BrickPos brick_pos(const Brick& br) {
    int bid = blockIdx.x;
    if ((br.nbricks & 7) == 0) bid = (bid & 7) * (br.nbricks >> 3) + (bid >> 3);
    BrickPos p;
    if constexpr (GEN) {
        const int r = bid / br.nb3;
        p.o3 = (bid - r * br.nb3) << br.lb3;
        const int r2 = r / br.nb2;
        p.o2 = (r - r2 * br.nb2) << br.lb2;
        p.o1 = r2 << br.lb1;
    } else {
        p.o3 = (bid & ((1 << br.lnb3) - 1)) << br.lb3;
        p.o2 = ((bid >> br.lnb3) & ((1 << br.lnb2) - 1)) << br.lb2;
        p.o1 = (bid >> (br.lnb3 + br.lnb2)) << br.lb1;
    }
    p.bvol = 1 << (br.lb1 + br.lb2 + br.lb3);
    p.id = bid;
    return p;
}

// k-th voxel of this thread: grid coordinates and linear index (false if
// none). Order within the brick: x3 fastest, then x1, then x2, so the 64 lanes
// of a wave cover 16 x3 voxels in each of 4 x1 planes of one x2 row.
template <bool GEN>
__device__ __forceinline__ bool brick_voxel(const G3& g, const Brick& br, const BrickPos& p,
                                            int k, int& i1, int& i2, int& i3, unsigned& idx) {
    const int v = threadIdx.x + k * kThreads;
    if (v >= p.bvol) return false;
    i3 = p.o3 + (v & ((1 << br.lb3) - 1));
    i1 = p.o1 + ((v >> br.lb3) & ((1 << br.lb1) - 1));
    i2 = p.o2 + (v >> (br.lb3 + br.lb1));
    if constexpr (GEN) {
        if (i1 >= g.n1 || i2 >= g.n2) return false;   // ragged brick
        idx = ((unsigned)(i1 * g.n2 + i2) << g.l3) | (unsigned)i3;
    } else {
        idx = ((unsigned)i1 << g.s1) | ((unsigned)i2 << g.l3) | (unsigned)i3;
    }
    return true;
}

// Box covering all stencil origins: [lo, lo + e) per axis (e = spread of
// the origins + 4). In LDS each x3 row holds whole aligned float4 segments:
// columns cb .. cb + p3 - 1 with cb = lo3 rounded down to a multiple of 4 and
// p3 = 4 ng, so the box is staged with 16-byte loads and stores (n3 is a
// multiple of 4: a segment never straddles the periodic wrap). Rows of one x1
// plane are p3 apart and planes pp = e2 p3 + pad apart with pp = 16 mod 64:
// the four 16-lane groups of a wave read four different planes, and with that
// pitch their addresses fall in disjoint LDS banks (32 banks per half wave or
// 64 per wave alike) as long as each group reads a contiguous run.
struct Box {
    int lo1, lo2, lo3, e1, e2, e3;
    int cb, ng, p3, pp;
    long long vol;     // LDS floats, e1 pp
};

__device__ __forceinline__ void box_layout(Box& b) {
    b.cb = b.lo3 & ~3;
    b.ng = ((b.lo3 + b.e3 - 1 - b.cb) >> 2) + 1;
    b.p3 = 4 * b.ng;
    const long long plane = (long long)b.e2 * b.p3;
    b.pp = (int)(plane + ((16 - plane) & 63));
    b.vol = (long long)b.e1 * b.pp;
}

// Block reduction of the per-thread origin bounds mn/mx through `red`.
// Contains a barrier; callers must not be reading `red` from an earlier call.
__device__ __forceinline__ Box reduce_box(int mn1, int mn2, int mn3, int mx1, int mx2, int mx3,
                                          int (*red)[6]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    mn1 = wave_min(mn1); mn2 = wave_min(mn2); mn3 = wave_min(mn3);
    mx1 = wave_max(mx1); mx2 = wave_max(mx2); mx3 = wave_max(mx3);
    if (lane == 0) {
        red[wid][0] = mn1; red[wid][1] = mn2; red[wid][2] = mn3;
        red[wid][3] = mx1; red[wid][4] = mx2; red[wid][5] = mx3;
    }
    __syncthreads();
    int lo1 = red[0][0], lo2 = red[0][1], lo3 = red[0][2];
    int hi1 = red[0][3], hi2 = red[0][4], hi3 = red[0][5];
#pragma unroll
    for (int w = 1; w < kThreads / 64; ++w) {
        lo1 = min(lo1, red[w][0]); lo2 = min(lo2, red[w][1]); lo3 = min(lo3, red[w][2]);
        hi1 = max(hi1, red[w][3]); hi2 = max(hi2, red[w][4]); hi3 = max(hi3, red[w][5]);
    }
    Box b;
    b.lo1 = lo1; b.lo2 = lo2; b.lo3 = lo3;
    b.e1 = hi1 - lo1 + 4; b.e2 = hi2 - lo2 + 4; b.e3 = hi3 - lo3 + 4;
    box_layout(b);
    return b;
}

// Copy the box of field `src` into LDS (requires b.vol within the LDS
// budget; rows e1 e2 < 2^14). Row `row` = a1 e2 + a2 starts at LDS float
// a1 pp + a2 p3 and holds columns cb .. cb + p3 - 1 as ng float4 segments. A
// thread always moves segment j = tid mod ng of rows tid / ng + k (kThreads /
// ng): one division per segment. Batches of independent 16-byte loads, then
// the 16-byte LDS stores.
constexpr int kSegBatch = 4;
template <bool GEN>
__device__ __forceinline__ void stage_box(float* box, const float* __restrict__ src, const G3& g,
                                          const Box& b) {
    const int nrows = b.e1 * b.e2;
    const int rpp = kThreads / b.ng;               // rows per pass
    int j;
    int r0 = quot((int)threadIdx.x, b.ng, quot_inv(b.ng), j);
    if (r0 >= rpp) r0 = nrows;                     // idle lanes of the last partial row set
    const unsigned col = (unsigned)((b.cb + 4 * j) & g.m3);
    const float inv_e2 = quot_inv(b.e2);
    float4* box4 = reinterpret_cast<float4*>(box);
    // general grids: the box origin wrapped once; a row index then wraps with
    // one subtraction (a second only for boxes wider than the grid)
    int lo1w = 0, lo2w = 0;
    if constexpr (GEN) {
        lo1w = wrapn(b.lo1, g.n1);
        lo2w = wrapn(b.lo2, g.n2);
    }
    auto wrap_up = [](int i, int n) {
        if (i >= n) {
            i -= n;
            if (i >= n) i %= n;
        }
        return i;
    };
    for (int r = r0; r < nrows; r += rpp * kSegBatch) {
        float4 tmp[kSegBatch];
        unsigned at[kSegBatch];   // LDS float4 index of each segment
#pragma unroll
        for (int u = 0; u < kSegBatch; ++u) {
            const int row = r + u * rpp;
            if (row < nrows) {
                int a2;
                const int a1 = quot(row, b.e2, inv_e2, a2);
                unsigned off;
                if constexpr (GEN)
                    off = ((unsigned)(wrap_up(lo1w + a1, g.n1) * g.n2 + wrap_up(lo2w + a2, g.n2))
                           << g.l3) | col;
                else
                    off = ((unsigned)((b.lo1 + a1) & g.m1) << g.s1) |
                          ((unsigned)((b.lo2 + a2) & g.m2) << g.l3) | col;
                tmp[u] = ldi4(src, off);
                at[u] = __umul24((unsigned)a1, (unsigned)(b.pp >> 2)) +
                        __umul24((unsigned)a2, (unsigned)b.ng) + j;
            }
        }
#pragma unroll
        for (int u = 0; u < kSegBatch; ++u)
            if (r + u * rpp < nrows) box4[at[u]] = tmp[u];
    }
}

// Tricubic value from the staged box at stencil origin q (grid units) with
// fractional offsets given by the displacement d: sum_a w1_a sum_c w2_c
// sum_k w3_k f(q + (a, c, k)).
__device__ __forceinline__ float interp_box(const float* box, const Box& b, const int q[3],
                                            const float d[3]) {
    float w1[4], w2[4], w3[4];
    cubic_basis(d[0] - floorf(d[0]), w1);
    cubic_basis(d[1] - floorf(d[1]), w2);
    cubic_basis(d[2] - floorf(d[2]), w3);
    const int plane = b.pp;
    const float* p0 = box + (q[0] - b.lo1) * b.pp + (q[1] - b.lo2) * b.p3 + (q[2] - b.cb);
    float acc = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        float sa = 0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float* p = p0 + a * plane + c * b.p3;
            float t = w3[0] * p[0];
            t = fmaf(w3[1], p[1], t);
            t = fmaf(w3[2], p[2], t);
            t = fmaf(w3[3], p[3], t);
            sa = c == 0 ? w2[0] * t : fmaf(w2[c], t, sa);
        }
        acc = a == 0 ? w1[0] * sa : fmaf(w1[a], sa, acc);
    }
    return acc;
}

// Tricubic value by direct global gathers (bricks whose box does not fit).
template <bool GEN, typename T>
__device__ __forceinline__ float interp_global(const T* __restrict__ src, const G3& g,
                                               long long n, int i1, int i2, int i3,
                                               const float d[3]) {
    Stencil st;
    make_stencil<GEN>(g, i1, i2, i3, d[0], d[1], d[2], st);
    float u;
    gather<1, T>(src, n, st, &u);
    return u;
}

// Per-brick stencil bounding boxes of a departure field: 6 ints per brick
// (lo1, lo2, lo3, e1, e2, e3), indexed by BrickPos::id.
template <bool GEN>
__global__ __launch_bounds__(kThreads) void k_brick_boxes(const float* __restrict__ d,
                                                          int* __restrict__ table, G3 g,
                                                          Brick br, long long n) {
    __shared__ int red[kThreads / 64][6];
    const BrickPos bp = brick_pos<GEN>(br);
    int mn1 = 1 << 30, mn2 = 1 << 30, mn3 = 1 << 30;
    int mx1 = -(1 << 30), mx2 = -(1 << 30), mx3 = -(1 << 30);
#pragma unroll
    for (int k = 0; k < kVox; ++k) {
        int i1, i2, i3;
        unsigned idx;
        if (brick_voxel<GEN>(g, br, bp, k, i1, i2, i3, idx)) {
            const int q1 = i1 + (int)floorf(ldi(d, idx)) - 1;
            const int q2 = i2 + (int)floorf(ldi(d + n, idx)) - 1;
            const int q3 = i3 + (int)floorf(ldi(d + 2 * n, idx)) - 1;
            mn1 = min(mn1, q1); mx1 = max(mx1, q1);
            mn2 = min(mn2, q2); mx2 = max(mx2, q2);
            mn3 = min(mn3, q3); mx3 = max(mx3, q3);
        }
    }
    const Box b = reduce_box(mn1, mn2, mn3, mx1, mx2, mx3, red);
    if (threadIdx.x == 0) {
        int* t = table + 6 * bp.id;
        t[0] = b.lo1; t[1] = b.lo2; t[2] = b.lo3;
        t[3] = b.e1; t[4] = b.e2; t[5] = b.e3;
    }
}

// Single-field gather u = src(x + d(x)) with epilogue; `table` holds the
// per-brick boxes of d (NULL: reduce them here).
template <class Epi, bool GEN>
__global__ __launch_bounds__(kThreads, kGatherWaves) void k_gather_lds(
    const float* __restrict__ src, const float* __restrict__ d, const int* __restrict__ table,
    Epi epi, G3 g, Brick br, long long n) {
    __shared__ __align__(16) float box[kBoxCap];
    __shared__ int red[kThreads / 64][6];
    const BrickPos bp = brick_pos<GEN>(br);
    float dd[kVox][3];
    int q[kVox][3];
    int ii[kVox][3];
    unsigned gi[kVox];
    bool on[kVox];
    typename Epi::Pre pre[kVox];
    int mn1 = 1 << 30, mn2 = 1 << 30, mn3 = 1 << 30;
    int mx1 = -(1 << 30), mx2 = -(1 << 30), mx3 = -(1 << 30);
#pragma unroll
    for (int k = 0; k < kVox; ++k) {
        on[k] = brick_voxel<GEN>(g, br, bp, k, ii[k][0], ii[k][1], ii[k][2], gi[k]);
        if (on[k]) {
            dd[k][0] = ldi(d, gi[k]);
            dd[k][1] = ldi(d + n, gi[k]);
            dd[k][2] = ldi(d + 2 * n, gi[k]);
            pre[k] = epi.load(gi[k]);
        }
    }
    Box b;
    if (table) {
        const int* t = table + 6 * bp.id;
        b.lo1 = t[0]; b.lo2 = t[1]; b.lo3 = t[2];
        b.e1 = t[3]; b.e2 = t[4]; b.e3 = t[5];
        box_layout(b);
        if (b.vol <= kBoxCap) stage_box<GEN>(box, src, g, b);
    }
#pragma unroll
    for (int k = 0; k < kVox; ++k) {
        if (!on[k]) continue;
#pragma unroll
        for (int a = 0; a < 3; ++a) q[k][a] = ii[k][a] + (int)floorf(dd[k][a]) - 1;
        mn1 = min(mn1, q[k][0]); mx1 = max(mx1, q[k][0]);
        mn2 = min(mn2, q[k][1]); mx2 = max(mx2, q[k][1]);
        mn3 = min(mn3, q[k][2]); mx3 = max(mx3, q[k][2]);
    }
    if (!table) {
        b = reduce_box(mn1, mn2, mn3, mx1, mx2, mx3, red);
        if (b.vol <= kBoxCap) stage_box<GEN>(box, src, g, b);
    }
    if (b.vol <= kBoxCap) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kVox; ++k)
            if (on[k]) epi.store(gi[k], interp_box(box, b, q[k], dd[k]), pre[k]);
    } else {
#pragma unroll
        for (int k = 0; k < kVox; ++k)
            if (on[k])
                epi.store(gi[k],
                          interp_global<GEN>(src, g, n, ii[k][0], ii[k][1], ii[k][2], dd[k]),
                          pre[k]);
    }
}

// RK2 backtrace for +v and -v (Section 2.5.2), LDS-staged:
//   y~ = x - s h_t v(x),  y = x - s (h_t/2) (v(x) + v(y~)),  s = +1, -1.
// c_a = h_t / h_a converts velocity to voxels per step. For each direction
// the three components of v are staged through the brick's box in turn.
template <bool GEN>
__global__ __launch_bounds__(kThreads, kBacktraceWaves) void k_backtrace_lds(
    const float* __restrict__ v, float* __restrict__ dp, float* __restrict__ dm, G3 g, Brick br,
    long long n, float c1, float c2, float c3) {
    __shared__ __align__(16) float box[kBoxCapBT];
    __shared__ int red[kThreads / 64][6];
    const BrickPos bp = brick_pos<GEN>(br);
    const float c[3] = {c1, c2, c3};
    float vx[kVox][3];
    int ii[kVox][3];
    unsigned gi[kVox];
    bool on[kVox];
#pragma unroll
    for (int k = 0; k < kVox; ++k) {
        on[k] = brick_voxel<GEN>(g, br, bp, k, ii[k][0], ii[k][1], ii[k][2], gi[k]);
        if (on[k]) {
#pragma unroll
            for (int a = 0; a < 3; ++a) vx[k][a] = ldi(v + a * n, gi[k]);
        }
    }
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        const float sg = dir == 0 ? -1.f : 1.f;   // y~ = x + sg h_t v(x)
        float dd[kVox][3];
        int q[kVox][3];
        int mn1 = 1 << 30, mn2 = 1 << 30, mn3 = 1 << 30;
        int mx1 = -(1 << 30), mx2 = -(1 << 30), mx3 = -(1 << 30);
#pragma unroll
        for (int k = 0; k < kVox; ++k) {
            if (!on[k]) continue;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                dd[k][a] = sg * c[a] * vx[k][a];
                q[k][a] = ii[k][a] + (int)floorf(dd[k][a]) - 1;
            }
            mn1 = min(mn1, q[k][0]); mx1 = max(mx1, q[k][0]);
            mn2 = min(mn2, q[k][1]); mx2 = max(mx2, q[k][1]);
            mn3 = min(mn3, q[k][2]); mx3 = max(mx3, q[k][2]);
        }
        __syncthreads();   // `red` and `box` of the previous direction are free
        const Box b = reduce_box(mn1, mn2, mn3, mx1, mx2, mx3, red);
        const bool fits = b.vol <= kBoxCapBT;
        float u[kVox][3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float* src = v + f * n;
            if (fits) {
                if (f > 0) __syncthreads();   // previous component's reads are done
                stage_box<GEN>(box, src, g, b);
                __syncthreads();
#pragma unroll
                for (int k = 0; k < kVox; ++k)
                    if (on[k]) u[k][f] = interp_box(box, b, q[k], dd[k]);
            } else {
#pragma unroll
                for (int k = 0; k < kVox; ++k)
                    if (on[k])
                        u[k][f] = interp_global<GEN>(src, g, n, ii[k][0], ii[k][1], ii[k][2],
                                                     dd[k]);
            }
        }
        float* out = dir == 0 ? dp : dm;
#pragma unroll
        for (int k = 0; k < kVox; ++k) {
            if (!on[k]) continue;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                sti(out + a * n, gi[k], sg * 0.5f * c[a] * (vx[k][a] + u[k][a]));
        }
    }
}

// ------------------------------------------------------------------------
// General extents: n1, n2 any even products of 2, 3, 5 (n3 a power of two).
// The single-field gathers and the backtrace are the LDS-staged kernels
// instantiated for ragged bricks and a modulo wrap (GEN); multi-field
// interpolation reads its stencil directly from global memory.
__device__ __forceinline__ void coords_gen(const G3& g, unsigned idx, int& i1, int& i2,
                                           int& i3) {
    i3 = (int)(idx & (unsigned)g.m3);
    const unsigned r = idx >> g.l3;
    i2 = (int)(r % (unsigned)g.n2);
    i1 = (int)(r / (unsigned)g.n2);
}

template <int NF>
__global__ __launch_bounds__(kThreads) void k_interp_gen(const float* __restrict__ f,
                                                         const float* __restrict__ d,
                                                         float* __restrict__ out, G3 g,
                                                         long long n) {
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= n) return;
    int i1, i2, i3;
    coords_gen(g, (unsigned)idx, i1, i2, i3);
    Stencil st;
    make_stencil<true>(g, i1, i2, i3, d[idx], d[n + idx], d[2 * n + idx], st);
    float r[NF];
    gather<NF>(f, n, st, r);
#pragma unroll
    for (int k = 0; k < NF; ++k) out[k * n + idx] = r[k];
}

unsigned blocks_for(long long n);

// brick of the single-field gathers (and of their per-brick box tables)
Brick gather_brick(const Geo& g) { return make_brick(g); }

template <class Epi>
int launch_gather_lds(const Geo& g, const float* src, const float* disp, const int* table,
                      const Epi& epi, hipStream_t s) {
    const Brick br = gather_brick(g);
    if (!g.pow2)
        hipLaunchKernelGGL((k_gather_lds<Epi, true>), dim3(br.nbricks), dim3(kThreads), 0, s, src,
                           disp, table, epi, make_g3(g), br, g.n);
    else
        hipLaunchKernelGGL((k_gather_lds<Epi, false>), dim3(br.nbricks), dim3(kThreads), 0, s,
                           src, disp, table, epi, make_g3(g), br, g.n);
    CL_LAUNCH_CHECK();
    return 0;
}

// out[k](x) = f[k](x + d(x)), k < nf (nf <= 4 per launch chunk)
template <int NF>
__global__ __launch_bounds__(kThreads) void k_interp(const float* __restrict__ f,
                                                     const float* __restrict__ d,
                                                     float* __restrict__ out, G3 g, long long n) {
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= n) return;
    int i1, i2, i3;
    coords(g, idx, i1, i2, i3);
    Stencil st;
    make_stencil(g, i1, i2, i3, d[idx], d[n + idx], d[2 * n + idx], st);
    float r[NF];
    gather<NF>(f, n, st, r);
#pragma unroll
    for (int k = 0; k < NF; ++k) out[k * n + idx] = r[k];
}

__global__ __launch_bounds__(kThreads) void k_final_adjoint(const float* __restrict__ mT,
                                                            const float* __restrict__ m1,
                                                            float* __restrict__ lam, long long n) {
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (idx < n) lam[idx] = m1[idx] - mT[idx];
}

// w^0 = (h_t/2) f^0 with f^0 = -grad m^0 . v~ (grad m stored as GT)
template <typename GT>
__global__ __launch_bounds__(kThreads) void k_inc_first(const GT* __restrict__ gm,
                                                        const float* __restrict__ vt,
                                                        float* __restrict__ w, long long n,
                                                        float half_ht) {
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= n) return;
    const float f = ldf(gm + idx) * vt[idx] + ldf(gm + n + idx) * vt[n + idx] +
                    ldf(gm + 2 * n + idx) * vt[2 * n + idx];
    w[idx] = -half_ht * f;
}

// out_a = add_a + h_t sum_j c_j lam^j d_a m^j  (trapezoid c_0 = c_nt = 1/2).
// ALS: instead of `add`, the PCG recursion als (alpha L s) is advanced in
// place to (r_a - mean_a) + mu als_a and added.
template <bool DOT, bool ALS, typename GT>
__global__ __launch_bounds__(kThreads) void k_assemble(const float* __restrict__ lam,
                                                       const GT* __restrict__ gm, int nt,
                                                       const float* __restrict__ add,
                                                       float* __restrict__ out, long long n,
                                                       float ht, const float* __restrict__ dv,
                                                       double* __restrict__ partial,
                                                       float* __restrict__ als,
                                                       const float* __restrict__ r, PcgDev pd) {
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    double dot = 0.0;
    float am[3] = {0.f, 0.f, 0.f}, mu = 0.f;
    bool adv = false;
    if (ALS) adv = pcg_als_scalars(pd, am[0], am[1], am[2], mu);
    if (idx < n) {
        float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
        for (int j = 0; j <= nt; ++j) {
            const float c = (j == 0 || j == nt) ? 0.5f * ht : ht;
            const float l = c * lam[(long long)j * n + idx];
            const GT* gj = gm + (long long)j * 3 * n;
            acc0 = fmaf(l, ldf(gj + idx), acc0);
            acc1 = fmaf(l, ldf(gj + n + idx), acc1);
            acc2 = fmaf(l, ldf(gj + 2 * n + idx), acc2);
        }
        if (ALS) {
            float a[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                a[c] = als[c * n + idx];
                if (adv) {
                    a[c] = fmaf(mu, a[c], r[c * n + idx] - am[c]);
                    als[c * n + idx] = a[c];
                }
            }
            acc0 += a[0];
            acc1 += a[1];
            acc2 += a[2];
        } else if (add) {
            acc0 += add[idx];
            acc1 += add[n + idx];
            acc2 += add[2 * n + idx];
        }
        out[idx] = acc0;
        out[n + idx] = acc1;
        out[2 * n + idx] = acc2;
        if (DOT)
            dot = (double)dv[idx] * acc0 + (double)dv[n + idx] * acc1 +
                  (double)dv[2 * n + idx] * acc2;
    }
    if (DOT) {
        __shared__ double sh[4];
        const double t = block_sum_256(dot, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = t;
    }
}

// Deformation gradient, eq. (e:def-grad): D F/Dt = (grad v) F along +v, one
// RK2 step along the characteristics given the gathered values
// F_y = F^j(y+) and G_y = G(y+) (G_ab = d_b v_a, fields row-major [9][n]):
//   f0 = G_y F_y, F~ = F_y + h_t f0, f1 = G(x) F~, F^{j+1} = F_y + (h_t/2)(f0 + f1).
// Fy == NULL means F^0 = I (nothing to gather). F may alias Fy.
__global__ __launch_bounds__(kThreads) void k_defgrad_update(const float* __restrict__ Fy,
                                                             const float* __restrict__ Gy,
                                                             const float* __restrict__ G,
                                                             float* F, long long n, float ht) {
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= n) return;
    float gy[9], fy[9], gx[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        gy[q] = Gy[q * n + idx];
        gx[q] = G[q * n + idx];
        fy[q] = Fy ? Fy[q * n + idx] : ((q % 4 == 0) ? 1.f : 0.f);
    }
    float f0[9], ft[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float acc = 0.f;
#pragma unroll
            for (int b = 0; b < 3; ++b) acc = fmaf(gy[3 * a + b], fy[3 * b + c], acc);
            f0[3 * a + c] = acc;
            ft[3 * a + c] = fy[3 * a + c] + ht * acc;
        }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float acc = 0.f;
#pragma unroll
            for (int b = 0; b < 3; ++b) acc = fmaf(gx[3 * a + b], ft[3 * b + c], acc);
            F[(3 * a + c) * n + idx] = fy[3 * a + c] + 0.5f * ht * (f0[3 * a + c] + acc);
        }
}

// det of the 3x3 field in float64
__global__ __launch_bounds__(kThreads) void k_det(const float* __restrict__ F,
                                                  double* __restrict__ det, long long n) {
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= n) return;
    double a[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) a[q] = (double)F[q * n + idx];
    det[idx] = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
               a[2] * (a[3] * a[7] - a[4] * a[6]);
}

// ----------------------------------------------------------- mixed precision
// 8-byte stores of four halves (round to nearest, as __float2half)
__device__ __forceinline__ uint2 pack_h4(const float o[4]) {
    const __half2 lo = __floats2half2_rn(o[0], o[1]);
    const __half2 hi = __floats2half2_rn(o[2], o[3]);
    uint2 u;
    u.x = *reinterpret_cast<const unsigned*>(&lo);
    u.y = *reinterpret_cast<const unsigned*>(&hi);
    return u;
}

__global__ __launch_bounds__(kThreads) void k_to_half4(const float4* __restrict__ x,
                                                       uint2* __restrict__ y, long long n4) {
    const long long q = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (q >= n4) return;
    const float4 v = x[q];
    const float o[4] = {v.x, v.y, v.z, v.w};
    y[q] = pack_h4(o);
}

__global__ __launch_bounds__(kThreads) void k_to_half(const float* __restrict__ x,
                                                      __half* __restrict__ y, long long n) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) y[i] = __float2half(x[i]);
}

unsigned blocks_for(long long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

int launch_backtrace(const Geo& g, const float* v, float* dplus, float* dminus, double ht,
                     hipStream_t s) {
    const float c1 = (float)(ht * g.n1 / (2.0 * M_PI));
    const float c2 = (float)(ht * g.n2 / (2.0 * M_PI));
    const float c3 = (float)(ht * g.n3 / (2.0 * M_PI));
    const Brick br = make_brick(g);
    if (!g.pow2)
        hipLaunchKernelGGL(k_backtrace_lds<true>, dim3(br.nbricks), dim3(kThreads), 0, s, v,
                           dplus, dminus, make_g3(g), br, g.n, c1, c2, c3);
    else
        hipLaunchKernelGGL(k_backtrace_lds<false>, dim3(br.nbricks), dim3(kThreads), 0, s, v,
                           dplus, dminus, make_g3(g), br, g.n, c1, c2, c3);
    CL_LAUNCH_CHECK();
    return 0;
}

int launch_interp(const Geo& g, const float* f, int nfield, const float* disp, float* out,
                  hipStream_t s, const int* boxes) {
    if (nfield == 1) return launch_gather_lds(g, f, disp, boxes, EpiStore{out}, s);
    const G3 g3 = make_g3(g);
    int k = 0;
    while (k < nfield) {
        const int chunk = (nfield - k >= 3) ? 3 : (nfield - k);
        const float* fk = f + (long long)k * g.n;
        float* ok = out + (long long)k * g.n;
        if (!g.pow2) {
            if (chunk == 3)
                hipLaunchKernelGGL(k_interp_gen<3>, dim3(blocks_for(g.n)), dim3(kThreads), 0, s, fk, disp, ok, g3, g.n);
            else if (chunk == 2)
                hipLaunchKernelGGL(k_interp_gen<2>, dim3(blocks_for(g.n)), dim3(kThreads), 0, s, fk, disp, ok, g3, g.n);
            else
                hipLaunchKernelGGL(k_interp_gen<1>, dim3(blocks_for(g.n)), dim3(kThreads), 0, s, fk, disp, ok, g3, g.n);
        } else if (chunk == 3)
            hipLaunchKernelGGL(k_interp<3>, dim3(blocks_for(g.n)), dim3(kThreads), 0, s, fk, disp, ok, g3, g.n);
        else if (chunk == 2)
            hipLaunchKernelGGL(k_interp<2>, dim3(blocks_for(g.n)), dim3(kThreads), 0, s, fk, disp, ok, g3, g.n);
        else
            hipLaunchKernelGGL(k_interp<1>, dim3(blocks_for(g.n)), dim3(kThreads), 0, s, fk, disp, ok, g3, g.n);
        CL_LAUNCH_CHECK();
        k += chunk;
    }
    return 0;
}

int launch_make_A(const Geo& g, const float* divv, const float* dminus, float* A, double ht,
                  hipStream_t s, const int* boxes) {
    return launch_gather_lds(g, divv, dminus, boxes, EpiMakeA{divv, A, (float)ht}, s);
}

int launch_final_adjoint(const Geo& g, const float* mT, const float* m1, float* lamT,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_final_adjoint, dim3(blocks_for(g.n)), dim3(kThreads), 0, s, mT, m1, lamT,
                       g.n);
    CL_LAUNCH_CHECK();
    return 0;
}

int launch_adjoint_step(const Geo& g, const float* lam_next, const float* dminus, const float* A,
                        float* lam, hipStream_t s, const int* boxes) {
    return launch_gather_lds(g, lam_next, dminus, boxes, EpiScale{A, lam}, s);
}

template <typename GT>
int launch_inc_state_first(const Geo& g, const GT* gradm0, const float* vt, float* w0,
                           double ht, hipStream_t s) {
    hipLaunchKernelGGL(k_inc_first<GT>, dim3(blocks_for(g.n)), dim3(kThreads), 0, s, gradm0, vt,
                       w0, g.n, (float)(0.5 * ht));
    CL_LAUNCH_CHECK();
    return 0;
}
template int launch_inc_state_first<float>(const Geo&, const float*, const float*, float*,
                                           double, hipStream_t);
template int launch_inc_state_first<__half>(const Geo&, const __half*, const float*, float*,
                                            double, hipStream_t);

template <typename GT>
int launch_inc_state_step(const Geo& g, const float* w_prev, const float* dplus,
                          const GT* gradm_next, const float* vt, float* out, float coef,
                          float sign, hipStream_t s, const int* boxes) {
    return launch_gather_lds(g, w_prev, dplus, boxes,
                             EpiIncState<GT>{gradm_next, vt, out, g.n, coef, sign}, s);
}
template int launch_inc_state_step<float>(const Geo&, const float*, const float*, const float*,
                                          const float*, float*, float, float, hipStream_t,
                                          const int*);
template int launch_inc_state_step<__half>(const Geo&, const float*, const float*,
                                           const __half*, const float*, float*, float, float,
                                           hipStream_t, const int*);

template <typename GT>
int launch_assemble(const Geo& g, const float* lam, const GT* gradm, int nt, const float* add,
                    float* out, hipStream_t s, const float* dot_with, Reducer* red, int slot,
                    const PcgDev* als_pd, const float* r, float* als) {
    const unsigned nb = blocks_for(g.n);
    const float ht = (float)(1.0 / nt);
    if (als_pd && (add || !als || !r || !dot_with)) {
        set_error("the als update in the assembly takes als and r in place of the addend, "
                  "and the dot product");
        return CLAIRE_EINVAL;
    }
    if (als_pd) {
        hipLaunchKernelGGL((k_assemble<true, true, GT>), dim3(nb), dim3(kThreads), 0, s, lam,
                           gradm, nt, nullptr, out, g.n, ht, dot_with, red->partial, als, r,
                           *als_pd);
        CL_LAUNCH_CHECK();
        return red_fold_sum(*red, (int)nb, 1, 0, slot, s);
    }
    if (dot_with) {
        hipLaunchKernelGGL((k_assemble<true, false, GT>), dim3(nb), dim3(kThreads), 0, s, lam,
                           gradm, nt, add, out, g.n, ht, dot_with, red->partial, nullptr,
                           nullptr, PcgDev());
        CL_LAUNCH_CHECK();
        return red_fold_sum(*red, (int)nb, 1, 0, slot, s);
    }
    hipLaunchKernelGGL((k_assemble<false, false, GT>), dim3(nb), dim3(kThreads), 0, s, lam, gradm,
                       nt, add, out, g.n, ht, nullptr, nullptr, nullptr, nullptr, PcgDev());
    CL_LAUNCH_CHECK();
    return 0;
}
template int launch_assemble<float>(const Geo&, const float*, const float*, int, const float*,
                                    float*, hipStream_t, const float*, Reducer*, int,
                                    const PcgDev*, const float*, float*);
template int launch_assemble<__half>(const Geo&, const float*, const __half*, int, const float*,
                                     float*, hipStream_t, const float*, Reducer*, int,
                                     const PcgDev*, const float*, float*);

int brick_table_ints(const Geo& g) { return 6 * gather_brick(g).nbricks; }

int launch_to_half(const float* x, __half* y, long long n, hipStream_t s) {
    if ((n & 3) == 0 && ((reinterpret_cast<uintptr_t>(x) & 15) | (reinterpret_cast<uintptr_t>(y) & 7)) == 0)
        hipLaunchKernelGGL(k_to_half4, dim3(blocks_for(n / 4)), dim3(kThreads), 0, s,
                           reinterpret_cast<const float4*>(x), reinterpret_cast<uint2*>(y), n / 4);
    else
        hipLaunchKernelGGL(k_to_half, dim3(blocks_for(n)), dim3(kThreads), 0, s, x, y, n);
    CL_LAUNCH_CHECK();
    return 0;
}

int launch_brick_boxes(const Geo& g, const float* disp, int* table, hipStream_t s) {
    const Brick br = gather_brick(g);
    if (!g.pow2)
        hipLaunchKernelGGL(k_brick_boxes<true>, dim3(br.nbricks), dim3(kThreads), 0, s, disp,
                           table, make_g3(g), br, g.n);
    else
        hipLaunchKernelGGL(k_brick_boxes<false>, dim3(br.nbricks), dim3(kThreads), 0, s, disp,
                           table, make_g3(g), br, g.n);
    CL_LAUNCH_CHECK();
    return 0;
}

int launch_defgrad_update(const Geo& g, const float* Fy, const float* Gy, const float* G,
                          float* F, double ht, hipStream_t s) {
    hipLaunchKernelGGL(k_defgrad_update, dim3(blocks_for(g.n)), dim3(kThreads), 0, s, Fy, Gy, G,
                       F, g.n, (float)ht);
    CL_LAUNCH_CHECK();
    return 0;
}

int launch_det(const Geo& g, const float* F, double* det, hipStream_t s) {
    hipLaunchKernelGGL(k_det, dim3(blocks_for(g.n)), dim3(kThreads), 0, s, F, det, g.n);
    CL_LAUNCH_CHECK();
    return 0;
}

}  // namespace claire
