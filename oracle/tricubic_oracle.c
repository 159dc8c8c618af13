/*
 * FP64 tricubic Lagrange interpolation on a periodic grid -- TEST ORACLE.
 *
 * Test infrastructure only: the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it to check the HIP path. The product never links it.
 *
 * Method: Section 2.5.4 (interpolation) with polynomial order p = 3, i.e. a
 * tensor product of 1D cubic Lagrange polynomials through the four nodes
 * floor(q)-1 .. floor(q)+2 along each axis, nodes wrapped periodically.
 * Query points are given as a grid index plus a displacement in voxel units,
 * so that a zero displacement reproduces grid values exactly.
 *
 * Plain loops, no blocking: written to be checked by eye.
 */
#include <math.h>
#include <stddef.h>

/* Cubic Lagrange basis on nodes -1, 0, 1, 2 evaluated at s in [0, 1). */
static void lagrange_cubic(double s, double w[4])
{
    w[0] = -s * (s - 1.0) * (s - 2.0) / 6.0;
    w[1] = (s + 1.0) * (s - 1.0) * (s - 2.0) / 2.0;
    w[2] = -(s + 1.0) * s * (s - 2.0) / 2.0;
    w[3] = (s + 1.0) * s * (s - 1.0) / 6.0;
}

static long wrap(long i, long n)
{
    long r = i % n;
    return r < 0 ? r + n : r;
}

/* Value at the point whose coordinate along axis a is (base_a + disp_a) grid
 * units, base_a integer. */
static double interp_one(const double *f, long n1, long n2, long n3,
                         long b1, long b2, long b3,
                         double d1, double d2, double d3)
{
    double fl1 = floor(d1), fl2 = floor(d2), fl3 = floor(d3);
    long i1 = b1 + (long)fl1, i2 = b2 + (long)fl2, i3 = b3 + (long)fl3;
    double w1[4], w2[4], w3[4];
    lagrange_cubic(d1 - fl1, w1);
    lagrange_cubic(d2 - fl2, w2);
    lagrange_cubic(d3 - fl3, w3);
    double sum = 0.0;
    for (int a = 0; a < 4; ++a) {
        long j1 = wrap(i1 + a - 1, n1);
        for (int b = 0; b < 4; ++b) {
            long j2 = wrap(i2 + b - 1, n2);
            for (int c = 0; c < 4; ++c) {
                long j3 = wrap(i3 + c - 1, n3);
                sum += w1[a] * w2[b] * w3[c] * f[(j1 * n2 + j2) * n3 + j3];
            }
        }
    }
    return sum;
}

/* out[x] = f(x + d(x)) for every grid point x; d is [3][n1][n2][n3] in voxels.
 * nfield fields stored back to back (stride n1*n2*n3) share the same points. */
void oracle_tricubic_grid(const double *f, int nfield, int n1, int n2, int n3,
                          const double *d, double *out)
{
    long n = (long)n1 * n2 * n3;
    const double *d1 = d, *d2 = d + n, *d3 = d + 2 * n;
#pragma omp parallel for collapse(2) schedule(static)
    for (long i1 = 0; i1 < n1; ++i1)
        for (long i2 = 0; i2 < n2; ++i2)
            for (long i3 = 0; i3 < n3; ++i3) {
                long idx = (i1 * n2 + i2) * n3 + i3;
                for (int k = 0; k < nfield; ++k)
                    out[k * n + idx] = interp_one(f + k * n, n1, n2, n3, i1, i2, i3,
                                                  d1[idx], d2[idx], d3[idx]);
            }
}

/* out[p] = f(q_p) for arbitrary points q given in grid units, [npts][3]. */
void oracle_tricubic_points(const double *f, int n1, int n2, int n3,
                            const double *q, long npts, double *out)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < npts; ++p)
        out[p] = interp_one(f, n1, n2, n3, 0, 0, 0, q[3 * p], q[3 * p + 1], q[3 * p + 2]);
}
