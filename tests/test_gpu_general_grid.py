"""Grids whose extents are not all powers of two: n1 and n2 even products of
2, 3 and 5, n3 a power of two (the paper's NIREP images are 256 x 300 x 256).
These run the LDS-staged gathers on ragged bricks with a modulo wrap and
mixed-radix (4, 2, 3, 5) column transforms. Against the FP64 oracle at small
shapes that use every radix, ragged bricks and ragged column tiles; at the
NIREP shape through properties that hold at any size.

Bars as for the power-of-two grids: 1e-5 max-norm relative (float32), 1e-3
for the mixed-precision matvec, 1e-4 for v and J after Gauss--Newton steps.
"""
import numpy as np
import pytest

import oracle as O
from helpers import Parity, blob_problem, f32, rel_err
from synthetic import WORKLOADS, bandlimited_velocity, ellipsoid_phantom, noise

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
# radices: 24 = 4.2.3, 20 = 4.5, 30 = 2.3.5, 12 = 4.3, 18 = 2.3.3, 50 = 2.5.5;
# the last two shapes have one power-of-two column axis (16), which takes the
# power-of-two column kernels (as x1 = 256 of the NIREP grid does)
SHAPES = [(24, 20, 16), (30, 12, 32), (18, 50, 8), (16, 30, 16), (20, 16, 32)]


@pytest.fixture(scope="module")
def C():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_17493_amd import claire
    return claire


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("n", SHAPES)
def test_operators_general(C, n):
    grid = O.Grid(n)
    kmax = min(3, min(n) // 2 - 1)
    u = f32(ellipsoid_phantom(n, 3) + noise(n, 8, 0.01))
    v = f32(bandlimited_velocity(n, 4, kmax, 1.0) + noise((3,) + n, 9, 0.01))
    P = Parity("general%s" % (n,))
    for p in (1, 2):
        with C.Context(n, 4, 3e-2, p) as ctx:
            P.rel("grad p%d" % p, host(ctx.spectral(C.OP_GRAD, dev(u))),
                  O.spectral_gradient(grid, u), TOL)
            P.rel("div p%d" % p, host(ctx.spectral(C.OP_DIV, dev(v))),
                  O.spectral_divergence(grid, v), TOL)
            P.rel("reg p%d" % p, host(ctx.spectral(C.OP_REG, dev(v))),
                  O.regularization_operator(grid, v, 3e-2, p), TOL)
            P.rel("reg_inv p%d" % p, host(ctx.spectral(C.OP_REG_INV, dev(v))),
                  O.precondition(grid, v, 3e-2, p), TOL)
            P.rel("fd8 grad p%d" % p, host(ctx.spectral(C.OP_FD8_GRAD, dev(u))),
                  O.fd8_gradient(grid, u), TOL)
            P.rel("fd8 div p%d" % p, host(ctx.spectral(C.OP_FD8_DIV, dev(v))),
                  O.fd8_divergence(grid, v), TOL)
            if p == 1:
                ctx.set_beta(1e-2)
                P.rel("ni project", host(ctx.spectral(C.OP_NI_PROJECT, dev(v))),
                      O.ni_project(grid, v, 3e-2, 1e-2), TOL)
                P.rel("ni penalty", host(ctx.spectral(C.OP_NI_PENALTY, dev(v))),
                      O.divergence_penalty_gradient(grid, v, 1e-2), TOL)
    P.done()


@pytest.mark.parametrize("n", SHAPES[:2])
def test_interpolation_general(C, n):
    rng = np.random.default_rng(5)
    f = f32(rng.standard_normal((2,) + n))
    d = f32(np.stack([rng.uniform(-12, 12, n) for _ in range(3)]))
    with C.Context(n, 4, 1.0, 1) as ctx:
        got = host(ctx.interpolate(dev(f), dev(d)))
        assert rel_err(got, O.interpolate(f, d)) < TOL
        one = host(ctx.interpolate(dev(f[1]), dev(d)))
        assert rel_err(one, O.interpolate(f[1:], d)[0]) < TOL
        # whole-voxel displacements (beyond one period) are exact rolls
        s = (3 - n[0], -5, 2 * n[2] + 1)
        ds = np.stack([np.full(n, float(k)) for k in s])
        r = host(ctx.interpolate(dev(f[0]), dev(ds)))
        assert np.array_equal(r, np.roll(f[0], tuple(-k for k in s), axis=(0, 1, 2)))


@pytest.mark.parametrize("p,beta", [(1, 0.0), (2, 0.0), (1, 1e-2)])
def test_setup_and_matvec_general(C, p, beta):
    nt, alpha = 4, 1e-2
    grid, m0, m1, vstar = blob_problem(n=(24, 20, 32), kmax=4)
    v = f32(0.5 * vstar)
    vt = f32(bandlimited_velocity(grid.n, 77, 4, 0.5))
    st = O.setup_velocity(grid, m0, m1, v, alpha, nt, p, beta=beta)
    ref = O.hessian_matvec(st, vt)
    P = Parity("general setup p%d beta %g" % (p, beta))
    for precision in (0, 1):
        with C.Context(grid.n, nt, alpha, p) as ctx:
            ctx.set_images(dev(m0), dev(m1))
            ctx.set_beta(beta)
            ctx.set_precision(precision)
            ctx.set_velocity(dev(v))
            g, J = ctx.gradient()
            if precision == 0:
                P.rel("disp+", host(ctx.get_field(C.FIELD_DISP_PLUS)), st.d_plus, TOL)
                P.rel("m^nt", host(ctx.get_field(C.FIELD_STATE, nt)), st.m[nt], TOL)
                P.rel("lambda^0", host(ctx.get_field(C.FIELD_ADJOINT, 0)), st.lam[0], TOL)
                P.rel("g", host(g), st.g, TOL)
                P.value("J", J, st.J, TOL)
            P.rel("Hv prec%d" % precision, host(ctx.hessian_matvec(dev(vt))), ref,
                  TOL if precision == 0 else 1e-3)
    P.done()


def test_detdefgrad_general(C):
    nt = 4
    grid, m0, m1, vstar = blob_problem(n=(30, 12, 32), kmax=4)
    v = f32(1.5 * vstar)
    ref = O.deformation_determinant(grid, v, nt)
    with C.Context(grid.n, nt, 1e-2, 1) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        ctx.set_velocity(dev(v))
        det, s = ctx.detdefgrad(want_field=True)
        d = host(det)
    assert rel_err(d, ref) < TOL
    assert s["nonpositive"] == int((ref <= 0).sum())


@pytest.mark.parametrize("n", [(24, 20, 32), (32, 20, 32)])
def test_full_solve_general(C, n):
    nt, alpha = 4, 1e-2
    grid, m0, m1, vstar = blob_problem(n=n, kmax=4)
    v_ref, _, s_ref = O.gn_solve(grid, m0, m1, nt, 1, [alpha])
    with C.Context(grid.n, nt, alpha, 1) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        v, st = ctx.solve()
        vh = host(v)
    print("general-grid solve: GN %d/%d, matvecs %d/%d, v %.2e, J %.2e" % (
        st["gn_iters"], s_ref.gn_iters, st["matvecs"], s_ref.matvecs, rel_err(vh, v_ref),
        abs(st["J"] - s_ref.J) / s_ref.J))
    assert st["status"] == 0
    assert st["gn_iters"] == s_ref.gn_iters and st["matvecs"] == s_ref.matvecs
    assert rel_err(vh, v_ref) < 1e-4
    assert abs(st["J"] - s_ref.J) <= 1e-4 * s_ref.J


def test_twolevel_general(C):
    """Coarse grid 12 x 10 x 16 (radices 4.3 and 2.5)."""
    n, alpha = (24, 20, 32), 1e-2
    grid, m0, m1, vstar = blob_problem(n=n, kmax=4)
    v = f32(0.5 * vstar)
    st = O.setup_velocity(grid, m0, m1, v, alpha, 4, 1)
    r = f32(bandlimited_velocity(n, 5, 5, 1.0) + noise((3,) + n, 6, 0.1))
    ref = O.TwoLevelPreconditioner(st, inner_rtol=0.0, max_inner=6)(r)
    with C.Context(n, 4, alpha, 1) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        ctx.set_velocity(dev(v))
        z, its = ctx.precond_twolevel(dev(r), 0.0, 6)
        z = host(z)
    assert its == 6
    assert rel_err(z, ref) < TOL


def test_rejected_extents(C):
    for n in [(14, 16, 16), (16, 22, 16), (16, 16, 24), (16, 15, 16)]:
        with pytest.raises(C.ClaireError) as e:
            C.Context(n, 2, 1e-2, 1)
        assert e.value.code == -1
    # the two-level coarse grid must itself be supported: 30 / 2 = 15 is odd
    grid, m0, m1, _ = blob_problem(n=(16, 30, 16), kmax=3)
    with C.Context(grid.n, 2, 1e-2, 1) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        ctx.set_velocity(dev(np.zeros((3,) + grid.n)))
        with pytest.raises(C.ClaireError) as e:
            ctx.precond_twolevel(dev(np.zeros((3,) + grid.n)), 0.1)
        assert e.value.code == -1


# ---------------------------------------------------------------- NIREP shape
W = WORKLOADS["ellipsoids_nirep"]
N = W["n"]


@pytest.fixture(scope="module")
def nirep(C):
    seed = W["seed"]
    clean = dev(ellipsoid_phantom(N, seed))
    vstar = dev(bandlimited_velocity(N, seed + 1000, W["kmax"], W["vmax"]))
    m0 = clean + dev(noise(N, seed + 2000, W["noise"]))
    m1 = C.transport(clean, vstar, W["nt"]) + dev(noise(N, seed + 3000, W["noise"]))
    torch.cuda.synchronize()
    return m0.contiguous(), m1.contiguous(), vstar


def test_nirep_spectral_gradient(C):
    x = [torch.arange(k, device="cuda", dtype=torch.float64) * (2 * np.pi / k) for k in N]
    c1, c2, c3 = torch.meshgrid(*x, indexing="ij")
    f = torch.sin(3 * c1) * torch.cos(5 * c2) + torch.sin(17 * c3 - c1) + torch.cos(149 * c2)
    g = [3 * torch.cos(3 * c1) * torch.cos(5 * c2) - torch.cos(17 * c3 - c1),
         -5 * torch.sin(3 * c1) * torch.sin(5 * c2) - 149 * torch.sin(149 * c2),
         17 * torch.cos(17 * c3 - c1)]
    with C.Context(N, 1, 1e-3, 1) as ctx:
        out = ctx.spectral(C.OP_GRAD, f.float().contiguous())
        err = max(float((out[a].double() - g[a]).abs().max()) for a in range(3)) / 149.0
    print("NIREP spectral gradient: rel err %.2e" % err)
    assert err <= 1e-5


def test_nirep_transport_shift_and_constant(C, nirep):
    m0, _, vstar = nirep
    nt = W["nt"]
    h = [2 * np.pi / k for k in N]
    shift = (2, -3, 1)
    v = torch.empty((3,) + N, device="cuda")
    for a in range(3):
        v[a] = shift[a] * h[a] * nt
    out = C.transport(m0, v.contiguous(), nt)
    ref = torch.roll(m0, shifts=tuple(s * nt for s in shift), dims=(0, 1, 2))
    err = float((out - ref).abs().max() / ref.abs().max())
    const = C.transport(torch.full(N, 0.7, device="cuda"), vstar, nt)
    cerr = float((const - 0.7).abs().max())
    print("NIREP whole-voxel transport %.2e, constant %.2e" % (err, cerr))
    assert err <= 1e-5 and cerr <= 1e-5


def test_nirep_matvec_linear_and_solve(C, nirep):
    m0, m1, vstar = nirep
    with C.Context(N, W["nt"], W["alphas"][-1], W["reg_order"]) as ctx:
        ctx.set_images(m0, m1)
        ctx.set_velocity((0.5 * vstar).contiguous())
        vt = (0.3 * vstar).contiguous()
        h1 = ctx.hessian_matvec(vt)
        h2 = ctx.hessian_matvec((2 * vt).contiguous())
        torch.cuda.synchronize()
        assert torch.equal(h2, 2 * h1)
        assert float((vt.double() * h1.double()).sum()) > 0
        v, st = ctx.solve(gtol=W["gtol"], precision=1, max_gn=3)
        print("NIREP mixed solve, 3 GN steps: %d matvecs, %.2f s, J %.4f -> %.4f, rel_grad %.3f"
              % (st["matvecs"], st["seconds"], st["J0"], st["J"], st["rel_grad"]))
        assert np.isfinite(st["J"]) and st["J"] < st["J0"]


def test_full_solve_general_ni(C):
    """Near-incompressible solve on a general grid."""
    nt, alpha, beta = 4, 1e-2, 1e-2
    grid, m0, m1, vstar = blob_problem(n=(24, 20, 32), kmax=4)
    v_ref, _, s_ref = O.gn_solve(grid, m0, m1, nt, 1, [alpha], beta=beta)
    with C.Context(grid.n, nt, alpha, 1) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        v, st = ctx.solve(beta=beta)
        vh = host(v)
    print("general-grid NI solve: GN %d/%d, matvecs %d/%d, v %.2e" % (
        st["gn_iters"], s_ref.gn_iters, st["matvecs"], s_ref.matvecs, rel_err(vh, v_ref)))
    assert st["status"] == 0
    assert st["gn_iters"] == s_ref.gn_iters and st["matvecs"] == s_ref.matvecs
    assert rel_err(vh, v_ref) < 1e-4
    assert abs(st["J"] - s_ref.J) <= 1e-4 * s_ref.J
