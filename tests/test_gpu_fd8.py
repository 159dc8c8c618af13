"""FD8 first derivatives (Section 2.5.3, the paper's GPU stencil) on the GPU
against the FP64 oracle: the operators themselves (several shapes, including
8 voxels per axis where the +-4 neighbours coincide), the setup (gradient,
objective, adjoint) and a Hessian matvec with FD8 grad m^j and div v, det F
with FD8 grad v, and one Gauss--Newton step with 10 PCG matvecs.

Bar: 1e-5 max-norm relative (float32 arithmetic; the stencil takes
differences of neighbours first, so cancellation costs ~1e-7 / (k h) of the
derivative), 1e-4 for v and J after a Gauss--Newton step, as in the spectral
tests.
"""
import numpy as np
import pytest

import oracle as O
from helpers import blob_problem, f32, rel_err
from synthetic import bandlimited_velocity, noise

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


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


@pytest.mark.parametrize("n", [(8, 8, 8), (16, 32, 64), (64, 16, 8), (64, 64, 64)])
def test_fd8_operators(C, n):
    grid = O.Grid(n)
    kmax = max(1, min(n) // 4)
    u = f32(bandlimited_velocity(n, 11, kmax, 1.0)[0] + noise(n, 12, 0.01))
    v = f32(bandlimited_velocity(n, 13, kmax, 1.0))
    with C.Context(n, 1, 1e-2, 1) as ctx:
        g = host(ctx.spectral(C.OP_FD8_GRAD, dev(u)))
        d = host(ctx.spectral(C.OP_FD8_DIV, dev(v)))
    eg, ed = rel_err(g, O.fd8_gradient(grid, u)), rel_err(d, O.fd8_divergence(grid, v))
    print("FD8 %s: grad %.2e, div %.2e" % (n, eg, ed))
    assert eg <= TOL and ed <= TOL


@pytest.mark.parametrize("p", [1, 2])
def test_setup_and_matvec_fd8(C, p):
    nt, alpha = 4, 1e-2
    grid, m0, m1, vstar = blob_problem()
    v = f32(0.5 * vstar)
    vt = f32(bandlimited_velocity(grid.n, 77, 4, 0.5))
    st = O.setup_velocity(grid, m0, m1, v, alpha, nt, p, deriv="fd8")
    ref = O.hessian_matvec(st, vt)
    with C.Context(grid.n, nt, alpha, p) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        ctx.set_derivative(C.DERIV_FD8)
        ctx.set_velocity(dev(v))
        gm = host(ctx.get_field(C.FIELD_GRAD_STATE, nt))
        dv = host(ctx.get_field(C.FIELD_DIVV))
        g, J = ctx.gradient()
        hv = host(ctx.hessian_matvec(dev(vt)))
        errs = dict(grad_m=rel_err(gm, st.grad_m[nt]), div_v=rel_err(dv, st.div_v),
                    g=rel_err(host(g), st.g), J=abs(J - st.J) / st.J, Hv=rel_err(hv, ref))
    print("FD8 setup p%d:" % p, {k: "%.2e" % e for k, e in errs.items()})
    assert max(errs.values()) <= TOL
    # spectral and FD8 agree to the FD8 truncation error on this smooth problem
    st_s = O.setup_velocity(grid, m0, m1, v, alpha, nt, p)
    assert rel_err(st.g, st_s.g) < 5e-2


def test_detdefgrad_fd8(C):
    nt = 4
    grid, m0, m1, vstar = blob_problem()
    v = f32(1.5 * vstar)
    ref = O.deformation_determinant(grid, v, nt, deriv="fd8")
    with C.Context(grid.n, nt, 1e-2, 1) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        ctx.set_derivative(C.DERIV_FD8)
        ctx.set_velocity(dev(v))
        det, s = ctx.detdefgrad(want_field=True)
        d = host(det)
    print("FD8 det F: %.2e" % rel_err(d, ref))
    assert rel_err(d, ref) < TOL
    assert s["nonpositive"] == int((ref <= 0).sum())


def test_one_gn_step_fd8(C):
    nt, alpha = 4, 1e-2
    grid, m0, m1, vstar = blob_problem()
    v_ref, _, stats_ref = O.gn_solve(grid, m0, m1, nt, 1, [alpha], max_gn=1, fixed_pcg=10,
                                     deriv="fd8")
    with C.Context(grid.n, nt, alpha, 1) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        v, stats = ctx.solve(max_gn=1, fixed_pcg_iters=10, derivative=C.DERIV_FD8)
        vh = host(v)
    print("FD8 GN step: v %.2e, J %.2e" % (rel_err(vh, v_ref),
                                           abs(stats["J"] - stats_ref.J) / stats_ref.J))
    assert stats["matvecs"] == 10 and stats["linesearch_trials"] == stats_ref.ls_trials
    assert rel_err(vh, v_ref) < 1e-4
    assert abs(stats["J"] - stats_ref.J) <= 1e-4 * stats_ref.J
