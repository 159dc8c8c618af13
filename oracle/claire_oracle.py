"""FP64 CPU oracle of CLAIRE's Gauss--Newton--Krylov registration hot path.

TEST INFRASTRUCTURE ONLY. This module exists to check the HIP implementation:
only the tests, the smoke check and the benchmark's CPU-baseline leg may import
it. It shares no code with the HIP path; the only common inputs come from the
seeded generators in ``synthetic``.

Everything is float64 on the host: NumPy, ``scipy.fft`` for the Fourier
transforms, and a plain-C tricubic interpolation (``tricubic_oracle.c``).
No blocking, fusion or reordering beyond what the paper's formulas state, so
that each step can be read against the paper:

* problem statement, eq. (e:varopt-claire), Section 2.2;
* reduced gradient, eq. (e:rgrad), and adjoint, eq. (e:adjoint), Section 2.3;
* Hessian matvec, eq. (e:matvec), incremental state/adjoint, eqs. (e:incstate),
  (e:incadj), Section 2.4, with the Gauss--Newton simplification of
  Section 2.5.5 (all terms carrying the adjoint variable dropped);
* discretisation (nodal periodic grid, h_t = 1/n_t, trapezoidal time
  quadrature), Section 2.5.1;
* semi-Lagrangian time stepping (RK2 characteristics and RK2 along them),
  Section 2.5.2;
* pseudo-spectral differentiation, Section 2.5.3;
* cubic Lagrange interpolation, Section 2.5.4;
* inexact Gauss--Newton--Krylov with PCG, Armijo line search, forcing and
  stopping rules, Section 2.5.5 and Algorithms 1--2 (appendix);
* regularisation preconditioner, Section 2.5.6;
* parameter continuation, Section 2.6;
* deformation gradient transport, eq. (e:def-grad) (appendix);
* near-incompressible model (appendix, "(Near-)Incompressible
  Diffeomorphisms"): reduced gradient with the data term projected by
  I - grad M Delta^{-1} div, M = (alpha (beta (-Delta^{-1} + id))^{-1} + id)^{-1}.

Readings where the paper is silent or inconsistent (all listed in the design
notes of the repository):

* grid x_i = i*2*pi/n on [0, 2*pi)^3, x3 contiguous;
* adjoint and incremental adjoint: continuity equation with a minus sign on
  the divergence, i.e. d_t(lambda) + div(lambda v) = 0 backward in time;
* RK2 corrector u(t^{j+1}) = u(y) + h_t (f0 + f1)/2 (Heun's method);
* backward-in-time equations follow characteristics of -v;
* the incremental-state source f = -grad(m).v is formed on the grid and
  interpolated (derivatives are never taken on the deformed mesh);
* odd derivatives zero the Nyquist mode, even symbols keep it; the k = 0 mode
  of (alpha L)^{-1} is the identity;
* H^1 seminorm L = -Laplacian (symbol |k|^2), H^2 seminorm L = Laplacian^2
  (symbol |k|^4);
* PCG stops when ||r||_inf <= eta ||g||_inf, eta = min(1/2, sqrt(||g||_inf));
* Armijo: c1 = 1e-4, step halving from 1, at most 16 trials.

Parity pins live in tests/test_oracle_*.py (closed forms, invariants, brute
force). Functions with no such pin say "parity unpinned" in their docstring.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft

TWO_PI = 2.0 * np.pi
WORKERS = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_C_SRC = os.path.join(_HERE, "tricubic_oracle.c")
_C_LIB = os.path.join(_HERE, "libtricubic_oracle.so")
_lib = None


# ----------------------------------------------------------------------------
# plain-C interpolation kernel (built with gcc, loaded with ctypes)
# ----------------------------------------------------------------------------
def build_c(force: bool = False) -> str:
    """Compile the oracle's C interpolation into a shared library."""
    stale = (not os.path.exists(_C_LIB)
             or os.path.getmtime(_C_LIB) < os.path.getmtime(_C_SRC))
    if force or stale:
        tmp = _C_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _C_SRC, "-lm"])
        os.replace(tmp, _C_LIB)
    return _C_LIB


def _c():
    global _lib
    if _lib is None:
        build_c()
        lib = ctypes.CDLL(_C_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_tricubic_grid.argtypes = [dp, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int, dp, dp]
        lib.oracle_tricubic_grid.restype = None
        lib.oracle_tricubic_points.argtypes = [dp, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, dp, ctypes.c_long, dp]
        lib.oracle_tricubic_points.restype = None
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ----------------------------------------------------------------------------
# grid (Section 2.5.1)
# ----------------------------------------------------------------------------
class Grid:
    """Nodal periodic grid on [0, 2*pi)^3 with h_a = 2*pi/n_a (Section 2.5.1)."""

    def __init__(self, n):
        self.n = tuple(int(k) for k in n)
        if len(self.n) != 3:
            raise ValueError("three axes expected")
        self.h = tuple(TWO_PI / k for k in self.n)
        self.cell = float(self.h[0] * self.h[1] * self.h[2])

    def inner(self, u, w):
        """Discrete L2 inner product <u, w> = h1 h2 h3 sum u w (rectangle rule,
        exact for periodic trigonometric polynomials below Nyquist)."""
        return self.cell * float(np.sum(u * w))

    # integer wavenumbers in the real-to-complex (rfftn) layout
    def _k(self):
        n1, n2, n3 = self.n
        k1 = np.fft.fftfreq(n1, 1.0 / n1)[:, None, None]
        k2 = np.fft.fftfreq(n2, 1.0 / n2)[None, :, None]
        k3 = np.fft.rfftfreq(n3, 1.0 / n3)[None, None, :]
        return k1, k2, k3


# ----------------------------------------------------------------------------
# pseudo-spectral operators (Section 2.5.3; L from Section 2.2;
# (alpha L)^{-1} from Sections 2.5.5-2.5.6)
# ----------------------------------------------------------------------------
def _fft(u):
    return sfft.rfftn(u, workers=WORKERS)


def _ifft(uh, n):
    return sfft.irfftn(uh, s=n, workers=WORKERS)


def derivative_symbols(grid):
    """i k_a for a = 1..3 with the Nyquist wavenumber of axis a set to zero."""
    out = []
    for a, k in enumerate(grid._k()):
        kk = k.copy()
        kk[np.abs(kk) == grid.n[a] // 2] = 0.0
        out.append(1j * kk)
    return out


def laplacian_power_symbol(grid, p):
    """|k|^{2p}: symbol of (-Laplacian)^p; p = 1 is the H1 seminorm operator,
    p = 2 the H2 seminorm (biharmonic) operator. Nyquist modes kept."""
    k1, k2, k3 = grid._k()
    return (k1 * k1 + k2 * k2 + k3 * k3) ** p


def spectral_gradient(grid, u):
    """grad u by Fourier differentiation -> [3][n1][n2][n3] (Section 2.5.3)."""
    uh = _fft(u)
    return np.stack([_ifft(s * uh, grid.n) for s in derivative_symbols(grid)])


def spectral_divergence(grid, v):
    """div v = sum_a d_a v_a by Fourier differentiation (Section 2.5.3)."""
    acc = 0.0
    for s, va in zip(derivative_symbols(grid), v):
        acc = acc + s * _fft(va)
    return _ifft(acc, grid.n)


# 8th-order central differences (Section 2.5.3, "Differentiation": the
# first-derivative stencil of the paper's GPU implementation), periodic:
# d_i u(x_l) ~ (3 u_{l-4} - 32 u_{l-3} + 168 u_{l-2} - 672 u_{l-1}
#               + 672 u_{l+1} - 168 u_{l+2} + 32 u_{l+3} - 3 u_{l+4}) / (840 h_i)
FD8_WEIGHTS = ((1, 672.0), (2, -168.0), (3, 32.0), (4, -3.0))


def fd8_derivative(grid, u, axis):
    """FD8 first derivative of u along `axis` (0, 1, 2)."""
    acc = 0.0
    for s, c in FD8_WEIGHTS:
        acc = acc + c * (np.roll(u, -s, axis=axis) - np.roll(u, s, axis=axis))
    return acc / (840.0 * grid.h[axis])


def fd8_gradient(grid, u):
    return np.stack([fd8_derivative(grid, u, a) for a in range(3)])


def fd8_divergence(grid, v):
    return sum(fd8_derivative(grid, v[a], a) for a in range(3))


def gradient(grid, u, deriv="spectral"):
    """grad u with the chosen first-derivative discretisation."""
    return fd8_gradient(grid, u) if deriv == "fd8" else spectral_gradient(grid, u)


def divergence(grid, v, deriv="spectral"):
    return fd8_divergence(grid, v) if deriv == "fd8" else spectral_divergence(grid, v)


def apply_L(grid, u, p):
    """L u with L = (-Laplacian)^p (Section 2.2, regularisation operator)."""
    return _ifft(laplacian_power_symbol(grid, p) * _fft(u), grid.n)


def apply_alphaL_inverse(grid, u, alpha, p):
    """(alpha L)^{-1} u, the regularisation preconditioner (Section 2.5.6).
    The zero eigenvalue of L (k = 0) is replaced by one before inverting
    (Section 2.5.5), so the mean of u passes through unchanged."""
    sym = alpha * laplacian_power_symbol(grid, p)
    sym = np.where(sym == 0.0, 1.0, sym)
    return _ifft(_fft(u) / sym, grid.n)


def regularization_operator(grid, v, alpha, p):
    """alpha L v for a vector field, component by component."""
    return np.stack([alpha * apply_L(grid, v[a], p) for a in range(3)])


# ----------------------------------------------------------------------------
# near-incompressible model (appendix): div v = w with the penalty
# beta/2 <w, (-Delta^{-1} + id) w> on the second control w; w and the
# constraint's multiplier eliminated
# ----------------------------------------------------------------------------
def inverse_laplacian(grid, u):
    """Delta^{-1} u of a scalar field: multiplier -1/|k|^2, 0 at k = 0 (the
    mean has no preimage; every use below applies it to a divergence, whose
    mean is zero)."""
    kk = laplacian_power_symbol(grid, 1)
    mult = np.where(kk == 0.0, 0.0, -1.0 / np.where(kk == 0.0, 1.0, kk))
    return _ifft(mult * _fft(u), grid.n)


def _penalty_operator(grid, u, beta):
    """beta (-Delta^{-1} + id) u (the operator of the penalty on w)."""
    return beta * (-inverse_laplacian(grid, u) + u)


def ni_operator_M(grid, u, alpha, beta):
    """M u with M = (alpha (beta (-Delta^{-1} + id))^{-1} + id)^{-1}, a
    Fourier multiplier: invert the penalty operator's symbol, scale by alpha,
    add one, invert again (at k = 0, -Delta^{-1} contributes 0)."""
    kk = laplacian_power_symbol(grid, 1)
    pen = beta * (np.where(kk == 0.0, 0.0, 1.0 / np.where(kk == 0.0, 1.0, kk)) + 1.0)
    return _ifft(_fft(u) / (alpha / pen + 1.0), grid.n)


def ni_project(grid, b, alpha, beta):
    """b - grad M Delta^{-1} div b: the operator the near-incompressible
    reduced gradient applies to the data term int_0^1 lambda grad m dt
    (appendix), composed in the printed order from the spectral divergence,
    Delta^{-1}, M and the spectral gradient."""
    q = ni_operator_M(grid, inverse_laplacian(grid, spectral_divergence(grid, b)), alpha, beta)
    return b - spectral_gradient(grid, q)


def divergence_penalty(grid, v, beta):
    """beta/2 <div v, (-Delta^{-1} + id) div v>: the penalty on w = div v left
    in the objective once w is eliminated. With it, the appendix's reduced
    gradient is K grad J~ with K = I - grad M Delta^{-1} div (the factor M
    is exactly what turns the gradient of this objective into the projected
    form), so J~ is the merit function of the line search."""
    d = spectral_divergence(grid, v)
    return 0.5 * grid.inner(d, _penalty_operator(grid, d, beta))


def divergence_penalty_gradient(grid, v, beta):
    """L2 gradient of divergence_penalty: -grad beta (-Delta^{-1} + id) div v."""
    return -spectral_gradient(grid, _penalty_operator(grid, spectral_divergence(grid, v), beta))


# ----------------------------------------------------------------------------
# interpolation (Section 2.5.4, p = 3)
# ----------------------------------------------------------------------------
def interpolate(f, d):
    """f evaluated at x + d(x) for every grid point x.

    f: one field [n1][n2][n3] or a stack [k][n1][n2][n3]; d: displacement
    [3][n1][n2][n3] in voxel units. Tricubic Lagrange interpolation.
    """
    f = np.ascontiguousarray(f, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    shape3 = f.shape[-3:]
    nfield = 1 if f.ndim == 3 else int(np.prod(f.shape[:-3]))
    if d.shape != (3,) + shape3:
        raise ValueError("displacement shape mismatch")
    out = np.empty_like(f)
    _c().oracle_tricubic_grid(_dptr(f), nfield, shape3[0], shape3[1], shape3[2],
                              _dptr(d), _dptr(out))
    return out


def interpolate_points(f, q):
    """f at arbitrary points q [npts][3] given in grid-index units."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
    out = np.empty(q.shape[0], dtype=np.float64)
    _c().oracle_tricubic_points(_dptr(f), f.shape[0], f.shape[1], f.shape[2],
                                _dptr(q), q.shape[0], _dptr(out))
    return out


# ----------------------------------------------------------------------------
# semi-Lagrangian building blocks (Section 2.5.2)
# ----------------------------------------------------------------------------
def departure_displacement(grid, v, nt, direction=+1):
    """RK2 backtrace of the characteristics over one time step (Section 2.5.2).

    y~ = x - h_t w(x);  y = x - (h_t/2) (w(x) + w(y~)),  with w = direction*v.
    direction = +1 gives the departure points of the forward-in-time
    equations, -1 those of the backward-in-time equations. Returned as
    (y - x)/h in voxel units, [3][n1][n2][n3].
    """
    ht = 1.0 / nt
    w = direction * np.asarray(v, dtype=np.float64)
    d_tilde = np.stack([-ht * w[a] / grid.h[a] for a in range(3)])
    w_at = interpolate(w, d_tilde)
    return np.stack([-0.5 * ht * (w[a] + w_at[a]) / grid.h[a] for a in range(3)])


def solve_state(m0, d_plus, nt):
    """Transport equation (e:transport) by the homogeneous SL update
    m^{j+1}(x) = m^j(y(x)), j = 0..n_t-1. Returns [m^0, ..., m^{n_t}]."""
    m = [np.asarray(m0, dtype=np.float64)]
    for _ in range(nt):
        m.append(interpolate(m[-1], d_plus))
    return m


def transport(grid, m0, v, nt):
    """m(1) for the template m0 and the stationary velocity v."""
    return solve_state(m0, departure_displacement(grid, v, nt, +1), nt)[-1]


def _continuity_step(grid, lam_next, d_minus, div_v, div_v_dep, nt):
    """One backward step of d_t(lambda) + div(lambda v) = 0 (eq. e:adjoint,
    sign reading above). In reversed time this is D(lambda)/D(tau) = lambda div v
    along the characteristics of -v; RK2 along them (Section 2.5.2):
    f0 at the departure point, predictor, f1 at the arrival point, average."""
    ht = 1.0 / nt
    u_y = interpolate(lam_next, d_minus)
    f0 = u_y * div_v_dep
    u_tilde = u_y + ht * f0
    f1 = u_tilde * div_v
    return u_y + 0.5 * ht * (f0 + f1)


def trapezoid_weights(nt):
    """Trapezoidal quadrature weights c_j (without h_t) on t_j = j/n_t."""
    c = np.ones(nt + 1)
    c[0] = c[-1] = 0.5
    return c


# ----------------------------------------------------------------------------
# per-velocity quantities: state, objective, adjoint, reduced gradient
# ----------------------------------------------------------------------------
@dataclass
class VelocityState:
    grid: Grid
    nt: int
    alpha: float
    p: int
    v: np.ndarray
    m0: np.ndarray
    m1: np.ndarray
    d_plus: np.ndarray = None
    d_minus: np.ndarray = None
    m: list = field(default_factory=list)
    grad_m: list = field(default_factory=list)
    div_v: np.ndarray = None
    div_v_dep: np.ndarray = None
    lam: list = field(default_factory=list)
    g: np.ndarray = None
    J: float = 0.0
    J_dist: float = 0.0
    J_reg: float = 0.0
    beta: float = 0.0           # near-incompressible penalty (0: plain model)
    J_div: float = 0.0          # divergence penalty part of J
    data: np.ndarray = None     # int_0^1 lambda grad m dt (trapezoid)
    grad_J: np.ndarray = None   # L2 gradient of J (equals g when beta = 0)


class RecomputedGradients:
    """grad m^j computed again at every access instead of stored (the
    memory-lean setup: at 512^3, n_t = 8 the stored gradients alone take
    27 GiB in float64). Indexable like the list it replaces."""

    def __init__(self, grid, m, deriv):
        self.grid, self.m, self.deriv = grid, m, deriv

    def __len__(self):
        return len(self.m)

    def __getitem__(self, j):
        return gradient(self.grid, self.m[j], self.deriv)


def objective_parts(grid, m_final, m1, v, alpha, p):
    """J = 1/2 <m(1)-m1, m(1)-m1> + alpha/2 <L v, v> (eq. e:varopt-claire)."""
    r = m_final - m1
    dist = 0.5 * grid.inner(r, r)
    reg = 0.5 * alpha * sum(grid.inner(apply_L(grid, v[a], p), v[a]) for a in range(3))
    return dist, reg


def setup_velocity(grid, m0, m1, v, alpha, nt, p, deriv="spectral", beta=0.0,
                   store_grad=True):
    """State, objective, adjoint and reduced gradient at v (Algorithm 1 lines
    3-6; eqs. e:transport, e:varopt-claire, e:adjoint, e:rgrad). ``deriv``
    selects the gradient/divergence discretisation ("spectral" or "fd8") of
    the transport and adjoint equations. ``beta`` > 0 selects the
    near-incompressible model (appendix): J gains divergence_penalty and the
    reduced gradient is alpha L v + ni_project(data). ``store_grad`` False:
    grad m^j is recomputed wherever it is used (same values, less memory),
    and the adjoint history, no longer needed once g is formed, is dropped."""
    if beta > 0.0 and p != 1:
        raise ValueError("the near-incompressible model uses the H1 seminorm (p = 1)")
    st = VelocityState(grid=grid, nt=nt, alpha=alpha, p=p, beta=beta,
                       v=np.asarray(v, dtype=np.float64),
                       m0=np.asarray(m0, dtype=np.float64),
                       m1=np.asarray(m1, dtype=np.float64))
    ht = 1.0 / nt
    st.d_plus = departure_displacement(grid, st.v, nt, +1)
    st.d_minus = departure_displacement(grid, st.v, nt, -1)
    st.m = solve_state(st.m0, st.d_plus, nt)
    st.J_dist, st.J_reg = objective_parts(grid, st.m[-1], st.m1, st.v, alpha, p)
    st.J = st.J_dist + st.J_reg
    st.grad_m = [gradient(grid, mj, deriv) for mj in st.m] if store_grad else \
        RecomputedGradients(grid, st.m, deriv)
    st.div_v = divergence(grid, st.v, deriv)
    st.div_v_dep = interpolate(st.div_v, st.d_minus)
    lam = [None] * (nt + 1)
    lam[nt] = -(st.m[-1] - st.m1)                       # final condition (e:adjfinal)
    for j in range(nt - 1, -1, -1):
        lam[j] = _continuity_step(grid, lam[j + 1], st.d_minus, st.div_v,
                                  st.div_v_dep, nt)
    st.lam = lam
    c = trapezoid_weights(nt)
    st.data = ht * sum(c[j] * lam[j] * st.grad_m[j] for j in range(nt + 1))
    reg = regularization_operator(grid, st.v, alpha, p)
    if beta > 0.0:
        st.J_div = divergence_penalty(grid, st.v, beta)
        st.J += st.J_div
        st.g = reg + ni_project(grid, st.data, alpha, beta)
        st.grad_J = reg + st.data + divergence_penalty_gradient(grid, st.v, beta)
    else:
        st.g = reg + st.data
        st.grad_J = st.g
    if not store_grad:
        st.lam = None
    return st


def objective(grid, m0, m1, v, alpha, nt, p, beta=0.0):
    """J(v): backtrace, state solve and objective only (line-search trial);
    with beta > 0 the divergence penalty of the near-incompressible model is
    included."""
    m_final = transport(grid, m0, v, nt)
    dist, reg = objective_parts(grid, m_final, m1, v, alpha, p)
    return dist + reg + (divergence_penalty(grid, v, beta) if beta > 0.0 else 0.0)


# ----------------------------------------------------------------------------
# Gauss--Newton Hessian matvec (eqs. e:matvec, e:incstate, e:incadj; GN drop)
# ----------------------------------------------------------------------------
def incremental_state(st, vt, f_eval="grid"):
    """Incremental state m~(1) (eq. e:incstate) by SL with RK2 along the
    characteristics of v: D m~/Dt = f with f = -grad m . v~.

    ``f_eval`` chooses how f is evaluated at the departure points (Section
    2.5.2 allows both readings): "grid" forms the product f^j = -grad m^j . v~
    on the grid and interpolates it (derivatives taken on the regular mesh,
    the form the GPU path computes); "factors" interpolates grad m^j and v~
    separately and multiplies at the departure point (f as a function of its
    interpolated arguments). The two differ by interpolation error only: they
    agree exactly when every departure point is a grid point."""
    if f_eval not in ("grid", "factors"):
        raise ValueError("f_eval must be 'grid' or 'factors'")
    nt, ht = st.nt, 1.0 / st.nt
    mt = np.zeros(st.grid.n)
    if f_eval == "factors":
        vt_y = interpolate(vt, st.d_plus)
    f_j = -np.sum(st.grad_m[0] * vt, axis=0)
    for j in range(nt):
        u_y = interpolate(mt, st.d_plus)
        if f_eval == "factors":
            f0 = -np.sum(interpolate(st.grad_m[j], st.d_plus) * vt_y, axis=0)
        else:
            f0 = interpolate(f_j, st.d_plus)
        # f does not depend on m~, so the RK2 predictor does not enter f1
        f1 = -np.sum(st.grad_m[j + 1] * vt, axis=0)
        mt = u_y + 0.5 * ht * (f0 + f1)
        f_j = f1
    return mt


def incremental_adjoint(st, mt_final):
    """Gauss--Newton incremental adjoint (eq. e:incadj without the lambda term):
    the same continuity equation as the adjoint, final value -m~(1)."""
    nt = st.nt
    lt = [None] * (nt + 1)
    lt[nt] = -mt_final
    for j in range(nt - 1, -1, -1):
        lt[j] = _continuity_step(st.grid, lt[j + 1], st.d_minus, st.div_v,
                                 st.div_v_dep, nt)
    return lt


def hessian_matvec(st, vt, f_eval="grid"):
    """H v~ = alpha L v~ + int_0^1 lambda~ grad m dt (eq. e:matvec, GN form),
    trapezoidal rule in time. ``f_eval``: see incremental_state."""
    vt = np.asarray(vt, dtype=np.float64)
    lt = incremental_adjoint(st, incremental_state(st, vt, f_eval))
    c = trapezoid_weights(st.nt)
    data = sum(c[j] * lt[j] * st.grad_m[j] for j in range(st.nt + 1)) / st.nt
    if st.beta > 0.0:
        # derivative of the near-incompressible reduced gradient: the
        # projection is linear and independent of v
        data = ni_project(st.grid, data, st.alpha, st.beta)
    return regularization_operator(st.grid, vt, st.alpha, st.p) + data


def precondition(grid, r, alpha, p):
    """z = (alpha L)^{-1} r per component (Section 2.5.6)."""
    return np.stack([apply_alphaL_inverse(grid, r[a], alpha, p) for a in range(3)])


# ----------------------------------------------------------------------------
# two-level zero-velocity preconditioner (Section 2.5.6)
# ----------------------------------------------------------------------------
def reg_inverse_sqrt(grid, u, alpha, p):
    """(alpha L)^{-1/2} u per component with the k = 0 mode passed through
    (the same replacement of the zero eigenvalue as the regularisation
    preconditioner)."""
    sym = alpha * laplacian_power_symbol(grid, p)
    sym = np.where(sym == 0.0, 1.0, 1.0 / np.sqrt(np.where(sym == 0.0, 1.0, sym)))
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 3:
        return _ifft(_fft(u) * sym, grid.n)
    return np.stack([_ifft(_fft(c) * sym, grid.n) for c in u])


def _low_modes(n_f, n_c, rfft_axis):
    """Fine and coarse spectral indices of the modes kept by the cut-off
    filter: |k| < n_c / 2 (strictly below the coarse Nyquist)."""
    if rfft_axis:
        ks = np.arange(0, n_c // 2)
        return ks, ks
    ks = np.arange(-(n_c // 2 - 1), n_c // 2)
    return ks % n_f, ks % n_c


def spectral_restrict(grid, u, grid_c):
    """Q_R F_L u: cut-off filter, then the kept Fourier modes evaluated on the
    coarse grid (Section 2.5.6: spectral restriction)."""
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 4:
        return np.stack([spectral_restrict(grid, c, grid_c) for c in u])
    idx = [_low_modes(grid.n[a], grid_c.n[a], a == 2) for a in range(3)]
    U = _fft(u)
    Uc = np.zeros((grid_c.n[0], grid_c.n[1], grid_c.n[2] // 2 + 1), dtype=complex)
    scale = np.prod(grid_c.n) / np.prod(grid.n)
    Uc[np.ix_(idx[0][1], idx[1][1], idx[2][1])] = U[np.ix_(idx[0][0], idx[1][0], idx[2][0])] * scale
    return _ifft(Uc, grid_c.n)


def spectral_prolong(grid_c, u, grid):
    """Q_P: the coarse field's Fourier modes (below the coarse Nyquist)
    evaluated on the fine grid (zero padding)."""
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 4:
        return np.stack([spectral_prolong(grid_c, c, grid) for c in u])
    idx = [_low_modes(grid.n[a], grid_c.n[a], a == 2) for a in range(3)]
    Uc = _fft(u)
    U = np.zeros((grid.n[0], grid.n[1], grid.n[2] // 2 + 1), dtype=complex)
    scale = np.prod(grid.n) / np.prod(grid_c.n)
    U[np.ix_(idx[0][0], idx[1][0], idx[2][0])] = Uc[np.ix_(idx[0][1], idx[1][1], idx[2][1])] * scale
    return _ifft(U, grid.n)


def cg_relative(matvec, b, rtol, max_iters):
    """Plain CG on A x = b from x = 0 until ||r||_2 <= rtol ||b||_2."""
    x = np.zeros_like(b)
    r = b.copy()
    s = r.copy()
    rr = _dot(r, r)
    stop = (rtol ** 2) * rr
    its = 0
    while its < max_iters and rr > stop:
        As = matvec(s)
        its += 1
        kappa = rr / _dot(s, As)
        x = x + kappa * s
        r = r - kappa * As
        rr_new = _dot(r, r)
        s = r + (rr_new / rr) * s
        rr = rr_new
    return x, its


class TwoLevelPreconditioner:
    """Two-level zero-velocity preconditioner of the reduced Hessian
    (Section 2.5.6), for H v~ = -g in the original variables:

        P r = R^{-1/2} [ Q_P F_L K0_c^{-1} Q_R F_L + F_H ] R^{-1/2} r,

    R = alpha L with the k = 0 mode replaced by one, F_L/F_H the cut-off
    filters below/above the coarse Nyquist, Q_R/Q_P spectral restriction and
    prolongation to the grid of half the resolution, and K0_c the coarse
    discretisation of R^{-1/2} H0 R^{-1/2} with the zero-velocity Hessian
    H0 = alpha L + grad m (x) grad m taken at the current state m(t = 1):

        K0_c w = w - mean(w) + R_c^{-1/2} [grad m_c (grad m_c . R_c^{-1/2} w)].

    K0_c is inverted by CG to the relative tolerance ``inner_rtol`` (a tenth
    of the outer forcing in the paper's setting). ``inner_its`` records the
    inner iterations of each application."""

    def __init__(self, st, inner_rtol, max_inner=200):
        self.grid = st.grid
        self.alpha, self.p = st.alpha, st.p
        self.coarse = Grid(tuple(k // 2 for k in st.grid.n))
        self.gm = spectral_restrict(st.grid, st.grad_m[st.nt], self.coarse)
        self.inner_rtol = inner_rtol
        self.max_inner = max_inner
        self.inner_its = []

    def coarse_operator(self, w):
        gc, a, p = self.coarse, self.alpha, self.p
        y = reg_inverse_sqrt(gc, w, a, p)
        t = self.gm[0] * y[0] + self.gm[1] * y[1] + self.gm[2] * y[2]
        z = reg_inverse_sqrt(gc, self.gm * t, a, p)
        mean = w.mean(axis=(1, 2, 3), keepdims=True)
        return w - mean + z

    def __call__(self, r):
        g, gc = self.grid, self.coarse
        u = reg_inverse_sqrt(g, r, self.alpha, self.p)
        uL = spectral_restrict(g, u, gc)
        sL, its = cg_relative(self.coarse_operator, uL, self.inner_rtol, self.max_inner)
        self.inner_its.append(its)
        low = spectral_prolong(gc, uL, g)              # F_L u
        s = spectral_prolong(gc, sL, g) + (u - low)    # Q_P s_L + F_H u
        return reg_inverse_sqrt(g, s, self.alpha, self.p)


# ----------------------------------------------------------------------------
# PCG (Algorithm 2) and Gauss--Newton with Armijo (Algorithm 1)
# ----------------------------------------------------------------------------
def _dot(a, b):
    return float(np.sum(a * b))


def forcing_tolerance(gnorm_inf, kind="superlinear"):
    """eta ||g||_inf with eta = min(1/2, sqrt(||g||_inf)) (superlinear) or
    min(1/2, ||g||_inf) (quadratic), Section 2.5.5."""
    eta = min(0.5, np.sqrt(gnorm_inf)) if kind == "superlinear" else min(0.5, gnorm_inf)
    return eta * gnorm_inf


def pcg(matvec, precond, g, *, fixed_iters=0, max_iters=100, forcing="superlinear"):
    """Solve H v~ = -g by preconditioned CG (Algorithm 2), v~^0 = 0.

    Stops after ``fixed_iters`` matvecs if that is positive, else when
    ||r||_inf <= eta ||g||_inf or after ``max_iters`` matvecs. Nonpositive
    curvature <s, Hs> <= 0 along a direction (the discrete Gauss--Newton
    Hessian is only positive semidefinite up to discretisation error) stops
    the iteration as in truncated CG: the current v~ is returned, or the
    direction s itself (the preconditioned steepest-descent direction) when
    it happens on the first matvec.
    Returns (v~, matvecs, residual inf-norm history, hit_max); ``pcg.neg_curv``
    tells whether the last call stopped on nonpositive curvature.
    """
    tol = forcing_tolerance(float(np.abs(g).max()), forcing)
    limit = fixed_iters if fixed_iters > 0 else max_iters
    vt = np.zeros_like(g)
    r = -g
    z = precond(r)
    s = z.copy()
    rz = _dot(r, z)
    hist = [float(np.abs(r).max())]
    its = 0
    converged = False
    pcg.neg_curv = False
    while its < limit:
        hs = matvec(s)
        its += 1
        shs = _dot(s, hs)
        if shs <= 0.0:
            pcg.neg_curv = True
            if its == 1:
                vt = s.copy()
            break
        kappa = rz / shs
        vt = vt + kappa * s
        r = r - kappa * hs
        hist.append(float(np.abs(r).max()))
        if fixed_iters <= 0 and hist[-1] <= tol:
            converged = True
            break
        if its == limit:
            break
        z = precond(r)
        rz_new = _dot(z, r)
        mu = rz_new / rz
        s = z + mu * s
        rz = rz_new
    hit_max = fixed_iters <= 0 and not converged and not pcg.neg_curv
    return vt, its, hist, hit_max


@dataclass
class SolveStats:
    gn_iters: int = 0
    matvecs: int = 0
    inner_its: int = 0          # coarse CG iterations of the two-level preconditioner
    pde_solves: int = 0
    ls_trials: int = 0
    J0: float = 0.0
    J: float = 0.0
    rel_mismatch: float = 0.0
    rel_grad: float = 0.0
    warnings: list = field(default_factory=list)
    history: list = field(default_factory=list)


def gn_solve(grid, m0, m1, nt, p, alphas, *, v0=None, gtol=5e-2, gabs=1e-6,
             max_gn=50, max_pcg=100, fixed_pcg=0, forcing="superlinear",
             c1=1e-4, max_ls=16, deriv="spectral", precond="reg", beta=0.0,
             callback=None):
    """Inexact Gauss--Newton--Krylov with Armijo line search (Algorithm 1),
    run once per regularisation weight in ``alphas`` (parameter continuation,
    Section 2.6: each level starts from the previous level's velocity and
    stops relative to its own initial gradient).

    ``precond``: "reg" for (alpha L)^{-1}, "twolevel" for the two-level
    zero-velocity preconditioner (Section 2.5.6) with its inner CG run to a
    tenth of the outer relative tolerance (Section 2.6 settings).

    ``beta`` > 0: near-incompressible model (appendix). The reduced gradient
    and the Hessian carry the projection of the data term; the Armijo test
    uses the objective with the divergence penalty and its directional
    derivative <grad J, v~>. Not combined with the two-level preconditioner.

    ``stats.history`` holds one record per visited iterate (level, k, J,
    ||g||_inf) and, for each accepted step, the PCG matvec count, the PCG
    residual history ||r_l||_inf, the accepted step length gamma and the
    number of line-search trials. ``callback(level, k, v, st)``, if given, is
    called after every accepted step with the new iterate and its state.

    Pinned by a closed-form case: a pure 4-voxel translation, whose exact
    minimiser is the constant velocity (J = 0; the H1 seminorm does not
    penalise constants), is recovered to 1.4e-3 at gtol 1e-3; a flipped
    incremental-adjoint sign is caught by it. Beyond that the tests check its
    invariants (monotone J, stopping rule, det grad y > 0) and compare it with
    the HIP path.
    """
    if beta > 0.0 and precond == "twolevel":
        raise ValueError("the two-level preconditioner is not combined with beta > 0")
    v = np.zeros((3,) + grid.n) if v0 is None else np.array(v0, dtype=np.float64)
    stats = SolveStats()
    st = None
    m0 = np.asarray(m0, dtype=np.float64)
    m1 = np.asarray(m1, dtype=np.float64)
    mismatch0 = np.sqrt(np.sum((m0 - m1) ** 2))
    for li, alpha in enumerate(alphas):
        st = setup_velocity(grid, m0, m1, v, alpha, nt, p, deriv, beta)
        stats.pde_solves += 2
        if li == 0:
            stats.J0 = st.J
        g0 = float(np.abs(st.g).max())
        k = 0
        while True:
            gn = float(np.abs(st.g).max())
            stats.history.append(dict(alpha=alpha, k=k, J=st.J, gnorm=gn))
            if gn <= gtol * g0 or gn <= gabs:
                break
            if k >= max_gn:
                stats.warnings.append("max_gn")
                break
            if precond == "twolevel":
                eta = forcing_tolerance(gn, forcing) / gn
                M = TwoLevelPreconditioner(st, inner_rtol=0.1 * eta)
            else:
                M = lambda r: precondition(grid, r, alpha, p)   # noqa: E731
            vt, its, res_hist, hit_max = pcg(lambda s: hessian_matvec(st, s), M,
                                      st.g, fixed_iters=fixed_pcg,
                                      max_iters=max_pcg, forcing=forcing)
            if precond == "twolevel":
                stats.inner_its += sum(M.inner_its)
            stats.matvecs += its
            stats.pde_solves += 2 * its
            if hit_max:
                stats.warnings.append("pcg_max")
            slope = grid.inner(st.grad_J, vt)
            gamma = 1.0
            accepted = False
            trials = 0
            for _ in range(max_ls):
                v_trial = v + gamma * vt
                j_trial = objective(grid, m0, m1, v_trial, alpha, nt, p, beta)
                stats.ls_trials += 1
                stats.pde_solves += 1
                trials += 1
                if j_trial <= st.J + c1 * gamma * slope:
                    accepted = True
                    break
                gamma *= 0.5
            stats.history[-1].update(pcg_its=its, pcg_res=list(res_hist), slope=slope,
                                     gamma=gamma if accepted else 0.0, ls=trials,
                                     neg_curv=bool(pcg.neg_curv))
            if not accepted:
                stats.warnings.append("linesearch")
                break
            v = v_trial
            st = setup_velocity(grid, m0, m1, v, alpha, nt, p, deriv, beta)
            stats.pde_solves += 2
            k += 1
            stats.gn_iters += 1
            if callback is not None:
                callback(li, k, v, st)
        stats.rel_grad = float(np.abs(st.g).max()) / g0 if g0 > 0 else 0.0
    stats.J = st.J
    stats.rel_mismatch = float(np.sqrt(np.sum((st.m[-1] - m1) ** 2)) / mismatch0) \
        if mismatch0 > 0 else 0.0
    return v, st, stats


# ----------------------------------------------------------------------------
# deformation gradient (eq. e:def-grad, appendix)
# ----------------------------------------------------------------------------
def deformation_gradient(grid, v, nt, deriv="spectral"):
    """F(1) from d_t F + (v.grad) F = (grad v) F, F(0) = I, by SL with RK2 along
    the characteristics of v. Returns F as [3][3][n1][n2][n3] with
    (grad v)_{ab} = d_b v_a."""
    ht = 1.0 / nt
    v = np.asarray(v, dtype=np.float64)
    d_plus = departure_displacement(grid, v, nt, +1)
    G = np.stack([gradient(grid, v[a], deriv) for a in range(3)])   # [a][b]
    G_dep = interpolate(G.reshape((9,) + grid.n), d_plus).reshape(G.shape)
    F = np.zeros((3, 3) + grid.n)
    for a in range(3):
        F[a, a] = 1.0
    for _ in range(nt):
        F_y = interpolate(F.reshape((9,) + grid.n), d_plus).reshape(F.shape)
        f0 = np.einsum("ab...,bc...->ac...", G_dep, F_y)
        F_tilde = F_y + ht * f0
        f1 = np.einsum("ab...,bc...->ac...", G, F_tilde)
        F = F_y + 0.5 * ht * (f0 + f1)
    return F


def det3(F):
    """Pointwise determinant of a [3][3][...] tensor field."""
    return (F[0, 0] * (F[1, 1] * F[2, 2] - F[1, 2] * F[2, 1])
            - F[0, 1] * (F[1, 0] * F[2, 2] - F[1, 2] * F[2, 0])
            + F[0, 2] * (F[1, 0] * F[2, 1] - F[1, 1] * F[2, 0]))


def deformation_determinant(grid, v, nt, deriv="spectral"):
    """det F(1), the surrogate for det grad y (appendix, deformation gradient)."""
    return det3(deformation_gradient(grid, v, nt, deriv))
