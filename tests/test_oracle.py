"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: LAPACK's partial-pivoting
solve (same pivot rule), a manufactured solution built with independent einsum code, the
Stokes limit (one linear solve), the energy identity implied by skew-symmetry, the N = 1
closed form, Picard iteration (the alternative solver the paper names, Section 3.5),
brute-force multistart on tiny systems, quadratic convergence of Newton, and closed forms
for the a posteriori pressure recovery (eqns sup-vvar, blocksolve-2). A few tests plant a
mistake in the oracle's inputs (a transposed operand) and check that the pin catches it.
"""

import numpy as np
import pytest
import scipy.linalg as sla

from rbinputs import get_config, make_tensor_set, draw_mu
from rbinputs.synth import TensorSet


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


@pytest.fixture(scope="module")
def c1():
    return make_tensor_set(get_config("single_n10"))


@pytest.fixture(scope="module")
def c2():
    return make_tensor_set(get_config("batched_n50"))


def _random_set(N, Q=3, Qc=2, Qf=1, Np=4, Qb=1, seed=0, skew=False, scale=0.05):
    """Random dense tensors (no structure unless skew=True) for manufactured-solution tests."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((Q, N, N))
    A = np.einsum("qij,qkj->qik", A, A) + N * np.eye(N)[None]       # SPD terms
    C = scale * rng.standard_normal((Qc, N, N, N))
    if skew:
        C = 0.5 * (C - C.transpose(0, 3, 2, 1))
    F = rng.standard_normal((Qf, N))
    Bp = rng.standard_normal((Qb, Np, Np)) + 4 * np.eye(Np)[None]
    Asv = rng.standard_normal((Q, Np, N))
    Csv = rng.standard_normal((Qc, Np, N, N))
    Fs = rng.standard_normal((Qf, Np))
    return TensorSet(N=N, Q=Q, Qc=Qc, Qf=Qf, Np=Np, Qb=Qb, A=A, C=C, F=F, H=np.eye(N),
                     Bp=Bp, Asv=Asv, Csv=Csv, Fs=Fs)


def _op(ts, ta, tc):
    Am = np.tensordot(ta, ts.A, 1)
    Cm = np.tensordot(tc, ts.C, 1)
    return Am, Cm


# ---------------------------------------------------------------- theta ----

def test_theta_special_values(O):
    ta, tc, tf, tb = O.theta(12, 4, 2, 2, 0.0, 250.0)
    assert np.array_equal(ta, [1 / 250.0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0])
    assert np.array_equal(tc, [1, 1, 0, 0]) and np.array_equal(tf, [1, 0])
    assert np.array_equal(tb, [1, 0])
    a = np.pi / 3
    ta, tc, tf, tb = O.theta(12, 4, 2, 2, a, 100.0)
    assert abs(ta[1] - 0.5) < 1e-15 and abs(ta[2] - np.sqrt(3) / 2) < 1e-15
    assert abs(ta[6] + 0.5) < 1e-15 and abs(ta[8] - 0.5) < 1e-15      # cos 2a, 1 - cos a
    assert abs(ta[3] ** 2 - ta[4]) < 1e-15 and abs(ta[3] * ta[4] - ta[5]) < 1e-15
    assert np.array_equal(O.theta(3, 1, 1, 1, a, 100.0)[2], [1.0])
    with pytest.raises(ValueError):
        O.theta(65, 1, 1, 1, a, 100.0)


def test_theta_piola_power_families(O):
    """Expansions longer than the trigonometric lists are the Piola-mapped forms' power series
    in the angle (Section 5; 4n + 2 = 50 terms of a and 4n + 1 = 49 of c at n = 12): checked
    against closed forms of the truncated geometric series and of the limits."""
    re = 640.0
    ta, tc, _, _ = O.theta(50, 49, 2, 2, 0.0, re)
    assert ta[0] == 1.0 / re and np.all(ta[1:] == 0.0)          # alpha = 0: only the constant
    assert tc[0] == 1.0 and np.all(tc[1:] == 0.0)
    a = np.deg2rad(35.0)
    ta, tc, _, _ = O.theta(50, 49, 2, 2, a, re)
    assert abs(ta.sum() * re - (1 - a ** 50) / (1 - a)) < 1e-14 * (1 - a) ** -1
    assert abs(tc.sum() - (1 - a ** 49) / (1 - a)) < 1e-14 * (1 - a) ** -1
    assert np.allclose(ta[1:] / ta[:-1], a, rtol=1e-15) and np.allclose(tc[1:] / tc[:-1], a, rtol=1e-15)
    # a short family keeps the trigonometric list
    assert np.array_equal(O.theta(12, 4, 2, 2, a, re)[0][:3], O.theta(3, 1, 2, 2, a, re)[0])


# ----------------------------------------------------------------- GEPP ----

@pytest.mark.parametrize("n", [1, 2, 5, 17, 50, 64])
def test_gepp_matches_lapack(O, n):
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, st = O.gepp_solve(M, b)
    ref = np.linalg.solve(M, b)
    assert st == 0
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.cond(M) * np.linalg.norm(ref)


def test_gepp_pivot_order_matches_lapack_ties(O):
    """Ties in |pivot| go to the smallest current row index, as LAPACK's getrf does."""
    M = np.array([[1.0, 2, 3, 1], [-1, 0, 1, 2], [1, 1, -2, 0], [2, -2, 1, 1]])
    for perm in ([0, 1, 2, 3], [2, 0, 3, 1], [3, 2, 1, 0]):
        Mp = M[perm]
        _, st, piv = O.gepp_solve(Mp, np.ones(4), return_piv=True)
        lu, lapack_piv = sla.lu_factor(Mp)
        assert st == 0
        assert np.array_equal(piv, lapack_piv)


def test_gepp_singular_and_nonfinite(O):
    assert O.gepp_solve(np.zeros((3, 3)), np.ones(3))[1] == 2
    M = np.eye(3)
    M[1, 2] = np.nan
    assert O.gepp_solve(M, np.ones(3))[1] == 3
    assert O.gepp_solve(np.eye(3), np.array([1.0, np.inf, 0]))[1] == 3


# --------------------------------------------------------------- Newton ----

@pytest.mark.parametrize("skew", [False, True])
def test_manufactured_solution(O, skew):
    """f := A u* + C(u*, u*) (independent einsum) -> Newton returns u*."""
    ts = _random_set(12, skew=skew)
    os_ = O.OracleSet(ts)
    rng = np.random.default_rng(5)
    ta, tc = np.array([1.0, 0.3, 0.2]), np.array([1.0, 0.7])
    Am, Cm = _op(ts, ta, tc)
    ustar = rng.standard_normal(12)
    f = Am @ ustar + np.einsum("ijk,j,k->i", Cm, ustar, ustar)
    u, st, it, hist = O.newton(os_, 12, ta, tc, f, tol=1e-14, maxit=30)
    assert st == 0
    assert np.linalg.norm(u - ustar) <= 1e-12 * np.linalg.norm(ustar)


def test_manufactured_catches_transposed_operands(O):
    """Planted mistakes: C with its test and advecting indices swapped, or a wrong term in A,
    must move the root away from u*. (Swapping the advecting and advected indices is not a
    mistake: C(u,u) and the symmetrised Jacobian are invariant under it.)"""
    ts = _random_set(8, skew=False, scale=0.1)
    ta, tc = np.array([1.0, 0.3, 0.2]), np.array([1.0, 0.7])
    Am, Cm = _op(ts, ta, tc)
    ustar = np.random.default_rng(3).standard_normal(8)
    f = Am @ ustar + np.einsum("ijk,j,k->i", Cm, ustar, ustar)
    for bad in (dict(C=ts.C.transpose(0, 2, 1, 3)), dict(A=ts.A + 0.1 * np.triu(np.ones((8, 8))))):
        d = {k: getattr(ts, k) for k in ("A", "C", "F", "H", "Bp", "Asv", "Csv", "Fs")}
        d.update({k: np.ascontiguousarray(v) for k, v in bad.items()})
        ts_bad = TensorSet(N=8, Q=3, Qc=2, Qf=1, Np=4, Qb=1, **d)
        u, st, it, _ = O.newton(O.OracleSet(ts_bad), 8, ta, tc, f, tol=1e-14, maxit=30)
        assert np.linalg.norm(u - ustar) > 1e-6 * np.linalg.norm(ustar)


def test_stokes_limit_single_linear_solve(O, c2):
    os_ = O.OracleSet(c2)
    ta, tc, tf, _ = O.theta(c2.Q, c2.Qc, c2.Qf, c2.Qb, 0.3, 400.0)
    f = tf @ c2.F
    u, st, it, hist = O.newton(os_, c2.N, ta, np.zeros_like(tc), f, tol=1e-12, maxit=10)
    Am = np.tensordot(ta, c2.A, 1)
    ref = np.linalg.solve(Am, f)
    assert st == 0 and it == 2
    assert hist[1] <= 1e-14 * hist[0]
    assert np.linalg.norm(u - ref) <= 1e-13 * np.linalg.cond(Am) * np.linalg.norm(ref)


def test_first_iterate_is_stokes_solution(O, c2):
    os_ = O.OracleSet(c2)
    ta, tc, tf, _ = O.theta(c2.Q, c2.Qc, c2.Qf, c2.Qb, 0.4, 300.0)
    f = tf @ c2.F
    u1, st, it, _ = O.newton(os_, c2.N, ta, tc, f, tol=1e-12, maxit=1)
    assert st == 1 and it == 1
    assert np.allclose(u1, np.linalg.solve(np.tensordot(ta, c2.A, 1), f), rtol=1e-12, atol=0)


def test_energy_identity(O, c2):
    """Skew-symmetry gives u^T C(u,u) = 0, so the root satisfies u^T A(mu) u = f^T u."""
    os_ = O.OracleSet(c2)
    for a, re in [(0.1, 150.0), (0.55, 900.0)]:
        ta, tc, tf, _ = O.theta(c2.Q, c2.Qc, c2.Qf, c2.Qb, a, re)
        f = tf @ c2.F
        u, st, it, _ = O.newton(os_, c2.N, ta, tc, f)
        assert st == 0
        uAu = u @ np.tensordot(ta, c2.A, 1) @ u
        assert abs(uAu - f @ u) <= 1e-13 * abs(uAu)


def test_n1_closed_form(O, c1):
    """For N = 1 skew-symmetry forces C_111 = 0, so u = f / a exactly."""
    os_ = O.OracleSet(c1)
    ta, tc, tf, _ = O.theta(c1.Q, c1.Qc, c1.Qf, c1.Qb, np.deg2rad(10), 200.0)
    f = tf @ c1.F
    u, st, it, _ = O.newton(os_, 1, ta, tc, f[:1])
    a = np.tensordot(ta, c1.A, 1)[0, 0]
    assert st == 0 and abs(u[0] - f[0] / a) <= 1e-15 * abs(f[0] / a)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_picard_agrees_with_newton(O, c1, n):
    os_ = O.OracleSet(c1)
    ta, tc, tf, _ = O.theta(c1.Q, c1.Qc, c1.Qf, c1.Qb, np.deg2rad(10), 200.0)
    f = (tf @ c1.F)[:n]
    un, st, _, _ = O.newton(os_, n, ta, tc, f, tol=1e-15, maxit=20)
    up, sp, _ = O.picard(os_, n, ta, tc, f, tol=1e-15, maxit=2000)
    assert sp == 0
    assert np.linalg.norm(un - up) <= 1e-12 * np.linalg.norm(up)


def test_bruteforce_single_root_tiny(O, c1):
    """Multistart Newton from a 9x9 grid in a ball around the Stokes solution: one root."""
    os_ = O.OracleSet(c1)
    n = 2
    ta, tc, tf, _ = O.theta(c1.Q, c1.Qc, c1.Qf, c1.Qb, np.deg2rad(10), 200.0)
    f = (tf @ c1.F)[:n]
    us = np.linalg.solve(np.tensordot(ta, c1.A, 1)[:n, :n], f)
    R = 3 * np.linalg.norm(us)
    roots = []
    for x in np.linspace(-R, R, 9):
        for y in np.linspace(-R, R, 9):
            u, st, _, _ = O.newton(os_, n, ta, tc, f, tol=1e-14, maxit=50, u0=us + [x, y])
            if st == 0:
                roots.append(u)
    roots = np.array(roots)
    assert len(roots) > 40
    assert np.max(np.linalg.norm(roots - roots[0], axis=1)) <= 1e-12 * np.linalg.norm(roots[0])


def test_quadratic_convergence(O, c2):
    os_ = O.OracleSet(c2)
    ta, tc, tf, _ = O.theta(c2.Q, c2.Qc, c2.Qf, c2.Qb, 0.0, 100.0)   # the hardest corner
    f = tf @ c2.F * 3.0                                              # push the nonlinearity
    u, st, it, hist = O.newton(os_, c2.N, ta, tc, f, tol=1e-14, maxit=20)
    assert st == 0
    ratios = [hist[t + 1] / hist[t] ** 2 for t in range(len(hist) - 1) if hist[t + 1] > 1e-9 * hist[0]]
    assert len(ratios) >= 2
    assert max(ratios) < 10 * min(ratios) + 1e-3


def test_maxit_status(O, c2):
    os_ = O.OracleSet(c2)
    ta, tc, tf, _ = O.theta(c2.Q, c2.Qc, c2.Qf, c2.Qb, 0.2, 500.0)
    _, st, it, _ = O.newton(os_, c2.N, ta, tc, tf @ c2.F, maxit=1)
    assert st == 1 and it == 1


def test_singular_status(O, c2):
    os_ = O.OracleSet(c2)
    _, st, it, _ = O.newton(os_, c2.N, np.zeros(c2.Q), np.zeros(c2.Qc), np.ones(c2.N))
    assert st == 2 and it == 0


def test_batch_nested_matches_single(O, c2):
    os_ = O.OracleSet(c2)
    cfg = get_config("batched_n50")
    mu = draw_mu(cfg, 6)
    Nr = np.array([50, 20, 35, 1, 50, 7], dtype=np.int32)
    r = O.solve_batch(os_, mu, Nreq=Nr, pressure_np=c2.Np, nthreads=2)
    for b in range(6):
        n = Nr[b]
        sub = O.OracleSet(c2.leading(n))
        ta, tc, tf, tb = O.theta(c2.Q, c2.Qc, c2.Qf, c2.Qb, *mu[b])
        u, st, it, _ = O.newton(sub, n, ta, tc, tf @ c2.F[:, :n])
        assert st == r["status"][b] and it == r["iters"][b]
        # (f(mu) is summed by numpy here and by the C loop in the batch: rounding only)
        assert np.linalg.norm(u - r["u"][b, :n]) <= 1e-13 * np.linalg.norm(u)
        assert not np.any(r["u"][b, n:])
    bad = O.solve_batch(os_, mu[:2], Nreq=np.array([0, 51], dtype=np.int32))
    assert list(bad["status"]) == [4, 4]


# ------------------------------------------------------------- pressure ----

def test_pressure_manufactured(O):
    ts = _random_set(9, Np=5, Qb=2, seed=7)
    os_ = O.OracleSet(ts)
    rng = np.random.default_rng(8)
    u = rng.standard_normal(9)
    ta, tc, tf, tb = np.array([1.0, 0.5, 0.25]), np.array([1.0, -0.3]), np.array([1.0]), np.array([1.0, 0.4])
    p, st = O.pressure(os_, 9, 5, ta, tc, tf, tb, u)
    Bm = np.tensordot(tb, ts.Bp, 1)
    rhs = (tf @ ts.Fs - np.tensordot(ta, ts.Asv, 1) @ u
           - np.einsum("ijk,j,k->i", np.tensordot(tc, ts.Csv, 1), u, u))
    assert st == 0
    assert np.allclose(p, np.linalg.solve(Bm, rhs), rtol=1e-12, atol=1e-13)


def test_pressure_of_gradient_forcing(O):
    """g = grad(sum_j c_j p_j): the velocity load vanishes, u = 0, and at alpha = 0 the
    recovered pressure is c exactly (B(0) is the supremizer Gramian = I)."""
    from rbinputs import synth as S
    cfg = get_config("single_n10")
    d = S.assemble(8, 5, 6, 32, 3, 1, 1, 2, cfg["seeds"])
    K = d["K"]
    c = np.array([0.7, -1.2, 0.4, 2.0, -0.3])
    q = np.tensordot(c, d["p_c"], 1)                               # (W, 2)
    g = np.stack([S.deriv(q, K, 0), S.deriv(q, K, 1)])[None]       # (1, 2, W, 2)
    E = S.grid_modes(K, 32)
    gg, phi, s = S.on_grid(g, E), S.on_grid(d["phi_c"], E), S.on_grid(d["s_c"], E)
    F = np.einsum("qbx,ibx->qi", gg, phi) / E.shape[1]
    Fs = np.einsum("qbx,ibx->qi", gg, s) / E.shape[1]
    assert np.max(np.abs(F)) < 1e-12
    ts = TensorSet(N=8, Q=3, Qc=1, Qf=1, Np=5, Qb=2, A=d["A"], C=d["C"], F=F, H=d["H"],
                   Bp=d["Bp"], Asv=d["Asv"], Csv=d["Csv"], Fs=Fs)
    os_ = O.OracleSet(ts)
    r = O.solve_batch(os_, np.array([[0.0, 300.0]]), pressure_np=5)
    assert r["status"][0] == 0 and np.max(np.abs(r["u"])) < 1e-14
    assert np.allclose(r["p"][0], c, rtol=0, atol=1e-12)


def test_block_triangular_equals_coupled_solve(O, c2):
    """The velocity-then-pressure solve equals the coupled block system with s = 0 (eqn
    piolablock): the Newton root plus recovered p solve [J 0; A_sv+C_sv(u,.) B] at the root."""
    os_ = O.OracleSet(c2)
    ta, tc, tf, tb = O.theta(c2.Q, c2.Qc, c2.Qf, c2.Qb, 0.25, 700.0)
    u, st, _, _ = O.newton(os_, c2.N, ta, tc, tf @ c2.F)
    p, sp = O.pressure(os_, c2.N, c2.Np, ta, tc, tf, tb, u)
    Am, Cm = _op(c2, ta, tc)
    Asv = np.tensordot(ta, c2.Asv, 1)
    Csv = np.tensordot(tc, c2.Csv, 1)
    Bm = np.tensordot(tb, c2.Bp, 1)
    res_v = Am @ u + np.einsum("ijk,j,k->i", Cm, u, u) - tf @ c2.F
    res_s = Bm @ p + Asv @ u + np.einsum("ijk,j,k->i", Csv, u, u) - tf @ c2.Fs
    assert st == 0 and sp == 0
    assert np.linalg.norm(res_v) <= 1e-10 * np.linalg.norm(tf @ c2.F)
    assert np.linalg.norm(res_s) <= 1e-12 * np.linalg.norm(tf @ c2.Fs)


def _leray_case():
    """Qc = 1 synthetic set (N = Np = 8, |k| <= 6, 32 x 32 grid), a random velocity u in the
    span, and the pressure the continuous equations give for it.

    With M_0 = I the convection form is the true one, and at alpha = 0 the pressure form is
    b_0(p, w) = -int p div w. The supremizers solve -Laplace(s_i) = grad(p_i), so
    div(s_i) = -p_i and b_0(p_j, s_i) = (p_j, p_i) = delta_ij. They are gradients, so every
    solenoidal field is L2-orthogonal to them and A_sv = 0. The recovery equation
    b(p, s_i) = (g, s_i) - c(u, u, s_i) therefore reads (p, p_i) = (w, s_i) with
    w = g - (u . grad) u; writing w = w_sol + grad(P) (Leray), (w, s_i) = (grad P, s_i) =
    (P, p_i). So the recovered coefficients are the L2 projections (P, p_i) of the Leray
    pressure P, which solves Laplace(P) = div(w). P is computed here by FFT on the grid, a
    route that shares nothing with the tensors' quadrature.
    """
    from rbinputs import synth as S
    seeds = get_config("single_n10")["seeds"]
    N, Np, kmax, G = 8, 8, 6, 32
    d = S.assemble(N, Np, kmax, G, 3, 1, 1, 2, seeds, forcing_scale=1.0)
    K = d["K"]
    E = S.grid_modes(K, G)
    u = np.random.default_rng(11).standard_normal(N)
    Uc = np.tensordot(u, d["phi_c"], 1)                                  # (2, W, 2)
    U = S.on_grid(Uc, E)                                                 # (2, G^2)
    dU = np.stack([S.on_grid(S.deriv(Uc, K, a), E) for a in range(2)])   # dU[a, b] = d_a U^b
    w = S.on_grid(d["g_c"][0], E) - np.einsum("ax,abx->bx", U, dU)
    wh = [np.fft.fft2(w[b].reshape(G, G)) for b in range(2)]
    f = np.fft.fftfreq(G, d=1.0 / G)
    KX, KY = np.meshgrid(f, f, indexing="ij")                            # grid is x-major
    k2 = KX ** 2 + KY ** 2
    k2[0, 0] = 1.0
    Ph = -1j * (KX * wh[0] + KY * wh[1]) / (2.0 * np.pi * k2)           # Laplace P = div w
    Ph[0, 0] = 0.0
    P = np.fft.ifft2(Ph).real.reshape(-1)
    p_expected = S.on_grid(d["p_c"], E) @ P / G ** 2                     # (P, p_i)
    return d, u, p_expected


def _leray_set(d, **over):
    kw = dict(A=d["A"], C=d["C"], F=d["F"], H=d["H"], Bp=d["Bp"], Asv=d["Asv"], Csv=d["Csv"],
              Fs=d["Fs"])
    kw.update(over)
    return TensorSet(N=8, Q=3, Qc=1, Qf=1, Np=8, Qb=2, **kw)


def test_pressure_velocity_terms_leray_projection(O):
    """The velocity-dependent part of the recovery (C_sv(u, u), with A_sv(u) = 0), pinned by
    the continuous pressure of eqn sup-vvar: the recovered p is the L2 projection of the
    Leray pressure of g - (u . grad) u onto the pressure basis."""
    d, u, p_exp = _leray_case()
    ta, tc, tf, tb = O.theta(3, 1, 1, 2, 0.0, 300.0)
    p, st = O.pressure(O.OracleSet(_leray_set(d)), 8, 8, ta, tc, tf, tb, u)
    assert st == 0
    assert np.linalg.norm(p_exp) > 0.1                      # the velocity term matters
    assert np.max(np.abs(p - p_exp)) <= 1e-12 * np.max(np.abs(p_exp))


@pytest.mark.parametrize("plant", ["flipped_sign", "test_index_slot", "dropped_term"])
def test_pressure_leray_catches_planted_mistakes(O, plant):
    """A flipped sign of the convection term, the test index in the advecting slot, or a
    dropped convection term each move the recovered pressure by O(1) against the pin."""
    d, u, p_exp = _leray_case()
    Csv = {"flipped_sign": -d["Csv"],
           "test_index_slot": np.ascontiguousarray(d["Csv"].transpose(0, 2, 1, 3)),
           "dropped_term": np.zeros_like(d["Csv"])}[plant]
    ta, tc, tf, tb = O.theta(3, 1, 1, 2, 0.0, 300.0)
    p, _ = O.pressure(O.OracleSet(_leray_set(d, Csv=Csv)), 8, 8, ta, tc, tf, tb, u)
    assert np.max(np.abs(p - p_exp)) > 0.1 * np.max(np.abs(p_exp))
