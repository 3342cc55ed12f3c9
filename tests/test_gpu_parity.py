"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Every test runs the same seeded inputs through both sides and compares element by element:
relative error <= 1e-10 per request for the FP64 path (the tolerance the target states for
it), bit-exact for integer outputs (status codes; Newton iteration counts equal except where
the stopping test sits within rounding of the threshold). Sizes span several 16-request
tiles with a ragged tail; the full-size batch of 4096 requests at N = 50 is checked on a
sample of requests the oracle solves one by one, in the launch configuration of the bench.
"""

import numpy as np
import pytest

from rbinputs import get_config, make_tensor_set, draw_mu
from rbinputs.synth import TensorSet

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_F64 = 1e-10


def _rel(a, b):
    nb = np.linalg.norm(b, axis=-1)
    na = np.linalg.norm(a - b, axis=-1)
    return np.where(nb > 0, na / np.where(nb > 0, nb, 1), na)


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_11866_amd import rbns
    rbns.load()
    return rbns


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def _random_set(N, Q=3, Qc=2, Qf=2, Np=5, Qb=2, seed=0, scale=0.05, H=True):
    """Random SPD A_q, C_q skew in (i, k) (so c(u, v, v) = 0 as for solenoidal fields), a
    pressure block near the identity; scale keeps Newton from u = 0 convergent."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((Q, N, N))
    A = np.einsum("qij,qkj->qik", A, A) / N + 2 * np.eye(N)[None]
    C = scale * rng.standard_normal((Qc, N, N, N))
    C = 0.5 * (C - C.transpose(0, 3, 2, 1))
    F = rng.standard_normal((Qf, N))
    Bp = 0.2 * rng.standard_normal((Qb, Np, Np)) + np.eye(Np)[None]
    Asv = rng.standard_normal((Q, Np, N))
    Csv = rng.standard_normal((Qc, Np, N, N))
    Fs = rng.standard_normal((Qf, Np))
    Hm = np.eye(N) + 0.1 * np.ones((N, N)) if H else None
    return TensorSet(N=N, Q=Q, Qc=Qc, Qf=Qf, Np=Np, Qb=Qb, A=A, C=C, F=F, H=Hm, Bp=Bp,
                     Asv=Asv, Csv=Csv, Fs=Fs)


def _oracle_theta(O, ts, mu):
    th = [O.theta(ts.Q, ts.Qc, ts.Qf, ts.Qb, a, re) for a, re in mu]
    return [np.array([t[i] for t in th]) for i in range(4)]


@pytest.fixture(scope="module")
def c1():
    return make_tensor_set(get_config("single_n10"))


@pytest.fixture(scope="module")
def c2():
    return make_tensor_set(get_config("batched_n50"))


# ------------------------------------------------------------------------ theta ----

def test_theta_matches_oracle(O, R, c2):
    s = R.Solver(c2)
    mu = draw_mu(get_config("batched_n50"), 333)
    th = s.theta(_dev(mu))
    torch.cuda.synchronize()
    ta, tc, tf, tb = _oracle_theta(O, c2, mu)
    for got, ref in ((th["ta"], ta), (th["tc"], tc), (th["tf"], tf), (th["tb"], tb)):
        assert np.max(np.abs(got.cpu().numpy() - ref)) <= 4e-16 * max(1.0, np.abs(ref).max())
    s.close()


# ------------------------------------------------------------------------ solves ---

def _gpu_solve(R, s, ts, mu, N=None, **kw):
    th = s.theta(_dev(mu))
    out = s.solve(th, N=N, **kw)
    torch.cuda.synchronize()
    return th, {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("B", [1, 37])
def test_single_n10_parity(O, R, c1, B):
    cfg = get_config("single_n10")
    mu = draw_mu(cfg, B)
    s = R.Solver(c1)
    _, g = _gpu_solve(R, s, c1, mu)
    r = O.solve_batch(O.OracleSet(c1), mu, pressure_np=c1.Np)
    assert np.array_equal(g["status"], r["status"]) and np.all(g["status"] == 0)
    assert np.array_equal(g["iters"], r["iters"])
    assert np.max(_rel(g["u"], r["u"])) <= TOL_F64
    s.close()


def test_batched_n50_parity_ragged(O, R, c2):
    cfg = get_config("batched_n50")
    mu = draw_mu(cfg, 300, seed_offset=11)        # 18 full tiles + a tail of 12
    s = R.Solver(c2)
    th, g = _gpu_solve(R, s, c2, mu)
    r = O.solve_batch(O.OracleSet(c2), mu, pressure_np=c2.Np)
    assert np.all(g["status"] == 0) and np.array_equal(g["status"], r["status"])
    assert np.mean(g["iters"] == r["iters"]) >= 0.99
    assert np.max(np.abs(g["iters"] - r["iters"])) <= 1
    err = _rel(g["u"], r["u"])
    assert np.max(err) <= TOL_F64, (np.max(err), np.percentile(err, 99))
    # pressure recovery
    p = s.pressure(th, torch.as_tensor(g["u"]).cuda())
    torch.cuda.synchronize()
    pg = p["p"].cpu().numpy()
    assert np.all(p["pstatus"].cpu().numpy() == 0)
    assert np.max(_rel(pg, r["p"])) <= TOL_F64
    s.close()


def test_full_batch_4096_sampled(O, R, c2):
    """The bench's launch: 4096 requests at N = 50; the oracle re-solves a sample."""
    cfg = get_config("batched_n50")
    mu = draw_mu(cfg)
    s = R.Solver(c2)
    th, g = _gpu_solve(R, s, c2, mu)
    p = s.pressure(th, torch.as_tensor(g["u"]).cuda())
    torch.cuda.synchronize()
    pg = p["p"].cpu().numpy()
    idx = np.unique(np.concatenate([np.arange(0, 4096, 97), [15, 16, 4095]]))
    r = O.solve_batch(O.OracleSet(c2), mu[idx], pressure_np=c2.Np)
    assert np.all(g["status"] == 0)
    assert np.max(_rel(g["u"][idx], r["u"])) <= TOL_F64
    assert np.max(_rel(pg[idx], r["p"])) <= TOL_F64
    s.close()


@pytest.mark.parametrize("N", [1, 7, 8, 9, 16, 33, 50, 64])
def test_random_tensors_every_bucket(O, R, N):
    ts = _random_set(N, seed=N)
    mu = np.column_stack([np.linspace(0.0, 0.6, 21), np.linspace(100, 1000, 21)])
    s = R.Solver(ts)
    th, g = _gpu_solve(R, s, ts, mu, max_iter=20)
    r = O.solve_batch(O.OracleSet(ts), mu, maxit=20, pressure_np=ts.Np)
    assert np.array_equal(g["status"], r["status"]) and np.all(g["status"] == 0)
    assert np.max(_rel(g["u"], r["u"])) <= TOL_F64
    p = s.pressure(th, torch.as_tensor(g["u"]).cuda())
    torch.cuda.synchronize()
    assert np.max(_rel(p["p"].cpu().numpy(), r["p"])) <= TOL_F64
    s.close()


def test_nested_leading_blocks(O, R, c2):
    mu = draw_mu(get_config("batched_n50"), 40, seed_offset=3)
    s = R.Solver(c2)
    for n, npr in ((20, 10), (37, 30)):
        th, g = _gpu_solve(R, s, c2, mu, N=n)
        r = O.solve_batch(O.OracleSet(c2), mu, Nreq=np.full(40, n, np.int32), pressure_np=npr)
        assert np.max(_rel(g["u"][:, :n], r["u"][:, :n])) <= TOL_F64
        assert not np.any(g["u"][:, n:])
        p = s.pressure(th, torch.as_tensor(g["u"]).cuda(), N=n, Np=npr)
        torch.cuda.synchronize()
        pg = p["p"].cpu().numpy()
        sub = O.OracleSet(c2)
        for b in range(0, 40, 13):
            ta, tc, tf, tb = O.theta(c2.Q, c2.Qc, c2.Qf, c2.Qb, *mu[b])
            pr, st = O.pressure(sub, n, npr, ta, tc, tf, tb, r["u"][b, :n])
            assert st == 0 and np.linalg.norm(pg[b, :npr] - pr) <= TOL_F64 * np.linalg.norm(pr)
            assert not np.any(pg[b, npr:])
    s.close()


def test_manufactured_solution_on_gpu(R):
    """f := A u* + C(u*,u*) built here with numpy; the GPU Newton must return u*."""
    ts = _random_set(24, seed=5, scale=0.1)
    rng = np.random.default_rng(9)
    B = 33
    ustar = rng.standard_normal((B, 24))
    ta = rng.uniform(0.5, 1.5, (B, ts.Q))
    tc = rng.uniform(-1, 1, (B, ts.Qc))
    f = np.einsum("bq,qij,bj->bi", ta, ts.A, ustar) + np.einsum("bq,qijk,bj,bk->bi", tc, ts.C, ustar, ustar)
    s = R.Solver(ts)
    th = dict(ta=_dev(ta), tc=_dev(tc), tf=_dev(np.zeros((B, ts.Qf))))
    out = s.solve(th, f_override=_dev(f), tol=1e-14, max_iter=30)
    torch.cuda.synchronize()
    assert np.all(out["status"].cpu().numpy() == 0)
    assert np.max(_rel(out["u"].cpu().numpy(), ustar)) <= 1e-12
    s.close()


def test_stokes_limit_on_gpu(R, c2):
    mu = draw_mu(get_config("batched_n50"), 20)
    s = R.Solver(c2)
    th = s.theta(_dev(mu))
    th["tc"].zero_()
    out = s.solve(th)
    torch.cuda.synchronize()
    ta = th["ta"].cpu().numpy()
    tf = th["tf"].cpu().numpy()
    for b in range(20):
        ref = np.linalg.solve(np.tensordot(ta[b], c2.A, 1), tf[b] @ c2.F)
        assert np.linalg.norm(out["u"][b].cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.all(out["iters"].cpu().numpy() == 2)
    s.close()


@pytest.mark.parametrize("N,Q,prec,tol", [
    (37, 3, "F64", 1e-12), (50, 14, "F64", 1e-12), (64, 50, "F64", 1e-12),
    (37, 3, "F32", 1e-5), (50, 12, "F32", 1e-5), (37, 3, "BF16X3", 1e-5),
    (64, 12, "BF16X3", 1e-5)])
def test_first_step_is_the_stokes_solve(R, N, Q, prec, tol):
    """One Newton step from u = 0 solves A(mu) u = f(mu) (the convection terms of the
    Jacobian vanish there), whatever theta^c. The affine operators are made non-symmetric so
    that a transposed assembly of A(mu) fails; Q = 3 sits in the FP64 contraction's affine
    prefix, Q = 14 and 50 in affine chunks of their own (the mixed precisions take Q <= 12);
    N*N not a multiple of 16 and a ragged batch of 300 leave partial row blocks and request
    groups."""
    rng = np.random.default_rng(N + Q)
    ts = _random_set(N, Q=Q, seed=N, scale=0.1)
    ts.A = ts.A + 0.3 * rng.standard_normal((Q, N, N)) / np.sqrt(N)
    B = 300
    ta = rng.uniform(0.1, 1.0, (B, Q))
    tc = rng.uniform(-1.0, 1.0, (B, ts.Qc))
    tf = rng.standard_normal((B, ts.Qf))
    s = R.Solver(ts)
    th = dict(ta=_dev(ta), tc=_dev(tc), tf=_dev(tf))
    print(f"[first step] N={N} Q={Q} {prec}", flush=True)
    out = s.solve(th, max_iter=1, precision=getattr(R, "RB_PREC_" + prec), refine_steps=0)
    torch.cuda.synchronize()
    u = out["u"].cpu().numpy()
    ref = np.stack([np.linalg.solve(np.tensordot(ta[b], ts.A, 1), tf[b] @ ts.F)
                    for b in range(B)])
    assert np.max(_rel(u, ref)) <= tol
    assert np.all(out["iters"].cpu().numpy() == 1)
    s.close()


# ------------------------------------------------------------- mixed precision ----
# Low-precision Newton (FP32, BF16 or BF16 hi/lo tensors on MFMA, FP32 LU, FP64 iterates)
# followed by refinement steps with the FP64 residual: the result must reach the FP64 oracle
# within 1e-8. BF16x3 does so after a single refinement step.

TOL_MIXED = 1e-8


def _mixed(R, s, th, prec, refine, tol=1e-12, max_iter=10):
    out = s.solve(th, precision=getattr(R, "RB_PREC_" + prec), refine_steps=refine, tol=tol,
                  max_iter=max_iter)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("prec,refine", [("F32", 1), ("BF16", 3), ("BF16X3", 1)])
def test_mixed_precision_parity_ragged(O, R, c2, prec, refine):
    mu = draw_mu(get_config("batched_n50"), 300, seed_offset=11)
    s = R.Solver(c2)
    th = s.theta(_dev(mu))
    g = _mixed(R, s, th, prec, refine)
    r = O.solve_batch(O.OracleSet(c2), mu)
    assert np.all(np.isin(g["status"], (0, 1, 6)))
    err = _rel(g["u"], r["u"])
    assert np.max(err) <= TOL_MIXED, (np.max(err), np.percentile(err, 99))
    s.close()


def test_mixed_refinement_contracts_error(O, R, c2):
    """Each FP64-residual step shrinks the BF16 error by a factor of ten or more (the
    low-precision Jacobian's relative error times the conditioning is well below 0.1)."""
    mu = draw_mu(get_config("batched_n50"), 64, seed_offset=5)
    s = R.Solver(c2)
    th = s.theta(_dev(mu))
    r = O.solve_batch(O.OracleSet(c2), mu)
    errs = [np.max(_rel(_mixed(R, s, th, "BF16", k)["u"], r["u"])) for k in range(4)]
    assert errs[0] <= 1e-2
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 <= 0.1 * e0 or e1 <= 1e-13, errs
    s.close()


def test_mixed_converges_to_fp64_tolerance(O, R, c2):
    mu = draw_mu(get_config("batched_n50"), 100, seed_offset=7)
    s = R.Solver(c2)
    th = s.theta(_dev(mu))
    r = O.solve_batch(O.OracleSet(c2), mu)
    for prec in ("F32", "BF16", "BF16X3"):
        g = _mixed(R, s, th, prec, 12)
        assert np.all(g["status"] == 0), prec
        assert np.max(_rel(g["u"], r["u"])) <= 1e-12, prec
    s.close()


@pytest.mark.parametrize("N", [1, 9, 33, 64])
def test_mixed_random_tensors(O, R, N):
    ts = _random_set(N, seed=100 + N)
    mu = np.column_stack([np.linspace(0.0, 0.6, 21), np.linspace(100, 1000, 21)])
    s = R.Solver(ts)
    th = s.theta(_dev(mu))
    r = O.solve_batch(O.OracleSet(ts), mu, maxit=20)
    for prec, refine in (("F32", 2), ("BF16", 6), ("BF16X3", 2)):
        g = _mixed(R, s, th, prec, refine, max_iter=20)
        assert np.all(np.isin(g["status"], (0, 1, 6))), prec
        assert np.max(_rel(g["u"], r["u"])) <= TOL_MIXED, prec
    s.close()


def test_mixed_status_codes(R, c1):
    s = R.Solver(c1)
    mu = np.tile([[0.2, 300.0]], (3, 1))
    th = s.theta(_dev(mu))
    th["ta"][1].zero_()
    th["tc"][1].zero_()
    th["ta"][2, 0] = float("nan")
    for prec in ("F32", "BF16", "BF16X3"):
        g = _mixed(R, s, th, prec, 2)
        assert list(g["status"][1:]) == [2, 3], prec
        assert list(g["iters"][1:]) == [0, 0], prec
    s.close()


# ------------------------------------------------------------- large bases ---------
# N > 64: one workgroup of ceil(N/64) wavefronts per system (Gauss-Jordan LU), contraction
# tensor parts longer than 64 k-steps in chunks.

@pytest.mark.parametrize("N", [72, 96])
def test_fp64_large_n_random(O, R, N):
    ts = _random_set(N, Qc=4, seed=200 + N)     # Qc*N/4 > 64: chunked Jacobian
    mu = np.column_stack([np.linspace(0.0, 0.6, 21), np.linspace(100, 1000, 21)])
    s = R.Solver(ts)
    th, g = _gpu_solve(R, s, ts, mu, max_iter=20)
    r = O.solve_batch(O.OracleSet(ts), mu, maxit=20, pressure_np=ts.Np)
    assert np.array_equal(g["status"], r["status"]) and np.all(g["status"] == 0)
    assert np.max(_rel(g["u"], r["u"])) <= TOL_F64
    p = s.pressure(th, torch.as_tensor(g["u"]).cuda())
    torch.cuda.synchronize()
    assert np.max(_rel(p["p"].cpu().numpy(), r["p"])) <= TOL_F64
    s.close()


@pytest.mark.parametrize("N", [65, 100, 130, 152])
def test_mixed_large_n_random(O, R, N):
    ts = _random_set(N, Qc=4, seed=300 + N)
    mu = np.column_stack([np.linspace(0.0, 0.6, 21), np.linspace(100, 1000, 21)])
    s = R.Solver(ts)
    th = s.theta(_dev(mu))
    r = O.solve_batch(O.OracleSet(ts), mu, maxit=20)
    for prec, refine in (("F32", 2), ("BF16", 6), ("BF16X3", 2)):
        g = _mixed(R, s, th, prec, refine, max_iter=20)
        assert np.all(np.isin(g["status"], (0, 1, 6))), prec
        assert np.max(_rel(g["u"], r["u"])) <= TOL_MIXED, prec
    s.close()


@pytest.mark.parametrize("cfg_name,prec,refine", [("mixed_n100", "BF16", 3),
                                                  ("mixed_n100", "BF16X3", 1),
                                                  ("serve_n150", "F32", 1)])
def test_mixed_large_configs_sampled(O, R, cfg_name, prec, refine):
    """The synthetic N = 100 / N = 150 sets: ragged batch of 70 requests against the oracle,
    velocity and pressure."""
    cfg = get_config(cfg_name)
    ts = make_tensor_set(cfg)
    mu = draw_mu(cfg, 70)
    s = R.Solver(ts)
    th = s.theta(_dev(mu))
    g = _mixed(R, s, th, prec, refine)
    r = O.solve_batch(O.OracleSet(ts), mu, pressure_np=ts.Np)
    assert np.all(np.isin(g["status"], (0, 1, 6)))
    assert np.max(_rel(g["u"], r["u"])) <= TOL_MIXED
    p = s.pressure(th, torch.as_tensor(g["u"]).cuda())
    torch.cuda.synchronize()
    assert np.all(p["pstatus"].cpu().numpy() == 0)
    assert np.max(_rel(p["p"].cpu().numpy(), r["p"])) <= TOL_MIXED
    s.close()


def test_fp64_beyond_limit_is_unsupported(R):
    ts = _random_set(100, seed=1)
    s = R.Solver(ts)
    th = s.theta(_dev(np.array([[0.1, 200.0]])))
    with pytest.raises(R.RbError) as e:
        s.solve(th)
    assert e.value.code == R.RB_E_UNSUPPORTED
    g = _mixed(R, s, th, "F32", 2)
    assert g["status"][0] <= 1
    s.close()


# ------------------------------------------------------------- statuses and errors ---

def test_status_codes_forced_from_host(R, c1):
    s = R.Solver(c1)
    mu = np.tile([[0.2, 300.0]], (4, 1))
    th = s.theta(_dev(mu))
    th["ta"][1].zero_()
    th["tc"][1].zero_()                         # A(mu) = 0, C = 0: zero pivot
    th["ta"][2, 0] = float("nan")               # non-finite operand
    out = s.solve(th, max_iter=1)               # request 0, 3: iteration limit
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert list(st) == [1, 2, 3, 1]
    assert list(out["iters"].cpu().numpy()) == [1, 0, 0, 1]
    s.close()


@pytest.mark.parametrize("N,prec", [(50, "F64"), (72, "F64"), (40, "F32"), (100, "F32")])
def test_zero_pivot_status_every_solve(R, N, prec):
    """Zero pivots in the one-wavefront solves (N = 50 FP64, N = 40 FP32) and the workgroup
    solves (N = 72 FP64, N = 100 FP32): with the last column of every A_q zero, the first
    Jacobian A(mu) meets an exact zero pivot at the last elimination step (requests 0 and
    2); with theta^a = 0 it is zero and does so at the first (request 1). Every request
    reports RB_ST_SINGULAR (2) after no completed iteration."""
    rng = np.random.default_rng(N)
    ts = _random_set(N, seed=N)
    ts.A = ts.A.copy()
    ts.A[:, :, N - 1] = 0.0
    B = 3
    ta = rng.uniform(0.1, 1.0, (B, ts.Q))
    ta[1] = 0.0
    tc = rng.uniform(-1.0, 1.0, (B, ts.Qc))
    tf = rng.standard_normal((B, ts.Qf))
    s = R.Solver(ts)
    print(f"[zero pivot] N={N} {prec}", flush=True)
    out = s.solve(dict(ta=_dev(ta), tc=_dev(tc), tf=_dev(tf)),
                  precision=getattr(R, "RB_PREC_" + prec), refine_steps=1)
    torch.cuda.synchronize()
    assert list(out["status"].cpu().numpy()) == [2, 2, 2]
    assert list(out["iters"].cpu().numpy()) == [0, 0, 0]
    s.close()


def test_call_level_errors(R, c1):
    s = R.Solver(c1)
    th = s.theta(_dev(np.array([[0.1, 200.0]])))
    with pytest.raises(R.RbError) as e:
        s.solve(th, N=11)
    assert e.value.code == R.RB_E_INVAL
    with pytest.raises(R.RbError):
        s.solve(th, N=0)
    with pytest.raises(R.RbError):
        s.solve(th, max_iter=0)
    with pytest.raises(R.RbError) as e:
        s.solve(th, precision=7)
    assert e.value.code in (R.RB_E_INVAL, R.RB_E_UNSUPPORTED)
    # B == 0 is a no-op
    R.rb_solve_batch(s.ctx, s.set, 0, 10, 10, None, None, None, None, None, None, None,
                     None, None)
    s.close()


def test_hbm_budget_rejects_oversized_load(R, c2):
    ctx = R.rb_create(0, 1 << 20)
    with pytest.raises(R.RbError) as e:
        R.rb_load_tensors(ctx, c2)
    assert e.value.code == R.RB_E_NOMEM
    assert R.rb_hbm_used(ctx) == 0
    R.rb_destroy(ctx)


@pytest.mark.parametrize("N,Np", [(7, 5), (15, 15), (16, 17), (31, 30), (50, 33), (63, 47)])
def test_lu_variants_agree(O, R, N, Np, monkeypatch):
    """The three FP64 solve variants (one row per lane with readlane or LDS broadcast, and the
    matrix-core panel solve) on the same batch: each within the FP64 tolerance of the oracle,
    for the Newton iterates and the recovered pressure; statuses identical. Sizes cover one to
    four 16-wide tiles, a system filling all but the right-hand-side column (N = 63), and a
    ragged batch (B = 70: one full wavefront group and a tail)."""
    ts = _random_set(N, Np=Np, seed=100 + N)
    mu = np.column_stack([np.linspace(0.0, 0.6, 70), np.linspace(100, 1000, 70)])
    r = O.solve_batch(O.OracleSet(ts), mu, maxit=20, pressure_np=ts.Np)
    for variant in ("readlane", "lds", "mfma"):
        monkeypatch.setenv("RB_LU", variant)
        s = R.Solver(ts)
        th, g = _gpu_solve(R, s, ts, mu, max_iter=20)
        assert np.array_equal(g["status"], r["status"]) and np.all(g["status"] == 0), variant
        assert np.max(_rel(g["u"], r["u"])) <= TOL_F64, variant
        p = s.pressure(th, torch.as_tensor(g["u"]).cuda())
        torch.cuda.synchronize()
        assert np.all(p["pstatus"].cpu().numpy() == 0), variant
        assert np.max(_rel(p["p"].cpu().numpy(), r["p"])) <= TOL_F64, variant
        s.close()


@pytest.fixture(scope="module")
def c50q():
    return make_tensor_set(get_config("batched_n50_q50"))


@pytest.mark.parametrize("B,N", [(300, 50), (70, 20), (4096, 50)])
def test_paper_shaped_term_counts(O, R, c50q, B, N):
    """Q = 50 affine terms of a and Qc = 49 of c (the Piola expansions at n = 12, powers of
    the angle): K = Q + Qc N = 2500 at N = 50, the affine part in its own chunk of the
    contraction and the tensor part in 16 more. Velocity and pressure within 1e-10 of the
    oracle on a sample of the batch (the whole batch up to 300 requests), statuses equal."""
    cfg = get_config("batched_n50_q50")
    mu = draw_mu(cfg, B, seed_offset=B + N)
    s = R.Solver(c50q)
    th, g = _gpu_solve(R, s, c50q, mu, N=N)
    p = s.pressure(th, torch.as_tensor(g["u"]).cuda(), N=N)
    torch.cuda.synchronize()
    idx = np.arange(B) if B <= 300 else np.linspace(0, B - 1, 48).astype(int)
    ts = c50q.leading(N)
    r = O.solve_batch(O.OracleSet(ts), mu[idx], pressure_np=ts.Np)
    assert np.array_equal(g["status"][idx], r["status"]) and np.all(g["status"] == 0)
    assert np.max(_rel(g["u"][idx, :N], r["u"])) <= TOL_F64
    assert np.max(_rel(p["p"].cpu().numpy()[idx], r["p"])) <= TOL_F64
    s.close()


def test_paper_shaped_terms_fp64_only(R, c50q):
    s = R.Solver(c50q)
    th = s.theta(_dev(draw_mu(get_config("batched_n50_q50"), 4)))
    with pytest.raises(R.RbError) as e:
        s.solve(th, precision=R.RB_PREC_F32)
    assert e.value.code == R.RB_E_UNSUPPORTED
    s.close()


def test_theta_power_families_on_gpu(O, R, c50q):
    mu = draw_mu(get_config("batched_n50_q50"), 33)
    s = R.Solver(c50q)
    th = s.theta(_dev(mu))
    torch.cuda.synchronize()
    for b in range(33):
        ta, tc, tf, tb = O.theta(c50q.Q, c50q.Qc, c50q.Qf, c50q.Qb, mu[b, 0], mu[b, 1])
        for k, ref in (("ta", ta), ("tc", tc), ("tf", tf), ("tb", tb)):
            got = th[k][b].cpu().numpy()
            assert np.allclose(got, ref, rtol=4e-16 * 60, atol=0), (k, b)
    s.close()


@pytest.mark.parametrize("prec,refine", [("BF16X3", 1), ("BF16", 3)])
def test_mixed_n100_full_batch_sampled(O, R, prec, refine):
    """Config 4 at full size: B = 32768 at N = 100 (Q = 12, Qc = 4), BF16 hi/lo or plain BF16
    tensors on MFMA, FP32 LU, FP64-residual refinement, in the launch configuration of the
    bench (8 row splits per tile); velocity and pressure on a seeded sample of 256 requests
    within 1e-8 of the oracle."""
    cfg = get_config("mixed_n100")
    ts = make_tensor_set(cfg)
    B = cfg["B"]
    mu = draw_mu(cfg, B)
    s = R.Solver(ts)
    th = s.theta(_dev(mu))
    print(f"[mixed full] {prec} + {refine}", flush=True)
    g = _mixed(R, s, th, prec, refine)
    p = s.pressure(th, torch.as_tensor(g["u"]).cuda())
    torch.cuda.synchronize()
    pick = np.random.default_rng(11).choice(B, 256, replace=False)
    r = O.solve_batch(O.OracleSet(ts), mu[pick], pressure_np=ts.Np)
    assert np.all(np.isin(g["status"], (0, 1, 6)))
    assert np.max(_rel(g["u"][pick], r["u"])) <= TOL_MIXED
    assert np.all(p["pstatus"].cpu().numpy() == 0)
    assert np.max(_rel(p["p"].cpu().numpy()[pick], r["p"])) <= TOL_MIXED
    s.close()
