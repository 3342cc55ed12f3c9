"""GPU parity of uneven batches (requests of mixed basis size N in one call) and the autotuner.

Each uneven result is compared with the FP64 oracle at the request's own N (1e-10 on the FP64
path, 1e-8 after mixed-precision refinement) and with the same request solved in a same-N
batch (1e-12: the two differ only in the order of floating-point sums when the tile shapes
differ). The same shape is solved five times with other parameters and eager work between
the calls, so the plain, capturing and replaying paths are all covered and every replay is
checked.
"""

import numpy as np
import pytest

from rbinputs import get_config, make_tensor_set, draw_mu, draw_basis_sizes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rel(a, b):
    nb = np.linalg.norm(b, axis=-1)
    return np.linalg.norm(a - b, axis=-1) / np.where(nb > 0, nb, 1)


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_11866_amd import rbns
    rbns.load()
    return rbns


@pytest.fixture(scope="module")
def c3():
    return make_tensor_set(get_config("uneven_n20_100"))


@pytest.fixture(scope="module")
def c2():
    return make_tensor_set(get_config("batched_n50"))


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def _uneven(R, s, th, Nreq, **kw):
    out = s.solve_uneven(th, _dev(Nreq, torch.int32), **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _oracle_per_request(O, ts, mu, Nreq, **kw):
    return O.solve_batch(O.OracleSet(ts), mu, Nreq=np.asarray(Nreq, np.int32), **kw)


def test_uneven_fp32_three_calls_same_shape(oracle_lib, R, c3):
    """Config 3's mix (N in {20,...,100}, FP32 storage and contraction, refinement): a ragged
    batch of 700 requests, three calls with different parameters and the same group sizes."""
    O = oracle_lib
    cfg = get_config("uneven_n20_100")
    Nreq = draw_basis_sizes(cfg, 700)
    s = R.Solver(c3)
    for call in range(5):                 # plain, capture + replay, then replays
        mu = draw_mu(cfg, 700, seed_offset=call)
        th = s.theta(_dev(mu))
        g = _uneven(R, s, th, Nreq, precision=R.RB_PREC_F32, refine_steps=2)
        r = _oracle_per_request(O, c3, mu, Nreq)
        err = _rel(g["u"], r["u"])
        print(call, {int(n): (np.bincount(g["status"][Nreq == n], minlength=2).tolist(),
                              float(np.max(err[Nreq == n]))) for n in np.unique(Nreq)})
        assert np.all(np.isin(g["status"], (0, 1, 6))), (call, np.bincount(g["status"]))
        assert np.max(err) <= 1e-8, (call, np.max(err))
        for b in range(0, 700, 97):                 # zero beyond each request's own N
            assert not np.any(g["u"][b, Nreq[b]:])
        # eager work on the same stream between the graph replays
        s.solve(s.theta(_dev(mu[:50])), N=20, precision=R.RB_PREC_F32, refine_steps=1)
        torch.cuda.synchronize()
    # the same requests in same-N batches
    for n in np.unique(Nreq):
        idx = np.nonzero(Nreq == n)[0]
        thn = {k: v[torch.as_tensor(idx, device="cuda")] for k, v in th.items() if v is not None}
        out = s.solve(thn, N=int(n), precision=R.RB_PREC_F32, refine_steps=2)
        torch.cuda.synchronize()
        assert np.max(_rel(g["u"][idx], out["u"].cpu().numpy())) <= 1e-12
    s.close()


def test_uneven_fp64_matches_oracle(oracle_lib, R, c2):
    O = oracle_lib
    cfg = get_config("batched_n50")
    rng = np.random.default_rng(4)
    Nreq = rng.choice(np.array([1, 8, 30, 50], np.int32), size=333)
    mu = draw_mu(cfg, 333, seed_offset=9)
    s = R.Solver(c2)
    th = s.theta(_dev(mu))
    r = _oracle_per_request(O, c2, mu, Nreq)
    for call in range(3):
        g = _uneven(R, s, th, Nreq)
        assert np.array_equal(g["status"], r["status"]) and np.all(g["status"] == 0)
        assert np.max(_rel(g["u"], r["u"])) <= 1e-10
    s.close()


def test_uneven_pressure_matches_oracle(oracle_lib, R, c2):
    """Velocity and pressure of a mixed-N batch, each request at its own N."""
    O = oracle_lib
    cfg = get_config("batched_n50")
    rng = np.random.default_rng(8)
    Nreq = rng.choice(np.array([3, 17, 30, 50], np.int32), size=261)
    Nreq[5] = 0                                     # invalid size: status 4, p = 0
    mu = draw_mu(cfg, 261, seed_offset=12)
    s = R.Solver(c2)
    th = s.theta(_dev(mu))
    Nd = _dev(Nreq, torch.int32)
    out = s.solve_uneven(th, Nd)
    pr = s.pressure_uneven(th, out["u"], Nd)
    torch.cuda.synchronize()
    ok = Nreq > 0
    r = O.solve_batch(O.OracleSet(c2), mu[ok], Nreq=Nreq[ok], pressure_np=c2.Np)
    ps = pr["pstatus"].cpu().numpy()
    pg = pr["p"].cpu().numpy()
    assert ps[5] == R.RB_ST_BADN and not np.any(pg[5])
    assert np.all(ps[ok] == 0)
    assert np.max(_rel(pg[ok], r["p"])) <= 1e-10
    # the same requests through the same-N entry point
    for n in (17, 50):
        idx = np.nonzero(Nreq == n)[0]
        sel = torch.as_tensor(idx, device="cuda")
        thn = {k: v[sel] for k, v in th.items() if v is not None}
        p1 = s.pressure(thn, out["u"][sel], N=n)
        torch.cuda.synchronize()
        assert np.max(_rel(pg[idx], p1["p"].cpu().numpy())) <= 1e-13
    s.close()


def test_uneven_bad_sizes_and_empty_groups(R, c2):
    cfg = get_config("batched_n50")
    Nreq = np.array([50, 0, -3, 51, 20, 50], np.int32)
    mu = draw_mu(cfg, 6)
    s = R.Solver(c2)
    th = s.theta(_dev(mu))
    g = _uneven(R, s, th, Nreq)
    assert list(g["status"]) == [0, 4, 4, 4, 0, 0]
    assert list(g["iters"][1:4]) == [0, 0, 0]
    assert not np.any(g["u"][1:4])
    s.close()


def test_uneven_argument_errors(R, c2):
    s = R.Solver(c2)
    th = s.theta(_dev(draw_mu(get_config("batched_n50"), 2)))
    Nd = _dev(np.array([10, 20], np.int32), torch.int32)
    out = dict(u=torch.empty(2, 40, dtype=torch.float64, device="cuda"),
               iters=torch.empty(2, dtype=torch.int32, device="cuda"),
               status=torch.empty(2, dtype=torch.int32, device="cuda"))
    with pytest.raises(R.RbError) as e:                     # ldu below the set's N
        R.rb_solve_uneven(s.ctx, s.set, 2, Nd, 40, th["ta"], th["tc"], th["tf"], None, None,
                          R.make_opts(), out["u"], out["iters"], out["status"])
    assert e.value.code == R.RB_E_INVAL
    s.close()


def test_autotune_choice_is_used_and_exact(oracle_lib, R, c2):
    O = oracle_lib
    mu = draw_mu(get_config("batched_n50"), 512, seed_offset=21)
    s = R.Solver(c2)
    th = s.theta(_dev(mu))
    ns, lv = s.autotune(th)
    assert 1 <= ns <= 64 and lv in (0, 1)
    assert R.rb_tuned_config(s.ctx, s.set, 50, R.RB_PREC_F64, 512) == (ns, lv)
    out = s.solve(th)
    torch.cuda.synchronize()
    r = O.solve_batch(O.OracleSet(c2), mu)
    assert np.all(out["status"].cpu().numpy() == 0)
    assert np.max(_rel(out["u"].cpu().numpy(), r["u"])) <= 1e-10
    s.close()


def test_uneven_full_size_fresh_mix_then_replay(oracle_lib, R, c3):
    """Config 3 at full size: 16384 requests, N in {20,...,100}, FP32 + two refinement steps.
    A fresh random N mix runs as plain launches, the same mix again is captured and then
    replayed; each call is checked on a sample of 256 requests against the oracle (1e-8)."""
    O = oracle_lib
    cfg = get_config("uneven_n20_100")
    B = 16384
    Nreq = draw_basis_sizes(cfg, B, seed_offset=77)          # not the bench's mix
    s = R.Solver(c3)
    pick = np.random.default_rng(5).choice(B, 256, replace=False)
    for call in range(3):                                  # eager, capture + replay, replay
        mu = draw_mu(cfg, B, seed_offset=100 + call)
        th = s.theta(_dev(mu))
        print(f"[uneven full] call {call}", flush=True)
        g = _uneven(R, s, th, Nreq, precision=R.RB_PREC_F32, refine_steps=2)
        assert np.all(np.isin(g["status"], (0, 1, 6))), (call, np.bincount(g["status"]))
        r = _oracle_per_request(O, c3, mu[pick], Nreq[pick])
        assert np.max(_rel(g["u"][pick], r["u"])) <= 1e-8, call
    s.close()
