"""GPU tests of the continuous-batching server (rb_server_*).

A request's result must not depend on the batch it was served in: the same request is
served alone and in the middle of a stream of other requests of mixed basis size, and the
two results must agree bit for bit (each request's arithmetic is independent of the other
columns of its tile, and a served group's tile shapes depend on its N alone, never on the
batch size). Every result is also checked against the FP64 oracle at the request's own N.
"""

import time

import numpy as np
import pytest

from rbinputs import get_config, make_tensor_set, draw_mu, draw_basis_sizes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_11866_amd import rbns
    rbns.load()
    return rbns


def _collect(srv, n, timeout=60.0):
    got = {}
    t0 = time.time()
    while len(got) < n:
        for r in srv.poll():
            got[r["ticket"]] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(got)} of {n} results after {timeout} s")
        time.sleep(0.001)
    return got


def _alone_and_in_mix(R, O, ts, cfg, prec, refine, tol_u, pressure, max_batch=256, lanes=3,
                      burst=50):
    s = R.Solver(ts)
    srv = R.Server(s, precision=prec, refine_steps=refine, max_batch=max_batch, lanes=lanes,
                   pressure=pressure)
    try:
        mu = draw_mu(cfg, 600, seed_offset=31)
        Nreq = draw_basis_sizes(cfg, 600, seed_offset=31)
        x = 300                                           # the request served twice
        t_alone = srv.submit(mu[x, 0], mu[x, 1], Nreq[x], tags=[-1])
        alone = _collect(srv, 1)[t_alone[0]]
        tickets = []
        for k in range(0, 600, burst):                    # arrivals in bursts
            tickets.extend(srv.submit(mu[k:k + burst, 0], mu[k:k + burst, 1],
                                      Nreq[k:k + burst], tags=np.arange(k, k + burst)))
            time.sleep(0.0005)
        got = _collect(srv, 600)
        mix = got[tickets[x]]
        assert alone["status"] == mix["status"] and alone["iters"] == mix["iters"]
        assert np.array_equal(alone["u"], mix["u"])
        if pressure:
            assert np.array_equal(alone["p"], mix["p"])
        st = srv.stats()
        assert st["completed"] == 601 and st["submitted"] == 601 and st["error"] == ""
        assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"] * 1.006
        assert 0 <= st["p50_queue_ms"] <= st["p99_queue_ms"] <= st["p99_ms"] * 1.006
        assert st["batches"] >= 2                         # the stream was batched, not queued whole
        # every result against the oracle at its own N
        r = O.solve_batch(O.OracleSet(ts), mu, Nreq=Nreq, pressure_np=ts.Np if pressure else 0)
        for b, t in enumerate(tickets):
            g = got[t]
            assert g["tag"] == b and g["N"] == Nreq[b]
            assert g["status"] in (0, 1, 6), (b, g["status"])
            assert _rel(g["u"], r["u"][b, :Nreq[b]]) <= tol_u, b
            if pressure:
                assert g["pstatus"] == 0
                assert _rel(g["p"][:ts.Np], r["p"][b]) <= tol_u, b
    finally:
        srv.stop()
        s.close()


def test_server_fp64_alone_equals_in_mix(oracle_lib, R):
    cfg = dict(get_config("batched_n50"), N_choices=(10, 25, 40, 50))
    ts = make_tensor_set(get_config("batched_n50"))
    _alone_and_in_mix(R, oracle_lib, ts, cfg, R.RB_PREC_F64, 0, 1e-10, pressure=True)


def test_server_fp64_alone_equals_in_large_mixed_batch(oracle_lib, R):
    """One burst of 600 requests with max_batch 4096: every size-class group of the batch
    holds more than 64 requests (several tiles), where the default row split of a one-off
    batch would differ from a lone request's; the served result must still be identical."""
    cfg = dict(get_config("batched_n50"), N_choices=(10, 25, 40, 50))
    ts = make_tensor_set(get_config("batched_n50"))
    _alone_and_in_mix(R, oracle_lib, ts, cfg, R.RB_PREC_F64, 0, 1e-10, pressure=True,
                      max_batch=4096, lanes=1, burst=600)


@pytest.mark.parametrize("prec,refine", [("BF16", 4), ("BF16X3", 1)])
def test_server_bf16_serving_set(oracle_lib, R, prec, refine):
    cfg = get_config("serve_n150")
    ts = make_tensor_set(cfg)
    _alone_and_in_mix(R, oracle_lib, ts, cfg, getattr(R, "RB_PREC_" + prec), refine, 1e-8,
                      pressure=False)


def test_server_budget_cuts_batches(R):
    cfg = get_config("batched_n50")
    ts = make_tensor_set(cfg)
    s = R.Solver(ts)
    mu = draw_mu(cfg, 512)
    budget = 4 << 20                     # ~ 2.6 MB per 128 requests at N = 50 (J, state)
    srv = R.Server(s, max_batch=512, lanes=2, hbm_budget_bytes=budget)
    try:
        t = srv.submit(mu[:, 0], mu[:, 1], 50)
        got = _collect(srv, 512)
        assert all(got[k]["status"] == 0 for k in t)
        st = srv.stats()
        assert st["batches"] > 1 and st["hbm_inflight_peak"] <= budget
    finally:
        srv.stop()
        s.close()


def test_server_bad_size_and_stop_drains(R):
    cfg = get_config("batched_n50")
    ts = make_tensor_set(cfg)
    s = R.Solver(ts)
    srv = R.Server(s)
    t = srv.submit([0.1, 0.2, 0.3], [200.0, 300.0, 400.0], [0, 50, 51])
    got = _collect(srv, 3)
    assert [got[k]["status"] for k in t] == [R.RB_ST_BADN, 0, R.RB_ST_BADN]
    srv.submit(np.full(100, 0.2), 500.0, 30)
    srv.stop()                                            # drains the queue before returning
    with pytest.raises(R.RbError):
        R.Server(s, lanes=17)
    s.close()


def test_server_burst_batches_by_class(R, oracle_lib):
    """A burst of 10000 requests in four size classes (N = 10, 25, 40, 50: classes 16, 32,
    48, 50), queued in one submission and served by one lane with max_batch 1000: every batch
    holds one class, so the server runs sum over classes of ceil(n_c / 1000) = 12 batches
    (ten if batches mixed classes), every request converges, and a sample agrees with the
    oracle at its own N."""
    O = oracle_lib
    cfg = get_config("batched_n50")
    ts = make_tensor_set(cfg)
    s = R.Solver(ts)
    rng = np.random.default_rng(5)
    n = 10000
    Ns = np.repeat(np.array([10, 25, 40, 50]), n // 4)
    rng.shuffle(Ns)
    mu = draw_mu(cfg, n, seed_offset=9)
    srv = R.Server(s, max_batch=1000, lanes=1)
    try:
        t = srv.submit(mu[:, 0], mu[:, 1], Ns)
        got = _collect(srv, n, timeout=120.0)
        assert all(got[k]["status"] == 0 for k in t)
        assert srv.stats()["batches"] == 12
        pick = rng.choice(n, 8, replace=False)
        r = O.solve_batch(O.OracleSet(ts), mu[pick], Nreq=Ns[pick])
        for m, i in enumerate(pick):
            assert _rel(got[t[i]]["u"], r["u"][m, :Ns[i]]) <= 1e-10, i
    finally:
        srv.stop()
        s.close()
