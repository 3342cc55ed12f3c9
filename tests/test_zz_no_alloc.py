"""The allocation-free solve (rb_solve_batch_noalloc) against rb_solve_batch, through the C ABI.

The variant keeps the Newton state in the library's static device array instead of a
per-stream workspace; it runs the same kernels with the same tile shapes, so its results must
equal rb_solve_batch's bit for bit. Two calls in a row, the second smaller, show that nothing
left in the shared array by the first call leaks into the second. The FP64 results are also
checked against the oracle at the FP64 path's tolerance (1e-10 relative per request).
"""

import numpy as np
import pytest

from rbinputs import draw_mu, get_config, make_tensor_set

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_11866_amd import rbns
    rbns.load()
    return rbns


@pytest.fixture(scope="module")
def c2():
    return make_tensor_set(get_config("batched_n50"))


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def _solve_both(R, ctx, sid, ts, mu, N, opts):
    B = mu.shape[0]
    th = [torch.empty((B, q), dtype=torch.float64, device="cuda")
          for q in (ts.Q, ts.Qc, ts.Qf, ts.Qb)]
    R.rb_theta(ctx, sid, B, _dev(mu), *th)
    out = {}
    for name, fn in (("batch", R.rb_solve_batch), ("noalloc", R.rb_solve_batch_noalloc)):
        u = torch.full((B, N), np.nan, dtype=torch.float64, device="cuda")
        it = torch.full((B,), -7, dtype=torch.int32, device="cuda")
        st = torch.full((B,), -7, dtype=torch.int32, device="cuda")
        print(f"[no-alloc] {name} B={B} N={N} precision={opts.precision}", flush=True)
        fn(ctx, sid, B, N, N, th[0], th[1], th[2], None, None, opts, u, it, st)
        torch.cuda.synchronize()
        out[name] = (u.cpu().numpy(), it.cpu().numpy(), st.cpu().numpy())
    return out


def test_noalloc_equals_solve_batch_fp64_two_calls(R, c2, oracle_lib):
    O = oracle_lib
    ctx = R.rb_create(0)
    try:
        sid = R.rb_load_tensors(ctx, c2)
        opts = R.make_opts()
        cfg = get_config("batched_n50")
        for B in (700, 130):                       # the second call is smaller
            mu = draw_mu(cfg, B, seed_offset=B)
            out = _solve_both(R, ctx, sid, c2, mu, 50, opts)
            ub, ib, sb = out["batch"]
            un, in_, sn = out["noalloc"]
            assert np.array_equal(un, ub)
            assert np.array_equal(in_, ib) and np.array_equal(sn, sb)
            assert np.all(sn == 0)
            pick = np.random.default_rng(B).choice(B, 12, replace=False)
            r = O.solve_batch(O.OracleSet(c2), mu[pick])
            err = np.linalg.norm(un[pick] - r["u"], axis=1) / np.linalg.norm(r["u"], axis=1)
            assert err.max() <= 1e-10
    finally:
        R.rb_destroy(ctx)


def test_noalloc_equals_solve_batch_mixed_precision(R, c2):
    ctx = R.rb_create(0)
    try:
        sid = R.rb_load_tensors(ctx, c2)
        cfg = get_config("batched_n50")
        for prec, N, B in ((R.RB_PREC_BF16X3, 40, 300), (R.RB_PREC_F32, 40, 70)):
            opts = R.make_opts(precision=prec, refine_steps=2)
            mu = draw_mu(cfg, B, seed_offset=3 * B)
            out = _solve_both(R, ctx, sid, c2, mu, N, opts)
            for x, y in zip(out["noalloc"], out["batch"]):
                assert np.array_equal(x, y)
    finally:
        R.rb_destroy(ctx)


def test_noalloc_call_errors(R, c2):
    ctx = R.rb_create(0)
    try:
        sid = R.rb_load_tensors(ctx, c2)
        opts = R.make_opts()
        cfg = get_config("batched_n50")
        # no packed operand yet for N = 30: the allocation-free call refuses to build one
        mu = draw_mu(cfg, 8)
        th = [torch.empty((8, q), dtype=torch.float64, device="cuda")
              for q in (c2.Q, c2.Qc, c2.Qf, c2.Qb)]
        R.rb_theta(ctx, sid, 8, _dev(mu), *th)
        u = torch.empty((8, 50), dtype=torch.float64, device="cuda")
        it = torch.empty(8, dtype=torch.int32, device="cuda")
        st = torch.empty(8, dtype=torch.int32, device="cuda")
        with pytest.raises(R.RbError) as e:
            R.rb_solve_batch_noalloc(ctx, sid, 8, 30, 50, th[0], th[1], th[2], None, None,
                                     opts, u, it, st)
        assert e.value.code == R.RB_E_STATE
        # a batch whose state exceeds the device array: rejected before any launch
        B = 4096
        big = [torch.zeros((B, q), dtype=torch.float64, device="cuda")
               for q in (c2.Q, c2.Qc, c2.Qf)]
        ub = torch.empty((B, 50), dtype=torch.float64, device="cuda")
        ib = torch.empty(B, dtype=torch.int32, device="cuda")
        with pytest.raises(R.RbError) as e:
            R.rb_solve_batch_noalloc(ctx, sid, B, 50, 50, big[0], big[1], big[2], None, None,
                                     opts, ub, ib, ib)
        assert e.value.code == R.RB_E_NOMEM and "scratch" in str(e.value)
        torch.cuda.synchronize()
    finally:
        R.rb_destroy(ctx)
