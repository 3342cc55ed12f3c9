"""Choose the body-force amplitude of a synthetic tensor set (input calibration).

TEST INFRASTRUCTURE ONLY. Prints, per configuration, the ``forcing_scale`` that makes the
small-data uniqueness number

    rho(mu) = gamma(mu) * ||f(mu)||_{A(mu)^-1}

equal to ``target`` at the worst parameter of a sample grid. With A(mu) = L L^T (Cholesky),
gamma(mu) is the Frobenius norm of the scaled tensor
    Ct[i,j,k] = sum_abc Linv[i,a] C(mu)[a,b,c] Linv[j,b] Linv[k,c],
which bounds |Ct(v,w)| <= gamma |v| |w|. Because every C_q is skew in its test and advected
indices (c(u,v,v) = 0 for solenoidal u), a root u satisfies ||u||_A <= ||f||_{A^-1}, and for
rho < 1 the root is unique (the standard small-data argument for steady Navier-Stokes).

The theta functions come from the oracle; nothing here comes from the GPU library. Run:
    python -m oracle.calibrate_forcing [config ...]
and copy the printed values into ``rbinputs/configs.py``.
"""

from __future__ import annotations

import sys

import numpy as np

from rbinputs import get_config, make_tensor_set
from . import oracle as O


def rho_grid(ts, cfg, na=8, nr=8):
    alphas = np.deg2rad(np.linspace(*cfg["alpha_deg"], na))
    res = np.linspace(*cfg["Re"], nr)
    if "fixed_mu" in cfg:
        alphas = np.array([np.deg2rad(cfg["fixed_mu"][0])])
        res = np.array([cfg["fixed_mu"][1]])
    out = []
    for a in alphas:
        for re in res:
            ta, tc, tf, tb = O.theta(ts.Q, ts.Qc, ts.Qf, ts.Qb, a, re)
            Am = np.tensordot(ta, ts.A, 1)
            Cm = np.tensordot(tc, ts.C, 1)
            f = tf @ ts.F
            L = np.linalg.cholesky(Am)
            Li = np.linalg.inv(L)
            Ct = np.einsum("ia,abc,jb,kc->ijk", Li, Cm, Li, Li, optimize=True)
            gamma = np.linalg.norm(Ct.ravel())
            fn = np.linalg.norm(Li @ f)
            out.append(gamma * fn)
    return np.array(out)


def calibrate(name, target=0.5):
    cfg = get_config(name, forcing_scale=1.0)
    ts = make_tensor_set(cfg)
    r = rho_grid(ts, cfg)
    return target / r.max(), r.max()


if __name__ == "__main__":
    names = sys.argv[1:] or ["single_n10", "batched_n50", "uneven_n20_100", "mixed_n100",
                             "serve_n150"]
    for nm in names:
        s, r1 = calibrate(nm)
        print(f"{nm}: forcing_scale = {s:.6g}   (rho at scale 1: {r1:.4g})", flush=True)
