"""Pressure parts of a combined velocity-pressure basis (the offline step of the pressure
reconstruction of Section 4.2).

TEST INFRASTRUCTURE ONLY. The paper's second construction of a combined basis builds the
velocity basis as usual and gives each velocity function a pressure part made of the same
snapshot combination: if phi_i = sum_j v_i^j u(mu_j) (eqn uRj), its pressure part is
psi_i = sum_j v_i^j p(mu_j) (eqn pRj). The synthetic velocity basis is not a snapshot POD,
so the coefficients v are taken as the minimum-norm ones that express the basis in the
snapshots: with U [N][K] the velocity coefficients and P [Np][K] the recovered pressure
coefficients of K training solutions, V = pinv(U) (U V = I when the K snapshots span the
basis) and the pressure parts have pressure-basis coefficients
    Pc = P V = P pinv(U)      ([Np][N]),
the least-squares map from velocity to pressure coefficients over the training set. The
training solutions come from the oracle's Newton solve and pressure recovery on a tensor
grid of Gauss-Legendre points in (alpha, Re), as the paper's ensemble is a 15 x 15 Gauss
grid of its two parameters.
"""

from __future__ import annotations

import numpy as np

from rbinputs.synth import gauss_grid_mu

from . import oracle as O


def gauss_grid(cfg, n=15):
    """The training parameters: n x n Gauss-Legendre points of (alpha, Re)."""
    return gauss_grid_mu(cfg, n)


def training_solutions(ts, mu, N=None, Np=None):
    """Velocity [K][N] and recovered pressure [K][Np] coefficients of the training set."""
    N = ts.N if N is None else N
    Np = ts.Np if Np is None else Np
    r = O.solve_batch(O.OracleSet(ts), mu, Nreq=np.full(len(mu), N, np.int32), pressure_np=Np)
    if not (np.all(r["status"] == 0) and np.all(r["pstatus"] == 0)):
        raise RuntimeError("training solve failed")
    return r["u"][:, :N], r["p"][:, :Np]


def pressure_map(U, P):
    """Pc = P^T pinv(U^T) from training rows U [K][N], P [K][Np]: returns [Np][N]. Singular
    values of U below 1e-8 of the largest are dropped (the training solutions of a
    parameter family with few affine terms span fewer than N directions)."""
    return P.T @ np.linalg.pinv(U.T, rcond=1e-8)
