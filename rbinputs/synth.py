"""Synthetic reduced-basis tensor sets on the unit periodic square.

The paper's offline stage (Sections 3.1-3.5 and 4.1) produces a solenoidal reduced velocity
basis, a pressure basis, supremizers (Riesz representers of the pressure functionals, eqn
``riesz``) and the reduced affine operators of Section 3.4 and the third-order convection
tensors of eqn ``tensor``. Its airfoil snapshots are not available, so this module builds a
synthetic stand-in with the same structure:

* velocity basis  phi_i = curl psi_i, psi_i a seeded random Fourier stream function
  (|k| <= kmax, amplitudes N(0,1)/|k|^2), L2-orthonormalised in order (nested);
  every phi_i is exactly divergence free, the analogue of the paper's conforming basis;
* pressure basis p_j: seeded random zero-mean Fourier scalars, L2-orthonormal, nested;
* supremizers s_j: the exact H^1-seminorm Riesz representers of b(p_j, .), i.e.
  -Laplace(s_j) = grad(p_j) (paper eqn ``riesz`` with b(p,w) = -int p div w);
* affine operators (row index = test function, as in a Galerkin matrix):
    A_q[i,j]      = a_q(phi_j, phi_i),  a_q(u,w) = sum_c int (grad u^c)^T K_q grad w^c
    C_q[i,j,k]    = c_q(phi_j, phi_k, phi_i),  c_q(u,v,w) = int ((u.grad) v) . (M_q w)
    F_q[i]        = int phi_i . g_q
    Bp_q[i,j]     = b_q(p_j, s_i),      b_q(p,w) = -int p (Bm_q : grad w)
    Asv_q[i,j]    = a_q(phi_j, s_i)
    Csv_q[i,j,k]  = c_q(phi_j, phi_k, s_i)
    Fs_q[i]       = int s_i . g_q
  with K_0 = I (the viscous form, eqn ``form-3``), M_0 = I (eqn ``form-4``) and Bm_0 = I
  (eqn ``form-2``); the q >= 1 terms use fixed seeded matrices, in the spirit of the
  constant-matrix-weighted forms of the paper's affine expansions (Section 5).

All fields are trigonometric polynomials, and every integrand is a product of at most three
of them, so trapezoidal quadrature on a uniform G x G grid with G > 3*kmax integrates it
exactly: the tensors equal their continuous values up to rounding, for any such G.

Scalar fields are stored as cosine/sine coefficient pairs over a fixed list of half-plane
wave vectors; derivatives act on those pairs exactly ("spectral derivatives").
"""

from __future__ import annotations

import dataclasses
import hashlib
import json
import os

import numpy as np

TWO_PI = 2.0 * np.pi


# --------------------------------------------------------------------------------------
# Fourier bookkeeping
# --------------------------------------------------------------------------------------

def wave_vectors(kmax):
    """Half-plane integer wave vectors with 0 < |k| <= kmax, sorted by (|k|^2, kx, ky).

    The half plane is kx > 0, or kx == 0 and ky > 0; with a cosine and a sine per wave
    vector this spans every real zero-mean trigonometric polynomial of degree <= kmax.
    Sorting by |k|^2 makes the list for a smaller cut-off a prefix of the larger one.
    """
    ks = []
    for kx in range(0, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            if (kx > 0 or (kx == 0 and ky > 0)) and kx * kx + ky * ky <= kmax * kmax:
                ks.append((kx, ky))
    ks.sort(key=lambda k: (k[0] ** 2 + k[1] ** 2, k[0], k[1]))
    return np.array(ks, dtype=np.int64)


def deriv(c, K, axis):
    """Exact derivative d/dx_axis of fields given as (..., W, 2) cos/sin coefficients."""
    kd = TWO_PI * K[:, axis].astype(np.float64)
    out = np.empty_like(c)
    out[..., 0] = kd * c[..., 1]       # d/dx cos(2 pi k.x) = -2 pi k sin; d/dx sin = 2 pi k cos
    out[..., 1] = -kd * c[..., 0]
    return out


def grid_modes(K, G):
    """Matrix E (2W x G^2): rows cos(2 pi k.x), sin(2 pi k.x) at the G x G grid points."""
    x = np.arange(G, dtype=np.float64) / G
    X, Y = np.meshgrid(x, x, indexing="ij")
    ph = TWO_PI * (K[:, 0, None, None] * X[None] + K[:, 1, None, None] * Y[None])
    E = np.empty((2 * K.shape[0], G * G))
    E[0::2] = np.cos(ph).reshape(K.shape[0], -1)
    E[1::2] = np.sin(ph).reshape(K.shape[0], -1)
    return E


def on_grid(c, E):
    """Evaluate (..., W, 2) coefficient fields at grid points -> (..., G^2)."""
    lead = c.shape[:-2]
    return (c.reshape(-1, c.shape[-2] * 2) @ E).reshape(*lead, E.shape[1])


def orthonormalise(X):
    """Gram-Schmidt (Householder QR) of the rows of X in order, positive diagonal.

    Returns T (lower triangular) such that rows of T @ X are orthonormal in the Euclidean
    inner product. Row i of the result depends only on rows 0..i of X (nested).
    """
    Qm, R = np.linalg.qr(X.T)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    R = s[:, None] * R
    return np.linalg.inv(R).T


def _rot(beta):
    c, s = np.cos(beta), np.sin(beta)
    return np.array([[c, -s], [s, c]])


# --------------------------------------------------------------------------------------
# Tensor set
# --------------------------------------------------------------------------------------

@dataclasses.dataclass
class TensorSet:
    """The affine operators of one synthetic reduced model (row index = test function)."""

    N: int
    Q: int
    Qc: int
    Qf: int
    Np: int
    Qb: int
    A: np.ndarray      # (Q, N, N)      A[q,i,j]   = a_q(phi_j, phi_i)
    C: np.ndarray      # (Qc, N, N, N)  C[q,i,j,k] = c_q(phi_j, phi_k, phi_i)
    F: np.ndarray      # (Qf, N)        F[q,i]     = (g_q, phi_i)
    H: np.ndarray      # (N, N)         H^1-seminorm Gram (= A[0]), norm of the stopping test
    Bp: np.ndarray     # (Qb, Np, Np)   Bp[q,i,j]  = b_q(p_j, s_i)
    Asv: np.ndarray    # (Q, Np, N)     Asv[q,i,j] = a_q(phi_j, s_i)
    Csv: np.ndarray    # (Qc, Np, N, N) Csv[q,i,j,k] = c_q(phi_j, phi_k, s_i)
    Fs: np.ndarray     # (Qf, Np)       Fs[q,i]    = (g_q, s_i)
    meta: dict = dataclasses.field(default_factory=dict)

    def leading(self, n, npr=None):
        """Nested sub-model: the leading n velocity (and npr pressure) functions."""
        npr = self.Np if npr is None else npr
        return TensorSet(
            N=n, Q=self.Q, Qc=self.Qc, Qf=self.Qf, Np=npr, Qb=self.Qb,
            A=np.ascontiguousarray(self.A[:, :n, :n]),
            C=np.ascontiguousarray(self.C[:, :n, :n, :n]),
            F=np.ascontiguousarray(self.F[:, :n]),
            H=np.ascontiguousarray(self.H[:n, :n]),
            Bp=np.ascontiguousarray(self.Bp[:, :npr, :npr]),
            Asv=np.ascontiguousarray(self.Asv[:, :npr, :n]),
            Csv=np.ascontiguousarray(self.Csv[:, :npr, :n, :n]),
            Fs=np.ascontiguousarray(self.Fs[:, :npr]),
            meta=dict(self.meta, N=n, Np=npr),
        )


def _basis_coefficients(N, Np, kmax, seeds):
    """Cos/sin coefficients of the orthonormal velocity, pressure and supremizer bases."""
    K = wave_vectors(kmax)
    W = K.shape[0]
    if 2 * W < max(N, Np):
        raise ValueError(f"kmax={kmax} gives {2 * W} real modes, fewer than N={N} / Np={Np}")
    k2 = (K[:, 0] ** 2 + K[:, 1] ** 2).astype(np.float64)

    # Velocity: phi = curl psi = (d_y psi, -d_x psi).
    rng = np.random.default_rng(seeds["basis"])
    psi = rng.standard_normal((N, W, 2)) / k2[None, :, None]
    phi = np.stack([deriv(psi, K, 1), -deriv(psi, K, 0)], axis=1)       # (N, 2, W, 2)
    # L2 inner product of two coefficient fields: 1/2 sum of coefficient products.
    T = orthonormalise(phi.reshape(N, -1) * np.sqrt(0.5))
    phi = (T @ phi.reshape(N, -1)).reshape(N, 2, W, 2)

    # Pressure: zero-mean scalars, L2-orthonormal.
    rng = np.random.default_rng(seeds["pbasis"])
    p = rng.standard_normal((Np, W, 2)) / k2[None, :, None]
    T = orthonormalise(p.reshape(Np, -1) * np.sqrt(0.5))
    p = (T @ p.reshape(Np, -1)).reshape(Np, W, 2)

    # Supremizers: -Laplace(s) = grad(p); per mode grad(p) / (4 pi^2 |k|^2).
    lap = (TWO_PI ** 2) * k2
    s = np.stack([deriv(p, K, 0), deriv(p, K, 1)], axis=1) / lap[None, None, :, None]
    return K, phi, p, s


def _form_matrices(Q, Qc, Qb, seeds):
    """K_q (SPD metric), M_q (symmetric convection weight), Bm_q (divergence weight)."""
    rng = np.random.default_rng(seeds["metric"])
    Ks = [np.eye(2)]
    for _ in range(1, Q):
        beta = rng.uniform(0.0, np.pi)
        lam = rng.uniform(0.5, 2.0, size=2)
        R = _rot(beta)
        Ks.append(R @ np.diag(lam) @ R.T)
    rng = np.random.default_rng(seeds["convect"])
    Ms = [np.eye(2)]
    for _ in range(1, Qc):
        gam = rng.uniform(0.0, np.pi)
        d = rng.uniform(-1.0, 1.0, size=2)
        d = d / np.max(np.abs(d))
        R = _rot(gam)
        Ms.append(R @ np.diag(d) @ R.T)
    rng = np.random.default_rng([seeds["metric"], 1])
    Bs = [np.eye(2)]
    for _ in range(1, Qb):
        Bm = rng.standard_normal((2, 2))
        Bs.append(0.5 * Bm / np.linalg.norm(Bm))
    return Ks, Ms, Bs


def _forcing(Qf, K, force_kmax, scale, seeds):
    """Body forces g_q = scale * (curl psi_q + grad chi_q), |k| <= force_kmax."""
    k2 = (K[:, 0] ** 2 + K[:, 1] ** 2)
    Wf = int(np.sum(k2 <= force_kmax ** 2))   # prefix of the sorted wave-vector list
    rng = np.random.default_rng(seeds["force"])
    W = K.shape[0]
    psi = np.zeros((Qf, W, 2))
    chi = np.zeros((Qf, W, 2))
    kf = np.sqrt(k2[:Wf].astype(np.float64))
    for q in range(Qf):
        psi[q, :Wf] = rng.standard_normal((Wf, 2)) / kf[:, None] ** 2
        chi[q, :Wf] = rng.standard_normal((Wf, 2)) / kf[:, None] ** 2
    g = np.stack([deriv(psi, K, 1), -deriv(psi, K, 0)], axis=1)
    g += np.stack([deriv(chi, K, 0), deriv(chi, K, 1)], axis=1)
    return scale * g                                                      # (Qf, 2, W, 2)


def assemble(N, Np, kmax, G, Q, Qc, Qf, Qb, seeds, force_kmax=4, forcing_scale=1.0,
             jchunk=None):
    """Build the affine operators by exact trapezoidal quadrature on a G x G grid."""
    if G <= 3 * kmax:
        raise ValueError(f"G={G} must exceed 3*kmax={3 * kmax} for exact quadrature")
    K, phi_c, p_c, s_c = _basis_coefficients(N, Np, kmax, seeds)
    Ks, Ms, Bs = _form_matrices(Q, Qc, Qb, seeds)
    g_c = _forcing(Qf, K, force_kmax, forcing_scale, seeds)
    E = grid_modes(K, G)
    X = G * G
    w = 1.0 / X

    phi = on_grid(phi_c, E)                                                  # (N, 2, X)
    dphi = np.stack([on_grid(deriv(phi_c, K, a), E) for a in range(2)], 1)   # (N, a, b, X)
    p = on_grid(p_c, E)                                                      # (Np, X)
    s = on_grid(s_c, E)                                                      # (Np, 2, X)
    ds = np.stack([on_grid(deriv(s_c, K, a), E) for a in range(2)], 1)       # (Np, a, b, X)
    g = on_grid(g_c, E)                                                      # (Qf, 2, X)

    # a_q(u, w) = sum_c sum_{a,a'} K[a,a'] int d_a u^c d_a' w^c
    def aform(du, dw, Km):
        Kdw = np.einsum("ab,nbcx->nacx", Km, dw)
        return (du.reshape(du.shape[0], -1) @ Kdw.reshape(dw.shape[0], -1).T) * w

    if len(Ks) <= 12 and len(Ms) <= 4:
        A = np.stack([aform(dphi, dphi, Km).T for Km in Ks])      # A[q,i,j] = a(phi_j, phi_i)
        Asv = np.stack([aform(dphi, ds, Km).T for Km in Ks])      # Asv[q,i,j] = a(phi_j, s_i)
    else:
        # long expansions: every form is linear in its weight matrix, so the Q (Qc) operators
        # are weighted sums of four base operators, one per weight entry
        E2 = np.eye(4).reshape(4, 2, 2)
        Ab = np.stack([aform(dphi, dphi, Eb).T for Eb in E2])
        Asb = np.stack([aform(dphi, ds, Eb).T for Eb in E2])
        A = np.einsum("qk,kij->qij", np.array(Ks).reshape(len(Ks), 4), Ab)
        Asv = np.einsum("qk,kij->qij", np.array(Ks).reshape(len(Ks), 4), Asb)

    F = np.einsum("qbx,ibx->qi", g, phi) * w
    Fs = np.einsum("qbx,ibx->qi", g, s) * w

    # b_q(p, w) = -int p (Bm : grad w), (grad w)_{ab} = d_b w^a
    Bp = np.stack([-np.einsum("ab,ibax,jx->ij", Bm, ds, p) * w for Bm in Bs])

    # c_q(u, v, t) = int ((u . grad) v) . (M_q t); tensors by chunks of the advecting index j.
    long_c = len(Ms) > 4 or len(Ks) > 12
    Mw = np.eye(4).reshape(4, 2, 2) if long_c else Ms       # base weights for long expansions
    Qw = len(Mw)
    Mphi = np.stack([np.einsum("bc,icx->ibx", Mm, phi) for Mm in Mw])      # (Qw, N, 2, X)
    Ms_ = np.stack([np.einsum("bc,icx->ibx", Mm, s) for Mm in Mw])          # (Qw, Np, 2, X)
    Ytest = np.concatenate([Mphi.reshape(Qw * N, 2 * X), Ms_.reshape(Qw * Np, 2 * X)])
    C = np.empty((Qw, N, N, N))
    Csv = np.empty((Qw, Np, N, N))
    if jchunk is None:
        jchunk = max(1, min(N, int(2e8 // (N * 2 * X * 8))))
    for j0 in range(0, N, jchunk):
        j1 = min(N, j0 + jchunk)
        # T[j,k,b,x] = sum_a phi_j^a d_a phi_k^b
        T = np.einsum("jax,kabx->jkbx", phi[j0:j1], dphi)
        R = (Ytest @ T.reshape((j1 - j0) * N, 2 * X).T) * w             # (Qc(N+Np), (j,k))
        R = R.reshape(-1, j1 - j0, N)
        C[:, :, j0:j1, :] = R[: Qw * N].reshape(Qw, N, j1 - j0, N)
        Csv[:, :, j0:j1, :] = R[Qw * N:].reshape(Qw, Np, j1 - j0, N)
    if long_c:
        Mk = np.array(Ms).reshape(len(Ms), 4)
        C = np.einsum("qk,kijl->qijl", Mk, C)
        Csv = np.einsum("qk,kijl->qijl", Mk, Csv)

    return dict(A=A, C=C, F=F, H=A[0].copy(), Bp=Bp, Asv=Asv, Csv=Csv, Fs=Fs,
                Ks=np.array(Ks), Ms=np.array(Ms), Bs=np.array(Bs), K=K,
                phi_c=phi_c, p_c=p_c, s_c=s_c, g_c=g_c)


def quadrature_fields(N, Np, kmax, G, Q, Qc, Qb, seeds):
    """The basis fields at the G x G quadrature points, as the offline tensor assembly consumes
    them (same bases and weight matrices as ``assemble``): phi (N, 2, X) with X = G^2,
    dphi (N, 2, 2, X) with dphi[i, a, b] = d_a phi_i^b, the supremizers s (Np, 2, X), the
    convection weights M (Qc, 2, 2) and the quadrature weight w = 1 / X."""
    K, phi_c, p_c, s_c = _basis_coefficients(N, Np, kmax, seeds)
    _, Ms, _ = _form_matrices(Q, Qc, Qb, seeds)
    E = grid_modes(K, G)
    phi = on_grid(phi_c, E)
    dphi = np.stack([on_grid(deriv(phi_c, K, a), E) for a in range(2)], 1)
    s_ = on_grid(s_c, E)
    return dict(phi=phi, dphi=dphi, s=s_, M=np.array(Ms), w=1.0 / (G * G))


def assemble_coupled(N, Np, kmax, G, Q, Qc, Qf, seeds, force_kmax=4, forcing_scale=1.0):
    """Operators of the coupled stabilised system (eqn block) as one velocity-only-shaped set.

    The supremizer-enriched velocity space V = [phi_1..phi_N, s_1..s_Np] and the pressure space
    give M = N + 2 Np unknowns x = (u, s, p). Written as A(mu) x + C(mu)(x, x) = f(mu):
      A_q (q < Q)   [[a_q(V_j, V_i), 0], [0, 0]]       (the velocity block, N + Np square)
      A_Q           [[0, B^T], [B, 0]] with B[i][j] = b(p_i, V_j), the pressure form with the
                    identity weight (b(p, w) = -int p div w), so B_vp = 0 for the solenoidal
                    phi and B_ps is the supremizer Gramian
      C_q           c_q(V_j, V_k, V_i) on the velocity block, zero elsewhere
      F_q           [(g_q, V_i); 0]
      H             blockdiag(a_0(V_j, V_i), I): H^1 seminorm on the velocity, L2 on p
    The bases, forms and forcing are those of ``assemble`` with the same seeds (nested: the
    first N velocity and Np pressure functions are the leading ones of a larger set). With the
    affine coefficients (theta^a, 1) the solution is (u, 0, p) with u the velocity-only
    solution and p its recovered pressure (eqn piolablock with B_vp = 0, f_p = 0).
    """
    if G <= 3 * kmax:
        raise ValueError(f"G={G} must exceed 3*kmax={3 * kmax} for exact quadrature")
    K, phi_c, p_c, s_c = _basis_coefficients(N, Np, kmax, seeds)
    Ks, Ms, _ = _form_matrices(Q, Qc, 1, seeds)
    g_c = _forcing(Qf, K, force_kmax, forcing_scale, seeds)
    E = grid_modes(K, G)
    X = G * G
    w = 1.0 / X
    Nv = N + Np
    M = Nv + Np
    v_c = np.concatenate([phi_c, s_c], axis=0)                               # (Nv, 2, W, 2)
    V = on_grid(v_c, E)                                                      # (Nv, 2, X)
    dV = np.stack([on_grid(deriv(v_c, K, a), E) for a in range(2)], 1)       # (Nv, a, b, X)
    pg = on_grid(p_c, E)                                                     # (Np, X)
    g = on_grid(g_c, E)

    def aform(du, dw, Km):
        Kdw = np.einsum("ab,nbcx->nacx", Km, dw)
        return (du.reshape(du.shape[0], -1) @ Kdw.reshape(dw.shape[0], -1).T) * w

    A = np.zeros((Q + 1, M, M))
    for q, Km in enumerate(Ks):
        A[q, :Nv, :Nv] = aform(dV, dV, Km).T                   # A[q,i,j] = a(V_j, V_i)
    divV = dV[:, 0, 0] + dV[:, 1, 1]                           # (Nv, X)
    Bm = -(pg @ divV.T) * w                                    # Bm[i, j] = b(p_i, V_j)
    A[Q, Nv:, :Nv] = Bm
    A[Q, :Nv, Nv:] = Bm.T
    C = np.zeros((Qc, M, M, M))
    MV = np.stack([np.einsum("bc,icx->ibx", Mm, V) for Mm in Ms])          # (Qc, Nv, 2, X)
    T = np.einsum("jax,kabx->jkbx", V, dV)                                 # (Nv, Nv, 2, X)
    R = (MV.reshape(Qc * Nv, 2 * X) @ T.reshape(Nv * Nv, 2 * X).T) * w
    C[:, :Nv, :Nv, :Nv] = R.reshape(Qc, Nv, Nv, Nv)
    F = np.zeros((Qf, M))
    F[:, :Nv] = np.einsum("qbx,ibx->qi", g, V) * w
    H = np.eye(M)
    H[:Nv, :Nv] = A[0, :Nv, :Nv]
    return dict(A=A, C=C, F=F, H=H, Nv=Nv, M=M)


def make_coupled_set(cfg, N, Np):
    """The coupled system of ``assemble_coupled`` for a configuration's bases and forms, as a
    TensorSet of size N + 2 Np with Q + 1 affine terms (no pressure data: p is an unknown)."""
    d = assemble_coupled(N, Np, cfg["kmax"], cfg["G_quad"], cfg["Q"], cfg["Qc"], cfg["Qf"],
                         cfg["seeds"], cfg.get("force_kmax", 4), cfg.get("forcing_scale", 1.0))
    M = d["M"]
    return TensorSet(N=M, Q=cfg["Q"] + 1, Qc=cfg["Qc"], Qf=cfg["Qf"], Np=0, Qb=1, A=d["A"],
                     C=d["C"], F=d["F"], H=d["H"], Bp=np.zeros((1, 0, 0)),
                     Asv=np.zeros((cfg["Q"] + 1, 0, M)), Csv=np.zeros((cfg["Qc"], 0, M, M)),
                     Fs=np.zeros((cfg["Qf"], 0)),
                     meta=dict(coupled=True, Nvel=N, Npres=Np, Nsup=Np))


_CACHE_KEYS = ("N", "Np", "kmax", "G_quad", "Q", "Qc", "Qf", "Qb", "force_kmax",
               "forcing_scale", "seeds")


def _cache_path(cfg, cache_dir):
    key = json.dumps({k: cfg[k] for k in _CACHE_KEYS}, sort_keys=True)
    h = hashlib.sha256(key.encode()).hexdigest()[:16]
    return os.path.join(cache_dir, f"tensors_{cfg.get('name', 'cfg')}_{h}.npz")


def make_tensor_set(cfg, cache_dir=None):
    """Tensor set for a configuration dict (see ``rbinputs.configs``), optionally cached."""
    path = _cache_path(cfg, cache_dir) if cache_dir else None
    if path and os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            d = {k: z[k] for k in z.files}
    else:
        d = assemble(cfg["N"], cfg["Np"], cfg["kmax"], cfg["G_quad"], cfg["Q"], cfg["Qc"],
                     cfg["Qf"], cfg["Qb"], cfg["seeds"], cfg.get("force_kmax", 4),
                     cfg.get("forcing_scale", 1.0))
        d = {k: d[k] for k in ("A", "C", "F", "H", "Bp", "Asv", "Csv", "Fs")}
        if path:
            os.makedirs(cache_dir, exist_ok=True)
            tmp = path + f".tmp{os.getpid()}.npz"
            np.savez(tmp, **d)
            os.replace(tmp, path)
    return TensorSet(N=cfg["N"], Q=cfg["Q"], Qc=cfg["Qc"], Qf=cfg["Qf"], Np=cfg["Np"],
                     Qb=cfg["Qb"], meta={k: cfg[k] for k in cfg if k != "seeds"}, **d)


# --------------------------------------------------------------------------------------
# Parameter and request streams
# --------------------------------------------------------------------------------------

def draw_mu(cfg, B=None, seed_offset=0):
    """Parameter samples mu = (alpha [rad], Re), shape (B, 2), float64.

    alpha ~ U[alpha_deg range] (degrees, converted to radians), Re ~ U[Re range]; a
    configuration with ``fixed_mu`` repeats that single parameter.
    """
    B = cfg["B"] if B is None else B
    if "fixed_mu" in cfg:
        a, re = cfg["fixed_mu"]
        return np.tile(np.array([[np.deg2rad(a), re]]), (B, 1))
    rng = np.random.default_rng([cfg["seeds"]["mu"], seed_offset])
    u = rng.random((B, 2))
    lo, hi = cfg["alpha_deg"]
    rlo, rhi = cfg["Re"]
    mu = np.empty((B, 2))
    mu[:, 0] = np.deg2rad(lo + (hi - lo) * u[:, 0])
    mu[:, 1] = rlo + (rhi - rlo) * u[:, 1]
    return mu


def gauss_grid_mu(cfg, n=15):
    """n x n Gauss-Legendre points over the configuration's (alpha, Re) box, alpha in rad (a
    training ensemble of the shape the paper uses: 15 x 15 Gauss points of its parameters)."""
    x, _ = np.polynomial.legendre.leggauss(n)
    lo, hi = np.deg2rad(cfg["alpha_deg"][0]), np.deg2rad(cfg["alpha_deg"][1])
    rlo, rhi = cfg["Re"]
    a = lo + (hi - lo) * (x + 1.0) / 2.0
    r = rlo + (rhi - rlo) * (x + 1.0) / 2.0
    A, Rr = np.meshgrid(a, r, indexing="ij")
    return np.column_stack([A.ravel(), Rr.ravel()])


def draw_basis_sizes(cfg, B=None, seed_offset=0):
    """Per-request basis sizes for uneven batches (int32, shape (B,))."""
    B = cfg["B"] if B is None else B
    rng = np.random.default_rng([cfg["seeds"]["ndraw"], seed_offset])
    if "N_choices" in cfg:
        return rng.choice(np.asarray(cfg["N_choices"], dtype=np.int32), size=B)
    if "N_range" in cfg:
        lo, hi = cfg["N_range"]
        return rng.integers(lo, hi + 1, size=B, dtype=np.int32)
    return np.full(B, cfg["N"], dtype=np.int32)


def draw_arrivals(cfg, rate, duration_s, seed_offset=0):
    """Poisson arrival times (seconds) at ``rate`` requests per second over ``duration_s``."""
    rng = np.random.default_rng([cfg["seeds"]["arrivals"], seed_offset, int(rate)])
    n = int(rate * duration_s * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    return t[t < duration_s]
