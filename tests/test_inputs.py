"""Pins of the synthetic input generator against closed forms and exactness properties.

The generator stands in for the paper's offline stage; these tests check what the
mathematics fixes for it: solenoidal velocity basis (the analogue of the paper's
divergence-conforming basis, Section 6.3), orthonormality and nestedness of the POD-like
bases (Section 3.2), exact quadrature, skew-symmetry of the convection tensors (eqn form-4
on solenoidal periodic fields), the supremizer Gramian (Section 3.4) and the velocity /
supremizer orthogonality (the 90-degree limit of the paper's principal-angle table).
"""

import numpy as np
import pytest

from rbinputs import get_config, make_tensor_set
from rbinputs import synth as S

SEEDS = get_config("single_n10")["seeds"]


def _small(N=10, Np=6, kmax=6, G=32, Q=3, Qc=2, Qf=2, Qb=2, **kw):
    return S.assemble(N, Np, kmax, G, Q, Qc, Qf, Qb, SEEDS, **kw)


def test_wave_vector_prefix_and_count():
    K6 = S.wave_vectors(6)
    K12 = S.wave_vectors(12)
    assert np.array_equal(K12[: len(K6)], K6)
    # half of the nonzero lattice points in the disc of radius kmax
    n = sum(1 for x in range(-6, 7) for y in range(-6, 7) if 0 < x * x + y * y <= 36)
    assert len(K6) == n // 2


def test_velocity_basis_divergence_free():
    d = _small()
    K = d["K"]
    phi = d["phi_c"]
    div = S.deriv(phi[:, 0], K, 0) + S.deriv(phi[:, 1], K, 1)
    assert np.max(np.abs(div)) <= 1e-12 * np.max(np.abs(phi))


def test_supremizers_curl_free():
    d = _small()
    K = d["K"]
    s = d["s_c"]
    curl = S.deriv(s[:, 1], K, 0) - S.deriv(s[:, 0], K, 1)
    assert np.max(np.abs(curl)) <= 1e-12 * np.max(np.abs(s))


def test_orthonormal_by_quadrature():
    d = _small(G=40)
    E = S.grid_modes(d["K"], 40)
    phi = S.on_grid(d["phi_c"], E)                  # (N, 2, X)
    gram = np.einsum("ibx,jbx->ij", phi, phi) / E.shape[1]
    assert np.max(np.abs(gram - np.eye(gram.shape[0]))) < 1e-13
    p = S.on_grid(d["p_c"], E)
    gp = p @ p.T / E.shape[1]
    assert np.max(np.abs(gp - np.eye(gp.shape[0]))) < 1e-13


def test_quadrature_exact_grid_independent():
    a = _small(G=19 + 1)    # smallest even grid above 3*kmax = 18
    b = _small(G=48)
    for k in ("A", "C", "F", "Bp", "Asv", "Csv", "Fs"):
        scale = max(1.0, np.max(np.abs(b[k])))
        assert np.max(np.abs(a[k] - b[k])) <= 1e-13 * scale, k


def test_quadrature_grid_too_coarse_rejected():
    with pytest.raises(ValueError):
        _small(G=18)


def test_nested_bases():
    big = _small(N=14, Np=8)
    sm = _small(N=9, Np=5)
    assert np.allclose(big["A"][:, :9, :9], sm["A"], rtol=0, atol=1e-10)
    assert np.allclose(big["C"][:, :9, :9, :9], sm["C"], rtol=0, atol=1e-12)
    assert np.allclose(big["F"][:, :9], sm["F"], rtol=0, atol=1e-12)
    assert np.allclose(big["Bp"][:, :5, :5], sm["Bp"], rtol=0, atol=1e-12)
    assert np.allclose(big["Csv"][:, :5, :9, :9], sm["Csv"], rtol=0, atol=1e-12)


def test_A0_closed_form():
    """A_0 = int grad phi_i : grad phi_j = sum_k 4 pi^2 |k|^2 (1/2) sum_c coef_i^c . coef_j^c."""
    d = _small()
    K = d["K"]
    k2 = (K[:, 0] ** 2 + K[:, 1] ** 2).astype(float)
    phi = d["phi_c"]                                   # (N, 2, W, 2)
    closed = 0.5 * np.einsum("w,icwz,jcwz->ij", 4 * np.pi ** 2 * k2, phi, phi)
    assert np.max(np.abs(closed - d["A"][0])) <= 1e-11 * np.max(np.abs(closed))


def test_A_symmetric_positive_definite():
    d = _small()
    for Aq in d["A"]:
        assert np.allclose(Aq, Aq.T, atol=1e-10)
        assert np.linalg.eigvalsh(Aq).min() > 0


def test_convection_skew_symmetry():
    """c(u, v, w) = -c(u, w, v) for solenoidal periodic u and symmetric weights M_q."""
    d = _small(Qc=3)
    C = d["C"]
    assert np.max(np.abs(C + C.transpose(0, 3, 2, 1))) <= 1e-13 * np.max(np.abs(C))
    # hence c(u, u, u) = 0 for any u in the span
    u = np.random.default_rng(0).standard_normal(C.shape[1])
    for q in range(C.shape[0]):
        assert abs(np.einsum("ijk,i,j,k->", C[q], u, u, u)) < 1e-12 * np.abs(C[q]).max()


def test_supremizer_gramian_identity_and_zero_Asv():
    """B_0[i,j] = b(p_j, s_i) = (s_i, s_j)_{H1} = (p_i, p_j)_{L2} = delta_ij; a_q(phi, s) = 0."""
    d = _small()
    assert np.max(np.abs(d["Bp"][0] - np.eye(d["Bp"].shape[1]))) < 1e-13
    assert np.max(np.abs(d["Asv"])) < 1e-11


def test_velocity_supremizer_principal_angle_90_degrees():
    d = _small(G=40)
    E = S.grid_modes(d["K"], 40)
    K = d["K"]
    dphi = np.stack([S.on_grid(S.deriv(d["phi_c"], K, a), E) for a in range(2)], 1)
    ds = np.stack([S.on_grid(S.deriv(d["s_c"], K, a), E) for a in range(2)], 1)
    cross = np.einsum("iabx,jabx->ij", dphi, ds) / E.shape[1]
    assert np.max(np.abs(cross)) < 1e-11   # cos(angle) = 0 in the H1 inner product


def test_loads_match_independent_quadrature():
    """F_q and Fs_q equal the L2 pairings of g_q with phi_i and s_i evaluated on a new grid."""
    d = _small()
    K = d["K"]
    g = d["g_c"]                                       # (Qf, 2, W, 2)
    E = S.grid_modes(K, 32)
    phi = S.on_grid(d["phi_c"], E)
    s = S.on_grid(d["s_c"], E)
    gg = S.on_grid(g, E)
    F = np.einsum("qbx,ibx->qi", gg, phi) / E.shape[1]
    assert np.allclose(F, d["F"], atol=1e-12)
    Fs = np.einsum("qbx,ibx->qi", gg, s) / E.shape[1]
    assert np.allclose(Fs, d["Fs"], atol=1e-12)


def test_make_tensor_set_cache_roundtrip(tmp_path):
    cfg = get_config("single_n10")
    a = make_tensor_set(cfg, cache_dir=str(tmp_path))
    b = make_tensor_set(cfg, cache_dir=str(tmp_path))
    assert np.array_equal(a.C, b.C) and np.array_equal(a.A, b.A)
    sub = b.leading(6, 4)
    assert sub.C.shape == (1, 6, 6, 6) and sub.Csv.shape == (1, 4, 6, 6)
