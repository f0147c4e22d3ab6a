"""Pins of the oracle's footprint reconstruction: SPA + HALS for P ~ F A
(Eq. 3, Sec. III-D)."""
import numpy as np
import pytest

import oracle
from oracle import segment as _seg  # noqa: F401  (module import check)
import importlib

S = importlib.import_module("oracle.segment")


def test_rank1_exact():
    rng = np.random.default_rng(0)
    f = rng.uniform(0.1, 1.0, size=40)
    f[7] = 1.0
    a = rng.uniform(0, 3, size=25)
    a[[3, 9]] = 0.0
    P = np.outer(f, a)
    F, A, picks = oracle.nmf_component(P, oracle.Params())
    assert F.shape[1] == 1
    np.testing.assert_allclose(F[:, 0], f, rtol=1e-12)
    np.testing.assert_allclose(A[0], a, rtol=1e-12, atol=1e-12)


def test_two_sources_with_pure_columns():
    M = 30
    f1 = np.zeros(M); f1[:18] = np.linspace(0.2, 1.0, 18)
    f2 = np.zeros(M); f2[12:] = np.linspace(1.0, 0.3, 18)
    A = np.array([[2.0, 0.0, 1.0, 0.5, 0.0, 3.0],
                  [0.0, 1.5, 1.0, 0.2, 2.5, 0.0]])
    P = np.stack([f1, f2], 1) @ A
    F, Ah, picks = oracle.nmf_component(P, oracle.Params())
    assert F.shape[1] == 2
    c1 = int(np.argmax(F[0]))          # pixel 0 belongs to source 1 only
    order = [c1, 1 - c1]
    np.testing.assert_allclose(F[:, order[0]], f1, atol=1e-9)
    np.testing.assert_allclose(F[:, order[1]], f2, atol=1e-9)
    np.testing.assert_allclose(Ah[order], A, atol=1e-8)


def test_spa_picks_pure_columns_of_separable_matrix():
    rng = np.random.default_rng(1)
    W = rng.uniform(0, 1, size=(20, 3))
    W /= W.max(0)
    H = np.concatenate([np.eye(3) * [3.0, 2.0, 2.5],
                        rng.dirichlet(np.ones(3), size=7).T * 0.9], axis=1)
    perm = rng.permutation(H.shape[1])
    P = W @ H[:, perm]
    picks = oracle.spa(P, 0.05, 6)
    pure = sorted(int(np.flatnonzero(perm == k)[0]) for k in range(3))
    assert sorted(picks) == pure


def test_hals_objective_non_increasing():
    rng = np.random.default_rng(2)
    P = np.abs(rng.standard_normal((50, 30)))
    F = np.abs(rng.standard_normal((50, 3)))
    A = np.zeros((3, 30))
    A = S._hals_update_A(P, F, A)
    prev = np.linalg.norm(P - F @ A)
    for _ in range(30):
        A = S._hals_update_A(P, F, A)
        cur = np.linalg.norm(P - F @ A)
        assert cur <= prev * (1 + 1e-14)
        prev = cur
        F = S._hals_update_F(P, F, A)
        cur = np.linalg.norm(P - F @ A)
        assert cur <= prev * (1 + 1e-14)
        prev = cur
        assert (F >= 0).all() and (A >= 0).all()


def test_zero_matrix_gives_nothing():
    F, A, picks = oracle.nmf_component(np.zeros((10, 5)), oracle.Params())
    assert F.shape == (10, 0) and picks == []


def test_segment_permutation_invariance():
    M = 24
    f1 = np.zeros(M); f1[:14] = np.linspace(0.3, 1.0, 14)
    f2 = np.zeros(M); f2[10:] = np.linspace(1.0, 0.4, 14)
    A = np.array([[2.0, 0.0, 1.0, 0.0, 3.0], [0.0, 1.5, 0.7, 2.5, 0.0]])
    P = np.stack([f1, f2], 1) @ A
    perm = np.array([3, 0, 4, 2, 1])
    F1, A1, _ = oracle.nmf_component(P, oracle.Params())
    F2, A2, _ = oracle.nmf_component(P[:, perm], oracle.Params())
    k1 = np.argsort(F1.argmax(0)); k2 = np.argsort(F2.argmax(0))
    np.testing.assert_allclose(F1[:, k1], F2[:, k2], atol=1e-9)
    np.testing.assert_allclose(A1[k1][:, perm], A2[k2], atol=1e-8)


def test_footprints_order_and_drop():
    K, H, W = 6, 20, 20
    p = np.zeros((K, H, W))
    g = np.exp(-((np.mgrid[0:H, 0:W][0] - 5.0) ** 2 + (np.mgrid[0:H, 0:W][1] - 5.0) ** 2) / 8.0)
    p[1] = 3 * g
    p[4] = 2 * g
    p[2, 15, 15] = 1.0          # a tiny second component: mask under 16 px, dropped
    labels = np.zeros((H, W), np.int32)
    labels[g > 0.05] = 1
    labels[15, 15] = 2
    out = oracle.footprints(p, labels, 2, oracle.Params())
    assert len(out) == 1 and out[0]["component"] == 1
    assert out[0]["peak"] == 5 * W + 5
    np.testing.assert_allclose(out[0]["activity"], [0, 3, 0, 0, 2, 0], atol=1e-9)
