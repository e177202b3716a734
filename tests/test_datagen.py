"""The seeded input generator: Philox known answers, addressing, recipes."""
import os

import numpy as np
import pytest
import torch

import datagen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(h, 16) for h in r]
        out = datagen.philox4x32_10(v[0:4], v[4:6])
        assert list(out) == v[6:10]


def test_rows_regenerate_independently():
    full = datagen.normal_matrix(7, 0x1001, 37, 13)
    part = datagen.normal_matrix(7, 0x1001, 5, 13, row0=20)
    np.testing.assert_array_equal(full[20:25], part)
    u = datagen.uniform_vector(7, 5, 50)
    np.testing.assert_array_equal(u[10:30], datagen.uniform_vector(7, 5, 20, k0=10))
    assert np.all((u > 0) & (u < 1))


def test_normal_moments():
    z = datagen.normal_matrix(3, 0x1000, 400, 250).ravel()
    assert abs(z.mean()) < 0.01
    assert abs(z.std() - 1.0) < 0.01
    # fourth moment of N(0,1) is 3
    assert abs(np.mean(z ** 4) - 3.0) < 0.1


def test_bf16_round_to_nearest_even_matches_torch():
    x = datagen.to_f32(datagen.normal_matrix(5, 0x1000, 64, 64) * 10.0)
    # include exact halfway cases: low 16 bits == 0x8000
    bits = x.view(np.uint32).copy()
    bits[0, :8] = (bits[0, :8] & 0xFFFF0000) | 0x8000
    x = bits.view(np.float32)
    ours = datagen.f32_to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, ref)
    back = datagen.bf16_bits_to_f64(ours)
    ref_back = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(back, ref_back)


def test_ar1_rows_have_toeplitz_covariance():
    w = datagen.logistic_workload(11, N=1, m_per=20000, n=6, kappa=2, k_true=2, n_blocks=2,
                                  dtype="f64")
    A = w.A[0]
    S = A.T @ A / A.shape[0]
    ref = 0.3 ** np.abs(np.subtract.outer(np.arange(6), np.arange(6)))
    assert np.max(np.abs(S - ref)) < 0.03


def test_config0_shape_and_plant():
    w = datagen.config0()
    assert w.N == 4 and all(a.shape == (500, 200) for a in w.A)
    assert w.A[0].dtype == np.float64
    nz = np.nonzero(w.x_true)[0]
    assert len(nz) == 10
    assert np.all((np.abs(w.x_true[nz]) >= 1) & (np.abs(w.x_true[nz]) <= 2))
    resid = w.b[0] - w.A[0] @ w.x_true
    assert 0.005 < resid.std() < 0.02


def test_unit_norm_columns_and_storage_rounding():
    w = datagen.linear_workload(2, N=2, m_per=300, n=40, kappa=5, k_true=5, noise=0.05,
                                n_blocks=4, dtype="bf16", normalize=True)
    A = datagen.widen(w.A[0])
    norms = np.sqrt(np.sum(A * A, axis=0))
    assert np.max(np.abs(norms - 1.0)) < 2 ** -7
    w32 = datagen.linear_workload(2, N=2, m_per=300, n=40, kappa=5, k_true=5, noise=0.05,
                                  n_blocks=4, dtype="f32", normalize=True)
    # BF16 storage is the RNE rounding of the canonical FP32 matrix
    np.testing.assert_array_equal(w.A[1], datagen.f32_to_bf16_bits(w32.A[1]))
    np.testing.assert_array_equal(w.b[1], w32.b[1])


def test_split_rows_uneven():
    assert datagen.split_rows(10, 4) == [3, 3, 2, 2]
    assert sum(datagen.split_rows(20001, 4)) == 20001


def test_logistic_labels_follow_the_planted_model():
    w = datagen.logistic_workload(4, N=1, m_per=20000, n=30, kappa=3, k_true=3, n_blocks=2,
                                  dtype="f32")
    b = w.b[0]
    assert set(np.unique(b)) == {-1.0, 1.0}
    logit = datagen.widen(w.A[0]) @ w.x_true
    # E[b | logit] = 2 sigmoid(logit) - 1
    sel = np.abs(logit) > 1.0
    agree = np.mean(np.sign(logit[sel]) == b[sel])
    expected = np.mean(1.0 / (1.0 + np.exp(-np.abs(logit[sel]))))
    assert abs(agree - expected) < 0.02


def test_softmax_labels_in_range():
    w = datagen.softmax_workload(9, N=2, m_per=200, n=20, C=4, kappa=3, k_true=3, n_blocks=2)
    for y in w.b:
        assert y.dtype == np.int32 and y.min() >= 0 and y.max() < 4
    assert np.count_nonzero(np.abs(w.x_true).sum(axis=1)) == 3


def test_gaussian_block_matches_the_fp64_recipe():
    # the fused generator draws the same normals as normal_matrix, rounds them
    # once to FP32 (and RNE from there to BF16); with normalisation the columns
    # have unit FP64 norm before rounding
    m, n = 300, 37
    supp, val = datagen.linear_model(9, n, 4)
    (A32, Abf), b = datagen.linear_partition(9, 2, m, n, supp, val, 0.05, "f32+bf16", False)
    G = datagen.normal_matrix(9, datagen.S_A + 2, m, n)
    np.testing.assert_array_equal(A32, G.astype(np.float32))
    np.testing.assert_array_equal(Abf, datagen.f32_to_bf16_bits(A32))
    (N32, Nbf), _ = datagen.linear_partition(9, 2, m, n, supp, val, 0.05, "f32+bf16", True)
    scale = 1.0 / np.linalg.norm(G, axis=0)
    np.testing.assert_allclose(N32.astype(np.float64), G * scale, rtol=1e-6, atol=1e-8)
    assert np.allclose(np.linalg.norm(N32.astype(np.float64), axis=0), 1.0, atol=1e-6)
    np.testing.assert_array_equal(Nbf, datagen.f32_to_bf16_bits(N32))
