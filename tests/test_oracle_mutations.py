"""Planted mistakes in the oracle (CPU only) must each fail one of the pins.

Each case patches one oracle function with a plausible bug -- a dropped
sign, a bucket that reuses the sign bit, a wrong Box-Muller radius, a
dropped term, a missing sign in the adjoint -- and checks that a pin from
test_oracle_rng / test_oracle_sketch rejects it.
"""
import numpy as np
import pytest

import oracle as O
import oracle.countgauss as OC
import tests.test_oracle_rng as R
import tests.test_oracle_sketch as S


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(OC, name, fn)
    monkeypatch.setattr(O, name, fn)


def test_dropped_sign_is_caught(monkeypatch):
    orig = OC.hash_rows

    def unsigned(seed, B, rows):
        h, s = orig(seed, B, rows)
        return h, np.ones_like(s)

    _patch(monkeypatch, "hash_rows", unsigned)
    with pytest.raises(AssertionError):
        S.test_lower_bound_lemma_single_collision_identity()
    with pytest.raises(AssertionError):
        S.test_exact_second_moment_of_M_minus_C()


def test_bucket_sharing_the_sign_bit_is_caught(monkeypatch):
    def overlapping(seed, B, rows):
        w = OC.hash_words(seed, rows).astype(np.uint64)
        s = np.where((w >> np.uint64(31)) == 0, 1.0, -1.0)
        h = (w * np.uint64(B)) >> np.uint64(32)
        return h.astype(np.int64), s

    _patch(monkeypatch, "hash_rows", overlapping)
    with pytest.raises(AssertionError):
        S.test_exact_second_moment_of_M_minus_C()


def test_wrong_box_muller_radius_is_caught(monkeypatch):
    def bad(words):
        u = OC.uniforms_from_words(words)
        rho0 = np.sqrt(-np.log(u[..., 0]))
        rho1 = np.sqrt(-np.log(u[..., 2]))
        t0, t1 = 2 * np.pi * u[..., 1], 2 * np.pi * u[..., 3]
        return np.stack([rho0 * np.cos(t0), rho0 * np.sin(t0),
                         rho1 * np.cos(t1), rho1 * np.sin(t1)], axis=-1)

    _patch(monkeypatch, "box_muller", bad)
    with pytest.raises(AssertionError):
        R.test_gaussian_entries_follow_standard_normal()


def test_reused_angle_is_caught(monkeypatch):
    def bad(words):
        u = OC.uniforms_from_words(words)
        rho0 = np.sqrt(-2 * np.log(u[..., 0]))
        rho1 = np.sqrt(-2 * np.log(u[..., 2]))
        t0 = 2 * np.pi * u[..., 1]
        return np.stack([rho0 * np.cos(t0), rho0 * np.sin(t0),
                         rho1 * np.cos(t0), rho1 * np.sin(t0)], axis=-1)

    _patch(monkeypatch, "box_muller", bad)
    with pytest.raises(AssertionError):
        R.test_box_muller_pairs_share_a_radius_and_carry_the_angle()


def test_dropped_last_row_in_csr_scatter_is_caught(monkeypatch):
    orig = OC.sx_csr

    def dropping(row_ptr, col_idx, vals, n, d, seed, B, row_offset=0):
        rp = np.array(row_ptr, copy=True)
        rp[-1] = rp[-2]
        k = int(rp[-1])
        return orig(rp, col_idx[:k], vals[:k], n, d, seed, B, row_offset)

    _patch(monkeypatch, "sx_csr", dropping)
    with pytest.raises(AssertionError):
        S.test_csr_matches_dense_and_row_offset_chunking()


def test_unsigned_adjoint_gather_is_caught(monkeypatch):
    def bad(dY, n, d, m, B, seed, row_offset=0):
        Z = OC.gaussian_matrix(seed, m, B).T @ np.asarray(dY, np.float64)
        h, _ = OC.hash_rows(seed, B, np.arange(n, dtype=np.uint64) + np.uint64(row_offset))
        return Z[h]

    _patch(monkeypatch, "adjoint_dense", bad)
    with pytest.raises(AssertionError):
        S.test_adjoint_identity_dense_and_csr()


def test_transposed_gaussian_is_caught(monkeypatch):
    # G stored B x m and used as its transpose gives a different (m x B)
    # matrix whose rows are no longer the published Philox stream.
    orig = OC.gaussian_block

    def transposed(seed, m, b0, nb):
        big = orig(seed, max(m, b0 + nb), 0, max(m, b0 + nb))
        return big.T[:m, b0:b0 + nb]

    _patch(monkeypatch, "gaussian_block", transposed)
    with pytest.raises(AssertionError):
        R.test_box_muller_pairs_share_a_radius_and_carry_the_angle()
