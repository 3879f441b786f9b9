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


def test_off_by_one_hash_word_is_caught(monkeypatch):
    def shifted(seed, rows):
        rows = np.asarray(rows, dtype=np.uint64)
        q = rows >> np.uint64(2)
        ctr = np.zeros(rows.shape + (4,), dtype=np.uint32)
        ctr[..., 0] = (q & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        ctr[..., 1] = (q >> np.uint64(32)).astype(np.uint32)
        out = OC.philox4x32_10(ctr, OC.seed_key(seed))
        lane = ((rows + np.uint64(1)) & np.uint64(3)).astype(np.int64)
        return np.take_along_axis(out, lane[..., None], axis=-1)[..., 0]

    _patch(monkeypatch, "hash_words", shifted)
    with pytest.raises(AssertionError):
        R.test_hash_uses_one_philox_block_per_four_rows()


def test_uniform_map_without_midpoint_is_caught(monkeypatch):
    def bad(w):
        w = np.asarray(w, dtype=np.uint32)
        return (w >> np.uint32(8)).astype(np.float64) * 2.0 ** -24

    _patch(monkeypatch, "uniforms_from_words", bad)
    with pytest.raises(AssertionError):
        R.test_uniform_map_is_open_interval_and_exact()


def test_transposed_gaussian_counter_is_caught(monkeypatch):
    # counter (q, b, 1, 0) instead of (b, q, 1, 0)
    def transposed(seed, m, b0, nb):
        nq = (m + 3) // 4
        ctr = np.zeros((nq, nb, 4), dtype=np.uint32)
        ctr[..., 0] = np.arange(nq, dtype=np.uint32)[:, None]
        ctr[..., 1] = np.arange(b0, b0 + nb, dtype=np.uint32)[None, :]
        ctr[..., 2] = 1
        z = OC.box_muller(OC.philox4x32_10(ctr, OC.seed_key(seed)))
        return np.transpose(z, (0, 2, 1)).reshape(nq * 4, nb)[:m]

    _patch(monkeypatch, "gaussian_block", transposed)
    with pytest.raises(AssertionError):
        R.test_box_muller_pairs_share_a_radius_and_carry_the_angle()


# ---- emulate_reduced: each planted mistake fails the hand-worked case ----
def _emulate_variant(kblock=128, g_scale=2.0 ** -6, exponent=None, rescale=True):
    def emulate(G, SX, precision, kblock_=kblock):
        G32 = np.asarray(G, np.float32).astype(np.float64)
        S32 = np.asarray(SX, np.float32).astype(np.float64)
        m, B = G32.shape
        Y = np.zeros((m, S32.shape[1]))
        for k0 in range(0, B, kblock):
            g = G32[:, k0:k0 + kblock]
            s = S32[k0:k0 + kblock]
            if precision == "bf16":
                Y += OC.quantise_bf16(g) @ OC.quantise_bf16(s)
                continue
            amax = np.max(np.abs(s)) if s.size else 0.0
            e = exponent(amax) if exponent else OC.fp8_block_exponent(amax)
            sx = 2.0 ** e
            P = OC.quantise_fp8_e4m3(g / g_scale) @ OC.quantise_fp8_e4m3(s / sx)
            Y += P * (g_scale * sx) if rescale else P
        return Y
    return emulate


def _e_minus_8_everywhere(amax):
    if amax == 0.0:
        return 0
    import math
    return math.frexp(amax)[1] - 8


@pytest.mark.parametrize("variant", [
    dict(kblock=64), dict(exponent=_e_minus_8_everywhere), dict(g_scale=2.0 ** -5),
    dict(g_scale=2.0 ** -7), dict(rescale=False)],
    ids=["block64", "e_minus_8", "g_scale_2^-5", "g_scale_2^-7", "no_rescale"])
def test_emulate_reduced_mistakes_are_caught(monkeypatch, variant):
    import tests.test_oracle_quant as Q
    # the unmutated function passes the worked case ...
    Q.test_emulate_reduced_worked_case()
    # ... and each mutation fails it
    _patch(monkeypatch, "emulate_reduced", _emulate_variant(**variant))
    with pytest.raises(AssertionError):
        Q.test_emulate_reduced_worked_case()


def test_shifted_row_of_nonzero_is_caught_by_scipy_cross_check(monkeypatch):
    # every stored entry attributed to the row after its own (the last row's
    # entries wrap to row 0): S X and the CSR adjoint must then disagree
    # with scipy.sparse's own CSR expansion
    orig = OC.row_of_nonzero

    def shifted(row_ptr):
        r = orig(row_ptr)
        n = len(row_ptr) - 1
        return (r + 1) % max(n, 1)

    _patch(monkeypatch, "row_of_nonzero", shifted)
    with pytest.raises(AssertionError):
        S.test_csr_oracle_matches_scipy_sparse_product()
    with pytest.raises(AssertionError):
        S.test_csr_adjoint_matches_scipy_sparse_transpose()


# ---- the dense Gaussian product, Algorithm 1 and Section 7 quantities ----
import oracle.anchors as OA  # noqa: E402
import oracle.lowerbound as OL  # noqa: E402
import tests.test_oracle_anchors as A  # noqa: E402
import tests.test_oracle_gaussian as GQ  # noqa: E402
import tests.test_oracle_lowerbound as LBT  # noqa: E402


def test_gaussian_product_csr_dropping_the_last_row_is_caught(monkeypatch):
    orig = OC.gaussian_product_csr

    def dropped(row_ptr, col_idx, vals, n, d, m, seed, row_offset=0, chunk=1 << 15):
        rp = np.array(row_ptr, copy=True)
        k = int(rp[-2])
        return orig(rp[:-1], col_idx[:k], vals[:k], n - 1, d, m, seed, row_offset, chunk)

    _patch(monkeypatch, "gaussian_product_csr", dropped)
    with pytest.raises(AssertionError):
        GQ.test_csr_form_matches_scipy_sparse_product()


def test_gaussian_product_with_half_variance_is_caught(monkeypatch):
    orig = OC.gaussian_product_dense

    def halved(X, m, seed, row_offset=0, chunk=1 << 15):
        return orig(X, m, seed, row_offset, chunk) * np.sqrt(0.5)

    _patch(monkeypatch, "gaussian_product_dense", halved)
    with pytest.raises(AssertionError):
        GQ.test_squared_norm_is_chi_square_m()


def test_row_extrema_taking_the_last_tie_is_caught(monkeypatch):
    def last_tie(Z):
        Z = np.asarray(Z, dtype=np.float64)
        m, d = Z.shape
        rev = Z[:, ::-1]
        return (d - 1 - np.argmax(rev, axis=1)), (d - 1 - np.argmin(rev, axis=1))

    monkeypatch.setattr(OA, "row_extrema", last_tie)
    monkeypatch.setattr(O, "row_extrema", last_tie)
    with pytest.raises(AssertionError):
        A.test_row_extrema_hand_worked_fixture()


def test_kl_without_log_determinant_is_caught(monkeypatch):
    def no_logdet(M):
        w = np.linalg.eigvalsh(np.asarray(M, dtype=np.float64))
        return 0.5 * (float(np.sum(1.0 / w)) - len(w))

    monkeypatch.setattr(OL, "kl_to_standard", no_logdet)
    with pytest.raises(AssertionError):
        LBT.test_kl_matches_quadrature_in_one_dimension()


def test_pair_statistic_against_m_instead_of_2m_is_caught(monkeypatch):
    def wrong(Y, m):
        P = OL.pair_norms(Y)
        vals = P[np.isfinite(P)]
        return float(np.max(np.abs(vals - m))) if vals.size else 0.0

    monkeypatch.setattr(OL, "pair_deviation", wrong)
    with pytest.raises(AssertionError):
        LBT.test_pair_deviation_hand_worked()
