"""Sizing from a target false-positive rate (the library's host-side model
and its inversion) against the oracle's fp64 model; no device work."""

import math

import pytest

import oracle.fpr as fpr

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2101_01719_amd as P

    P._L()
    return P


@pytest.mark.parametrize("a", [0.01, 0.5, 1.0, 5.0, 10.0, 20.0, 23.84, 31.5, 52.0, 100.0, 400.0])
def test_model_matches_oracle(P, a):
    got, ref = P.sbbf_fpr_model(a), fpr.sbbf_fpr(a)
    assert got == pytest.approx(ref, rel=1e-12, abs=1e-300)


def test_model_zero_load(P):
    assert P.sbbf_fpr_model(0.0) == 0.0


def _same_or_tie(B, ref, n, target, lanes=8):
    """The library's inversion equals the oracle's (pinned exactly on the CPU).
    The two sum the same series in fp64 in their own order, so they may differ
    by one block only where the model at the boundary equals the target to
    within fp64 rounding."""
    if B == ref:
        return
    assert abs(B - ref) == 1
    assert abs(fpr.sbbf_fpr(n / min(B, ref), lanes) / target - 1.0) < 1e-12


def _bracketed(n, target, B):
    """B is the oracle's answer up to fp64 rounding at the boundary."""
    ok_at = fpr.sbbf_fpr(n / B) <= target * (1 + 1e-12)
    ok_below = B == 1 or fpr.sbbf_fpr(n / (B - 1)) > target * (1 - 1e-12)
    return ok_at and ok_below


@pytest.mark.parametrize("n,target", [(1, 0.5), (1000, 0.01), (100_000, 0.0103), (1_000_000, 0.0274),
                                      (100_000_000, 0.0091), (123_457, 0.004), (10**9, 0.19), (50_000, 0.001)])
def test_blocks_for_fpr_matches_oracle(P, n, target):
    B = P.sbbf_blocks_for_fpr(n, target)
    assert _bracketed(n, target, B)
    _same_or_tie(B, fpr.blocks_for_fpr(n, target), n, target)


def test_blocks_for_fpr_band_endpoints(P):
    # The paper's band endpoints: 20 hashes per block gives about 0.4 %,
    # 52 about 19 %; aiming just above F(20) with 20 * 4096 keys gives 4096 blocks.
    n = 20 * 4096
    assert P.sbbf_blocks_for_fpr(n, fpr.sbbf_fpr(20.0) * (1 + 1e-9)) == 4096
    n = 52 * 1000
    assert P.sbbf_blocks_for_fpr(n, fpr.sbbf_fpr(52.0) * (1 + 1e-9)) == 1000


def test_blocks_for_fpr_table_geometry(P):
    # 1e8 keys at the rate the model gives for the evaluation table's
    # 4,194,304 blocks asks for (about) that many blocks.
    target = fpr.sbbf_fpr(1e8 / 4_194_304) * (1 + 1e-9)
    assert P.sbbf_blocks_for_fpr(100_000_000, target) == 4_194_304


def test_blocks_for_fpr_errors(P):
    assert P.sbbf_blocks_for_fpr(0, 0.01) == 1
    for bad in (0.0, 1.0, -0.5, 2.0, math.nan):
        with pytest.raises(P.SbbfError):
            P.sbbf_blocks_for_fpr(1000, bad)
    with pytest.raises(P.SbbfError):
        P.sbbf_blocks_for_fpr(2**62, 1e-6)  # needs more than 2^32 - 1 blocks


@pytest.mark.parametrize("lanes", [4, 8, 16])
@pytest.mark.parametrize("a", [0.01, 1.0, 12.2, 24.38, 48.8, 100.0])
def test_variant_model_matches_oracle(P, lanes, a):
    got, ref = P.sbbf_fpr_model_variant(a, lanes), fpr.sbbf_fpr(a, lanes)
    assert got == pytest.approx(ref, rel=1e-12, abs=1e-300)
    if lanes == 8:
        assert got == P.sbbf_fpr_model(a)


@pytest.mark.parametrize("lanes", [4, 16])
@pytest.mark.parametrize("n,target", [(1000, 0.01), (1_000_000, 0.0274), (100_000_000, 0.0091), (50_000, 0.001)])
def test_variant_blocks_for_fpr_matches_oracle(P, lanes, n, target):
    B = P.sbbf_blocks_for_fpr_variant(n, target, lanes)
    assert fpr.sbbf_fpr(n / B, lanes) <= target * (1 + 1e-12)
    assert B == 1 or fpr.sbbf_fpr(n / (B - 1), lanes) > target * (1 - 1e-12)
    _same_or_tie(B, fpr.blocks_for_fpr(n, target, lanes=lanes), n, target, lanes)


def test_variant_sizing_errors(P):
    for bad in (0, 3, 5, 32):
        with pytest.raises(P.SbbfError):
            P.sbbf_fpr_model_variant(10.0, bad)
        with pytest.raises(P.SbbfError):
            P.sbbf_blocks_for_fpr_variant(1000, 0.01, bad)
    assert P.sbbf_serialized_bytes_variant(10, 4) == 32 + 160
    assert P.sbbf_serialized_bytes_variant(10, 16) == 32 + 640
    assert P.sbbf_serialized_bytes_variant(10, 3) == 0
