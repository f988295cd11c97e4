"""The roofline arithmetic of bench.py without a GPU: the algorithmic work of the fused score (Section III-A
Eq. 4 per control-point evaluation, Section II-B Eq. 3 per pair), the instruction-priced ceiling, the ceiling
from measured issue rates (which must reduce to the instruction-priced one at the published rates), and the
HBM-traffic gate on the counters' source hash."""
import hashlib
import os

import pytest

from conftest import ROOT

import bench

CUS, CLOCK = 256, 2.4e9


def test_score_flops_of_the_benchmark_workload():
    # 7 moving control points, S = 4,000 supports, N = 1,000,000 queries:
    # per cp-eval 3 products + 2 adds for p.p', 2 more terms and a scale for t, a square and an accumulate
    # (10); per pair the reciprocal step and the alpha weighting (2)
    per_pair = 7 * 10 + 2
    assert bench.score_flops(7, 4000, 1_000_000) == pytest.approx(4000 * 1_000_000 * per_pair, rel=1e-15)
    assert bench.score_flops(7, 4000, 1_000_000) == pytest.approx(2.88e11, rel=1e-12)
    assert bench.score_flops(7, 0, 1_000_000) == 0.0


@pytest.mark.parametrize("Mm", [1, 3, 7, 16])
def test_instruction_ceiling_from_instruction_counts(Mm):
    """Units of 1/128 CU clock per (support, query) pair, counted by instruction class as the profiled counters
    record them: the matrix unit does 4 Mm MACs (x, y, z and the norm term of every moving point); the
    running fraction takes 2 Mm multiplies (Mm squares, Mm - 1 denominator products, one quotient), Mm FMAs
    (Mm - 1 numerator steps, one weighting) and one reciprocal at a quarter rate; the saturated form Mm
    reciprocals, Mm FMAs and one weighting FMA."""
    rational_units = 4 * Mm + 2 * Mm + Mm + 4 * 1
    saturated_units = 4 * Mm + 4 * Mm + Mm + 1
    assert bench.alu_peak(Mm, True) == pytest.approx(CUS * CLOCK * 128 * Mm / rational_units, rel=1e-12)
    assert bench.alu_peak(Mm, False) == pytest.approx(CUS * CLOCK * 128 * Mm / saturated_units, rel=1e-12)
    if Mm == 7:
        assert bench.alu_peak(7, True) == pytest.approx(10.39e12, rel=1e-3)
        assert bench.alu_peak(7, False) == pytest.approx(8.60e12, rel=1e-3)


def _published_peaks(mix_cycles=2.0):
    """Issue rates at the published figures: wave64 vector op in 2 cycles, reciprocal in 8, FP32 16x16x4 MFMA
    in 32, every probe at 2.4 GHz."""
    row = lambda cycles: {"4_waves_per_simd": {"cycles_per_instruction": cycles, "clock_ghz": 2.4}}
    return {"v_mfma_f32_16x16x4_f32": row(32.0), "v_mul_f32": row(2.0), "v_rcp_f32": row(8.0),
            "mfma_f32+8 v_mul_f32": {"4_waves_per_simd": {"cycles_per_vector_op_beyond_matrix": mix_cycles,
                                                          "clock_ghz": 2.4}}}


@pytest.mark.parametrize("rational", [True, False])
@pytest.mark.parametrize("Mm", [1, 7, 16])
def test_measured_ceiling_reduces_to_the_instruction_ceiling(Mm, rational):
    out = bench.measured_ceiling(_published_peaks(), Mm, rational, achieved_cp=1e12)
    for form in ("isolated_rates", "mixed_stream_rates"):
        assert out[form]["cp_evals_per_s"] == pytest.approx(bench.alu_peak(Mm, rational), rel=1e-12)
        assert out[form]["frac"] == pytest.approx(1e12 / bench.alu_peak(Mm, rational), rel=1e-12)
    # slower vector issue beside the matrix unit can only lower the mixed-stream ceiling
    slow = bench.measured_ceiling(_published_peaks(mix_cycles=3.0), Mm, rational, achieved_cp=1e12)
    assert slow["mixed_stream_rates"]["cp_evals_per_s"] < out["mixed_stream_rates"]["cp_evals_per_s"]
    assert slow["isolated_rates"]["cp_evals_per_s"] == pytest.approx(out["isolated_rates"]["cp_evals_per_s"])


def test_traffic_is_gated_on_the_counted_sources_and_workload():
    assert bench.score_traffic(7, 4000, 999_999) is None
    assert bench.score_traffic(8, 4000, 1_000_000) is None
    h = hashlib.sha256()
    for rel in bench.SCORE_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    t = bench.score_traffic(7, 4000, 1_000_000)
    if h.hexdigest()[:16] != bench.SCORE_COUNTERS["src_sha256_16"]:
        assert t is None  # sources changed since the counters were taken: reported as null
        return
    # algorithmic bytes: the queries (7 float32 each), the packed model (a 256-byte header with the constant
    # term, then 250 tiles of 656 float32) and the outputs (float32 score + int8 label); every one must be
    # moved, and beyond them at most one copy of the model per XCD L2 (8)
    model = 256 + 250 * 656 * 4
    algorithmic = 1_000_000 * 7 * 4 + model + 1_000_000 * 5
    assert algorithmic == 33_656_256
    assert algorithmic <= t <= algorithmic + 8 * model
