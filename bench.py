"""Benchmark: proxy collision checks/s of Fastron with the FK kernel on one MI355X.

Workload (7-DOF D-H arm, M = 8 control points, S = 4,000 support points with
alpha ~ N(0, 1), N = 1,000,000 query configurations uniform in [-pi, pi]^7,
gamma = 10). One step = the whole scoring path for one batch: prepare the
support set (FK of the supports, scaled operands, alpha / M) and score every
query (FK of the query fused with K_FK against all supports, weighted sum,
sign). Inputs are resident in device memory before timing starts.

Also reported on the same line: the fused score kernel's roofline position
(its own average duration from HIP events on the launch stream), the
precision and VALU forms, a full Algorithm 1 training run on 50,000 labelled
samples, and the CPU FP64 oracle timed on a bounded sample of the same
workload (which also gives the sign agreement with FP64).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Roofline of the FP32 fused score against the published FP32 peak
# (157.3 TFLOP/s: 256 CUs x 2.4 GHz x 256 FLOP/clk/CU, the vector and the
# matrix unit alike). Algorithmic work per control-point evaluation (cp-eval,
# one K_RQ): the squared distance and t = 1 + gamma/2 d^2 as a 3-term dot
# product plus the norms, 8 FLOP, and the square-and-accumulate of 1/t^2,
# 2 FLOP (the reciprocal itself is a transcendental, not counted); per
# (support, query) pair the alpha/M weighting adds 2 FLOP. Fixed base-frame
# points add exactly 1/M per pair and are folded into a constant, so only the
# Mm moving points count.
FP32_PEAK_TFLOPS = 157.3


def score_flops(Mm, S, N):
    return N * S * (10.0 * Mm + 2.0)


# Instruction-priced ALU ceiling of the same kernel, in cp-evals per second:
# the instructions one pair with Mm moving points needs, priced at the
# published rates (FP32 MFMA and vector FMA 128 lanes/clk/CU; transcendentals
# 32 lanes/clk/CU) with the matrix and vector units not overlapping. In units
# of 1/128 CU clock per pair:
#   cross term with the norms on the matrix unit        4 Mm
#   saturated-reciprocal sum: Mm reciprocals (4 each) + Mm FMAs + 1 weighting FMA
#                                                      -> 9 Mm + 1 in all
#   running-fraction sum: Mm squares + 2 (Mm - 1) for numerator and
#   denominator + one reciprocal (4) + the quotient + 1 weighting FMA
#                                                      -> 7 Mm + 4 in all
# e.g. Mm = 7: 8.60e12 (saturated) and 10.39e12 (fraction) cp-evals/s.
def alu_peak(Mm, rational):
    return 256 * 2.4e9 * 128 * Mm / ((7 * Mm + 4) if rational else (9 * Mm + 1))


# HBM bytes per launch of the FP32 score kernel on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), each scaled
# by what the same counter reads for a plain 256 MiB device copy (FETCH_SIZE
# reads 131,083.5 KiB for 262,144 KiB moved, WRITE_SIZE 262,144 KiB). The
# figures hold for the kernel sources whose hash is recorded here; once those
# change, the counters must be taken again and traffic is reported as null.
SCORE_COUNTERS = {
    "src_sha256_16": "7e0768eb387c2dbc",
    "workload": (7, 4000, 1_000_000),  # (M_moving, S, N)
    "fetch_kib": 16294.875, "fetch_scale": 262144.0 / 131083.5,
    "write_kib": 4882.8125, "write_scale": 1.0,
}
SCORE_SOURCES = ("paper_1910_06451_amd/csrc/score.hip", "paper_1910_06451_amd/csrc/score_device.h",
                 "paper_1910_06451_amd/csrc/model_layout.h", "paper_1910_06451_amd/csrc/fastron_internal.h",
                 "paper_1910_06451_amd/build.py")


def score_traffic(Mm, S, N):
    """Measured HBM bytes per score launch, or None if the counters do not cover this kernel build."""
    import hashlib
    h = hashlib.sha256()
    for rel in SCORE_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    c = SCORE_COUNTERS
    if h.hexdigest()[:16] != c["src_sha256_16"] or (Mm, S, N) != c["workload"]:
        return None
    return 1024.0 * (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)  # the clocks ramp over the first ~30 ms of work
    ap.add_argument("--S", type=int, default=4000)
    ap.add_argument("--N", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the main metric (for profiling runs)")
    ap.add_argument("--legs",
                    default="peaks,kernels,forms,precision,dof3,train,compare,obstacles,active,batched,retrain,mlp,"
                            "screen",
                    help="comma-separated extra legs (peaks, kernels, forms, precision, dof3, train, compare, "
                         "obstacles, active, batched, retrain, mlp, screen)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--mlp-epochs", type=int, default=10, help="epochs of the screening network in the extras")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (there is no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    legs = set() if args.no_extras else {x.strip() for x in args.legs.split(",") if x.strip()}
    unknown = legs - {"peaks", "mlp", "kernels", "forms", "precision", "dof3", "train", "compare", "obstacles", "active", "batched",
                      "retrain", "screen"}
    if unknown:
        print(f"unknown legs: {sorted(unknown)}", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1910_06451_amd import api, workloads as wl

    dev = torch.device("cuda:0")
    arm = wl.arm_7dof()
    gamma, S, N = 10.0, args.S, args.N
    sq_np, al_np = wl.model("bench7", S, arm.n)
    q_np = wl.configs("bench7/q", N, arm.n)
    sq, al, q = (torch.from_numpy(x).to(dev) for x in (sq_np, al_np, q_np))
    f = torch.empty(N, dtype=torch.float32, device=dev)
    lab = torch.empty(N, dtype=torch.int8, device=dev)
    Mm = int(np.sum(arm.frames > 0))  # control points that move; base-frame points are folded exactly

    def step():
        api.fk_score(arm, sq, al, gamma, q, out=(f, lab))

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        marks[i].record()
        step()
    marks[-1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    step_ms = [marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps)]
    checks_per_s = N / (ms * 1e-3)

    # dominant kernel alone: score against a prepared model, timed with events on the launch stream
    model = api.support_prep(arm, sq, al, gamma)
    stream = torch.cuda.current_stream()

    def kernel_ms(flags, reps):
        for _ in range(2):
            api.fk_score_prepared(arm, model, q, flags=flags, out=(f, lab))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            api.fk_score_prepared(arm, model, q, flags=flags, out=(f, lab))
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    def kernel_spread(flags, reps):
        """Per-launch durations from an event pair around each launch: (median, min)."""
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            api.fk_score_prepared(arm, model, q, flags=flags, out=(f, lab))
            b.record(stream)
        torch.cuda.synchronize()
        per = [a.elapsed_time(b) for a, b in ev]
        return float(np.median(per)), float(np.min(per))

    k_ms = kernel_ms(api.SCORE_FP32, args.steps)
    k_med, k_min = kernel_spread(api.SCORE_FP32, max(20, args.steps))
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cp_per_launch = N * S * Mm
    achieved = cp_per_launch / (k_ms * 1e-3)
    rational = api.score_rational(arm, gamma)
    peak = alu_peak(Mm, rational)
    tflops = score_flops(Mm, S, N) / (k_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": tflops / FP32_PEAK_TFLOPS, "traffic": score_traffic(Mm, S, N),
                "flops_per_launch": score_flops(Mm, S, N),
                "flops_per_unit": "10 per cp-eval (dot product + t: 8, square-accumulate: 2) + 2 per pair",
                "cp_evals_per_s": achieved, "instruction_ceiling_cp_evals_per_s": peak,
                "frac_of_instruction_ceiling": achieved / peak,
                "sum_form": "running fraction" if rational else "saturated reciprocal",
                "traffic_unit": "HBM bytes per launch",
                # queries (n floats each) + the FP32 part of the packed support set (256 B header,
                # 16-support tiles of 80 * Mp + 16 floats) + outputs (float score + int8 label)
                "algorithmic_bytes": N * arm.n * 4 + 256 + -(-S // 16) * (80 * ((arm.M + 3) & ~3) + 16) * 4 + N * 5,
                "kernel": f"k_score_mfma<{Mm},double>", "kernel_ms": k_ms,
                "kernel_ms_median": k_med, "kernel_ms_min": k_min, "cp_evals_per_launch": cp_per_launch}
    f_gpu = f.clone()
    lab_gpu = lab.cpu().numpy()
    f_np = f_gpu.cpu().numpy()

    extras = {}
    checks = []  # GPU results queued for the FP64 comparison of the CPU leg
    if "peaks" in legs:
        log("[bench] issue-rate probes and device copy")
        extras["peaks"] = peaks_run(dev)
        roofline["measured_ceiling"] = measured_ceiling(extras["peaks"], Mm, rational, achieved)
    if "kernels" in legs:
        log("[bench] FK, Gram-column and labeller kernels on 4,194,304 configurations")
        extras["kernels"] = kernels_run(api, wl, arm, dev)
    if "forms" in legs:
        forms = {}
        for name, flags in (("valu", api.SCORE_VALU), ("bf16_plain", api.SCORE_BF16 | api.BF16_PLAIN),
                            ("bf16_split3", api.SCORE_BF16 | api.BF16_SPLIT3)):
            log(f"[bench] form {name}")
            t = kernel_ms(flags, max(3, args.steps // 4))
            forms[name] = {"kernel_ms": t, "checks_per_s": N / (t * 1e-3), "vs_fp32": k_ms / t,
                           "labels": lab.cpu().numpy()}
        extras["forms"] = forms
    if "precision" in legs:
        log("[bench] precision form: S=16,384, N=4,194,304")
        extras["precision"] = precision_run(api, wl, arm, gamma, dev, checks)
    if "dof3" in legs:
        log("[bench] 3-DOF workload: FP64 training on 2,000 labelled samples, scoring")
        extras["dof3"] = dof3_run(api, wl, dev, checks)
    if "train" in legs:
        log("[bench] training run on 50,000 labelled samples")
        extras["train"] = train_run(api, wl, arm, dev)
    if "compare" in legs:
        log("[bench] FK kernel vs kernel on configurations")
        extras["compare"] = compare_run(api, wl, arm, dev, checks)
    if "obstacles" in legs:
        log("[bench] obstacle-count sweep")
        extras["obstacles"] = obstacles_run(api, wl, arm, dev, checks)
    if "active" in legs:
        log("[bench] moving obstacle: model updates after two-stage active learning")
        extras["active"] = active_run(api, wl, arm, dev)
    if "batched" in legs:
        log("[bench] batched form: 256 environments")
        extras["batched"] = batched_run(api, wl, arm, gamma, dev, checks)
    if "retrain" in legs:
        log("[bench] re-training 16 environments after their cubes move")
        extras["retrain16"] = retrain_run(api, wl, arm, dev)
    if "mlp" in legs:
        log("[bench] screening network training step")
        extras["mlp_train"] = mlp_run(api, wl, arm, dev)
    if "screen" in legs:
        log("[bench] learned screening (MLP + tau fallback)")
        extras["screen"] = screen_run(api, wl, arm, dev, epochs=args.mlp_epochs)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (FP64 oracle)")
        cpu, agree = cpu_baseline(arm, sq_np, al_np, q_np, gamma, f_np, lab_gpu, args.cpu_seconds, extras, checks)
    else:
        agree = {}

    out = {
        "metric": "proxy collision checks/s (7-DOF, fused FK + FK-kernel score + sign)",
        "value": checks_per_s,
        "unit": "checks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "step_ms_median": float(np.median(step_ms)),
        "step_ms_min": float(np.min(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded D-H arm, uniform configurations, alpha ~ N(0,1))",
        "config": {"workload": "7-DOF arm, M=8 control points, S=4000 supports, N=1,000,000 queries, gamma=10",
                   "S": S, "N": N, "M": int(arm.M), "M_moving": Mm, "gamma": gamma},
        "kernel_evals_per_s": N * S / (ms * 1e-3),
        "cp_evals_per_s": N * S * Mm / (ms * 1e-3),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(agree)
    if extras:
        for v in extras.get("forms", {}).values():
            v.pop("labels", None)
        out["extras"] = extras
    print(json.dumps(out), flush=True)


def peaks_run(dev, copy_bytes=256 << 20):
    """Issue rates measured on this device (probe/peaks.hip): each instruction kind alone in independent
    chains, at 2, 4 and 8 waves per SIMD, in SIMD cycles per wave64 instruction at the clock the kernel ran
    (shader clock counter against the 100 MHz constant clock); mixed rounds of one matrix instruction and 8
    vector multiplies; and a plain device copy of copy_bytes."""
    import ctypes

    import torch

    from paper_1910_06451_amd import build as hb

    lib = ctypes.CDLL(hb.PROBE_LIB)
    names = ["v_mul_f32", "v_fma_f32", "v_rcp_f32", "v_mfma_f32_16x16x4_f32", "v_mfma_f32_16x16x32_bf16",
             "mfma_f32+8 v_mul_f32", "mfma_bf16+8 v_mul_f32", "8 v_mul_f32+v_rcp_f32"]
    iters = [4000, 4000, 1200, 600, 1200, 500, 600, 3000]
    out = {}
    for kind, name in enumerate(names):
        vo, mo = ctypes.c_int(0), ctypes.c_int(0)
        lib.probe_ops_per_iter(kind, ctypes.byref(vo), ctypes.byref(mo))
        rows = {}
        for wps in (2, 4, 8):
            ms, cyc, tck, ncu = ctypes.c_double(0), ctypes.c_ulonglong(0), ctypes.c_ulonglong(0), ctypes.c_int(0)
            rc = lib.probe_run(kind, wps, iters[kind], ctypes.byref(ms), ctypes.byref(cyc), ctypes.byref(tck),
                               ctypes.byref(ncu))
            if rc != 0:
                raise RuntimeError(f"probe {name} failed ({rc})")
            ghz = cyc.value / (tck.value / 100e6) / 1e9 if tck.value else float("nan")
            simd_cycles = ms.value * 1e-3 * ghz * 1e9          # cycles each SIMD spent on its waves
            rounds = wps * iters[kind]                          # loop iterations per SIMD
            row = {"ms": ms.value, "clock_ghz": ghz}
            if mo.value and vo.value:
                row["cycles_per_round"] = simd_cycles / rounds / (mo.value // 8 or 1) / 8
                row["cycles_per_vector_op_beyond_matrix"] = None
            elif mo.value:
                row["cycles_per_instruction"] = simd_cycles / (rounds * mo.value)
            else:
                row["cycles_per_instruction"] = simd_cycles / (rounds * vo.value)
            rows[f"{wps}_waves_per_simd"] = row
        out[name] = rows
    # mixed rounds: cost of each vector multiply beyond the matrix instruction's own cycles
    for mixed, alone in (("mfma_f32+8 v_mul_f32", "v_mfma_f32_16x16x4_f32"),
                         ("mfma_bf16+8 v_mul_f32", "v_mfma_f32_16x16x32_bf16")):
        for key, row in out[mixed].items():
            row["cycles_per_vector_op_beyond_matrix"] = (row["cycles_per_round"]
                                                         - out[alone][key]["cycles_per_instruction"]) / 8
    src = torch.ones(copy_bytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    ms = ctypes.c_double(0)
    if lib.probe_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), copy_bytes, 10,
                      ctypes.byref(ms)) != 0:
        raise RuntimeError("probe copy failed")
    out["device_copy"] = {"bytes": copy_bytes, "ms": ms.value, "GB_per_s": 2 * copy_bytes / (ms.value * 1e-3) / 1e9,
                          "frac_of_8TBps": 2 * copy_bytes / (ms.value * 1e-3) / 8e12}
    del src, dst
    return out


def measured_ceiling(peaks, Mm, rational, achieved_cp):
    """Ceiling of the FP32 fused score from the measured issue rates (4 waves per SIMD), each converted to time
    at the clock its own probe ran (the part clocks down under dense vector work), the matrix and vector
    units not overlapping: per (support, query) pair Mm matrix instructions cover 256 pairs each; the running
    fraction takes 3 Mm vector instructions and one reciprocal per pair (the saturated form Mm reciprocals and
    Mm + 1 FMAs), 64 pairs per wave64 instruction. Also the same with the vector multiplies at the rate
    measured beside matrix work (mixed stream, at that probe's clock)."""
    key = "4_waves_per_simd"
    row = lambda name: peaks[name][key]
    c_mfma, f_mfma = row("v_mfma_f32_16x16x4_f32")["cycles_per_instruction"], row("v_mfma_f32_16x16x4_f32")["clock_ghz"]
    c_mul, f_mul = row("v_mul_f32")["cycles_per_instruction"], row("v_mul_f32")["clock_ghz"]
    c_rcp, f_rcp = row("v_rcp_f32")["cycles_per_instruction"], row("v_rcp_f32")["clock_ghz"]
    mix = row("mfma_f32+8 v_mul_f32")
    c_mix, f_mix = mix["cycles_per_vector_op_beyond_matrix"], mix["clock_ghz"]
    vec, rcp = (3 * Mm, 1) if rational else (Mm + 1, Mm)
    simds = 1024
    ns_iso = (Mm * c_mfma / 256 / f_mfma + vec * c_mul / 64 / f_mul + rcp * c_rcp / 64 / f_rcp)  # ns per pair
    ns_mix = (Mm * c_mfma / 256 + vec * c_mix / 64) / f_mix + rcp * c_rcp / 64 / f_rcp
    out = {}
    for name, ns in (("isolated_rates", ns_iso), ("mixed_stream_rates", ns_mix)):
        ceil = simds * Mm / (ns * 1e-9)
        out[name] = {"cp_evals_per_s": ceil, "frac": achieved_cp / ceil}
    out["clock_ghz"] = {"mfma_f32": f_mfma, "v_mul_f32": f_mul, "v_rcp_f32": f_rcp, "mixed": f_mix}
    out["cycles"] = {"mfma_f32": c_mfma, "v_mul_f32": c_mul, "v_rcp_f32": c_rcp, "v_mul_f32_beside_mfma": c_mix}
    return out


# Kernel width for training on geometric labels of the 7-DOF arm, picked by a
# grid search over {10, 30, 100} on 5,000 labelled samples (held-out accuracy
# 0.832 / 0.846 / 0.834), as the paper selects its parameters by grid search.
GAMMA_TRAIN_7DOF = 30.0


def _event_ms(fn, reps, rounds=3):
    """Milliseconds per call of fn from HIP events on the current stream: three warm-up calls, then the
    median over `rounds` rounds of `reps` back-to-back calls."""
    import torch

    for _ in range(3):
        fn()
    stream = torch.cuda.current_stream()
    per = []
    for _ in range(rounds):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        per.append(e0.elapsed_time(e1) / reps)
    return float(np.median(per))


def kernels_run(api, wl, arm, dev, N=4_194_304, reps=10):
    """The HBM-bound kernels of the path against 8 TB/s, and the labeller's rate: batched FK (reads n floats,
    writes 3M floats per configuration), one Gram-column update over N training points (reads 3M floats and
    F, writes F), and capsule-box labels against 20 cubes (FP64)."""
    import torch

    q = torch.from_numpy(wl.configs("kern/q", N, arm.n)).to(dev)
    P = api.fk_points(arm, q)
    F = torch.zeros(N, dtype=torch.float32, device=dev)
    lo, hi = wl.cubes("bench7/cubes", 20, 0.1, 0.25)
    t_fk = _event_ms(lambda: api.fk_points(arm, q), reps)
    t_gram = _event_ms(lambda: api.gram_update_points(P, 10.0, 12345, 0.5, F=F, want_kcol=False), reps)
    t_lab = _event_ms(lambda: api.label_capsule_box(arm, q, arm.radius, lo, hi, want_clearance=False), 3)
    t_clr = _event_ms(lambda: api.label_capsule_box(arm, q, arm.radius, lo, hi, want_clearance=True), 3)
    b_fk = N * (arm.n * 4 + arm.M * 12)
    b_gram = N * (arm.M * 12 + 8)
    hbm = 8.0e12
    return {"N": N,
            "fk_points": {"ms": t_fk, "configs_per_s": N / (t_fk * 1e-3), "bytes": b_fk,
                          "GB_per_s": b_fk / (t_fk * 1e-3) / 1e9, "frac_hbm": b_fk / (t_fk * 1e-3) / hbm},
            "gram_update": {"ms": t_gram, "points_per_s": N / (t_gram * 1e-3), "bytes": b_gram,
                            "GB_per_s": b_gram / (t_gram * 1e-3) / 1e9, "frac_hbm": b_gram / (t_gram * 1e-3) / hbm},
            # (link, box) pairs decided per second, culled ones included
            "label_capsule_box": {"ms": t_lab, "configs_per_s": N / (t_lab * 1e-3),
                                  "link_box_pairs_per_s": N * arm.n * 20 / (t_lab * 1e-3),
                                  "ms_with_clearance": t_clr, "configs_per_s_with_clearance": N / (t_clr * 1e-3)}}


def precision_run(api, wl, arm, gamma, dev, checks, S=16_384, N=4_194_304, fp64_sample=1_048_576, reps=5):
    """FP32 score versus the BF16 cross-term forms on S = 16,384 supports and N = 4,194,304 queries: kernel time
    of each form, max |df| and sign agreement against the FP32 path (all queries); an evenly spaced sample of
    fp64_sample queries of every form is queued for the FP64 comparison of the CPU leg."""
    import torch

    sq_np, al_np = wl.model("prec7", S, arm.n)
    q_np = wl.configs("prec7/q", N, arm.n)
    sq, al, q = (torch.from_numpy(x).to(dev) for x in (sq_np, al_np, q_np))
    model = api.support_prep(arm, sq, al, gamma)
    forms = {"fp32": api.SCORE_FP32, "bf16_plain": api.SCORE_BF16 | api.BF16_PLAIN,
             "bf16_split2": api.SCORE_BF16 | api.BF16_SPLIT2, "bf16_split3": api.SCORE_BF16 | api.BF16_SPLIT3}
    res, outs = {}, {}
    for name, flags in forms.items():
        f = torch.empty(N, dtype=torch.float32, device=dev)
        lab = torch.empty(N, dtype=torch.int8, device=dev)
        t = _event_ms(lambda: api.fk_score_prepared(arm, model, q, flags=flags, out=(f, lab)), reps)
        outs[name] = (f, lab)
        res[name] = {"kernel_ms": t, "checks_per_s": N / (t * 1e-3),
                     "cp_evals_per_s": N * S * int(np.sum(arm.frames > 0)) / (t * 1e-3)}
    f32, l32 = outs["fp32"]
    idx = np.linspace(0, N - 1, fp64_sample).astype(np.int64)
    for name, (f, lab) in outs.items():
        res[name]["vs_fp32"] = {"max_abs_df": float((f - f32).abs().max()),
                                "sign_agreement": float((lab == l32).float().mean())}
        res[name]["speed_vs_fp32"] = res["fp32"]["kernel_ms"] / res[name]["kernel_ms"]
        checks.append({"arm": arm, "sq": sq_np, "al": al_np, "gamma": gamma, "q": q_np[idx],
                       "f": f.cpu().numpy()[idx], "lab": lab.cpu().numpy()[idx], "into": res[name]})
    return {"S": S, "N": N, "fp64_sample": fp64_sample, "forms": res}


def dof3_run(api, wl, dev, checks, reps=20):
    """The 3-DOF workload: 2,000 configurations labelled against 5 cubes of side 0.15 (the first seed whose labels
    are 10-90 % in collision), Algorithm 1 in FP64 on the device (gamma = 10), then the model scores 10,000 fresh
    queries (accuracy / TPR / TNR against their geometric labels) and, for throughput, 1,000,000 queries."""
    import torch

    arm = wl.arm_3dof()
    for seed in range(wl.MASTER_SEED, wl.MASTER_SEED + 200):
        q = torch.from_numpy(wl.configs("train3", 2000, arm.n, seed=seed)).to(dev)
        lo, hi = wl.cubes("train3/cubes", 5, 0.15, None, seed=seed)
        y, _ = api.label_capsule_box(arm, q, arm.radius, lo, hi, want_clearance=False)
        frac = float((y == 1).float().mean())
        if 0.1 <= frac <= 0.9:
            break
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = api.train_points(api.fk_points(arm, q), y, 10.0, fp64=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    sup = out["support"].long()
    al = out["alpha"][sup].float().contiguous()
    model = api.support_prep(arm, q[sup].contiguous(), al, 10.0)
    qq = torch.from_numpy(wl.configs("train3/queries", 10_000, arm.n, seed=seed)).to(dev)
    yq, _ = api.label_capsule_box(arm, qq, arm.radius, lo, hi, want_clearance=False)
    f = torch.empty(10_000, dtype=torch.float32, device=dev)
    lab = torch.empty(10_000, dtype=torch.int8, device=dev)
    t_q = _event_ms(lambda: api.fk_score_prepared(arm, model, qq, out=(f, lab)), reps)
    tp = int(((lab == 1) & (yq == 1)).sum()); tn = int(((lab == -1) & (yq == -1)).sum())
    pos = int((yq == 1).sum()); neg = int((yq == -1).sum())
    N = 1_000_000
    qb = torch.from_numpy(wl.configs("dof3/q", N, arm.n)).to(dev)
    fb = torch.empty(N, dtype=torch.float32, device=dev)
    lb = torch.empty(N, dtype=torch.int8, device=dev)
    t_b = _event_ms(lambda: api.fk_score_prepared(arm, model, qb, out=(fb, lb)), reps)
    S = int(sup.numel())
    Mm = int(np.sum(arm.frames > 0))
    res = {"seed": seed, "train_collision_rate": frac, "train_ms_fp64": t_train * 1e3, "updates": out["updates"],
           "support": S, "converged": bool(out["converged"]),
           "queries_10k": {"ms": t_q, "accuracy": (tp + tn) / 10_000, "tpr": tp / max(pos, 1), "tnr": tn / max(neg, 1)},
           "throughput_1M": {"ms": t_b, "checks_per_s": N / (t_b * 1e-3), "kernel_evals_per_s": N * S / (t_b * 1e-3),
                             "cp_evals_per_s": N * S * Mm / (t_b * 1e-3),
                             "frac_alu": N * S * Mm / (t_b * 1e-3) / alu_peak(Mm, api.score_rational(arm, 10.0))}}
    checks.append({"arm": arm, "sq": q[sup].cpu().numpy(), "al": al.cpu().numpy(), "gamma": 10.0,
                   "q": qq.cpu().numpy(), "f": f.cpu().numpy(), "lab": lab.cpu().numpy(), "into": res["queries_10k"]})
    return res


def train_run(api, wl, arm, dev):
    """Label 50,000 configurations with the device labeller (20 cubes), FK them, run Algorithm 1."""
    import torch

    N = 50_000
    q = torch.from_numpy(wl.configs("bench7/train", N, arm.n)).to(dev)
    lo, hi = wl.cubes("bench7/cubes", 20, 0.1, 0.25)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y, _ = api.label_capsule_box(arm, q, arm.radius, lo, hi, want_clearance=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    P = api.fk_points(arm, q)
    out = api.train_points(P, y, GAMMA_TRAIN_7DOF)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return {"N": N, "gamma": GAMMA_TRAIN_7DOF, "label_ms": (t1 - t0) * 1e3, "train_ms": (t2 - t1) * 1e3,
            "updates": out["updates"], "support": int(out["support"].numel()), "converged": bool(out["converged"]),
            "us_per_update": (t2 - t1) * 1e6 / max(out["updates"], 1),
            "collision_rate": float((y == 1).float().mean().item())}


GAMMA_CONFIG_7DOF = 10.0  # the kernel on configurations: grid search over {0.1, 0.3, 1, 3, 10, 30, 100}


def rbf_peak(n):
    """ALU ceiling of the configuration-space score, pair evaluations per second: per pair ceil((n + 1) / 4)
    FP32 MFMA steps of 4 lanes-worth each, one saturated reciprocal (4), its square and the weighting FMA (1
    each), in 1/128 CU clock at the published rates (see alu_peak)."""
    return 256 * 2.4e9 * 128 / (4 * ((n + 1 + 3) // 4) + 6)


def compare_run(api, wl, arm, dev, checks, reps=5):
    """The paper's comparison of the FK kernel with the kernel on configurations (Section IV): both models
    trained by Algorithm 1 on the same 50,000 device-labelled configurations (20 cubes), each with the kernel
    parameter its own grid search chose, then checked against the geometric labels of 100,000 held-out
    configurations and timed on the 1,000,000 benchmark queries."""
    import torch

    N, NT, NQ = 50_000, 100_000, 1_000_000
    q = torch.from_numpy(wl.configs("bench7/train", N, arm.n)).to(dev)
    lo, hi = wl.cubes("bench7/cubes", 20, 0.1, 0.25)
    y, _ = api.label_capsule_box(arm, q, arm.radius, lo, hi, want_clearance=False)
    qt = torch.from_numpy(wl.configs("bench7/heldout", NT, arm.n)).to(dev)
    yt, _ = api.label_capsule_box(arm, qt, arm.radius, lo, hi, want_clearance=False)
    yt_np = yt.cpu().numpy()
    qq = torch.from_numpy(wl.configs("bench7/q", NQ, arm.n)).to(dev)
    f = torch.empty(NQ, dtype=torch.float32, device=dev)
    lab = torch.empty(NQ, dtype=torch.int8, device=dev)

    def metrics(pred):
        pos, neg = yt_np == 1, yt_np == -1
        return {"accuracy": float(np.mean(pred == yt_np)), "tpr": float(np.mean(pred[pos] == 1)),
                "tnr": float(np.mean(pred[neg] == -1))}

    res = {"N_train": N, "N_heldout": NT, "N_queries": NQ}
    # FK kernel
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = api.train_points(api.fk_points(arm, q), y, GAMMA_TRAIN_7DOF)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    sup = out["support"].long()
    model = api.support_prep(arm, q[sup].contiguous(), out["alpha"][sup].contiguous(), GAMMA_TRAIN_7DOF)
    _, lt = api.fk_score_prepared(arm, model, qt)
    ms = _event_ms(lambda: api.fk_score_prepared(arm, model, qq, out=(f, lab)), reps)
    S = int(sup.numel())
    res["fk"] = {"gamma": GAMMA_TRAIN_7DOF, "support": S, "updates": out["updates"], "converged": bool(out["converged"]),
                 "train_ms": t_train * 1e3, **metrics(lt.cpu().numpy()), "query_ms_1M": ms,
                 "checks_per_s": NQ / (ms * 1e-3), "kernel_evals_per_s": NQ * S / (ms * 1e-3)}
    # kernel on configurations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = api.rbf_train(q, y, GAMMA_CONFIG_7DOF)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    sup = out["support"].long()
    sx, sa = q[sup].contiguous(), out["alpha"][sup].contiguous()
    _, lt = api.rbf_score(sx, sa, GAMMA_CONFIG_7DOF, qt)
    ms = _event_ms(lambda: api.rbf_score(sx, sa, GAMMA_CONFIG_7DOF, qq, out=(f, lab)), reps)
    S = int(sup.numel())
    kev = NQ * S / (ms * 1e-3)
    res["configurations"] = {"gamma": GAMMA_CONFIG_7DOF, "support": S, "updates": out["updates"],
                             "converged": bool(out["converged"]), "train_ms": t_train * 1e3,
                             **metrics(lt.cpu().numpy()), "query_ms_1M": ms, "checks_per_s": NQ / (ms * 1e-3),
                             "kernel_evals_per_s": kev, "frac_alu": kev / rbf_peak(arm.n)}
    idx = np.linspace(0, NQ - 1, 2000).astype(np.int64)
    checks.append({"kind": "configurations", "sq": sx.cpu().numpy(), "al": sa.cpu().numpy(),
                   "gamma": GAMMA_CONFIG_7DOF, "q": qq[idx].cpu().numpy(), "f": f[idx].cpu().numpy(),
                   "lab": lab[idx].cpu().numpy(), "into": res["configurations"]})
    return res


def obstacles_run(api, wl, arm, dev, checks, counts=(1, 5, 10, 20, 30, 50), reps=3):
    """Support-set size, accuracy and query time against the number of obstacles (the paper's obstacle
    study, Section IV): for each count, 20,000 training and 20,000 held-out configurations labelled by the
    device labeller (cubes of side 0.1-0.25 m), both kernels trained by Algorithm 1 and timed on 1,000,000
    queries."""
    import torch

    N, NT, NQ = 20_000, 20_000, 1_000_000
    q = torch.from_numpy(wl.configs("obst/train", N, arm.n)).to(dev)
    qt = torch.from_numpy(wl.configs("obst/heldout", NT, arm.n)).to(dev)
    qq = torch.from_numpy(wl.configs("bench7/q", NQ, arm.n)).to(dev)
    f = torch.empty(NQ, dtype=torch.float32, device=dev)
    lab = torch.empty(NQ, dtype=torch.int8, device=dev)
    P = api.fk_points(arm, q)
    rows = []
    for c in counts:
        lo, hi = wl.cubes(f"obst/cubes{c}", c, 0.1, 0.25)
        y, _ = api.label_capsule_box(arm, q, arm.radius, lo, hi, want_clearance=False)
        yt, _ = api.label_capsule_box(arm, qt, arm.radius, lo, hi, want_clearance=False)
        yt_np = yt.cpu().numpy()
        row = {"cubes": c, "collision_rate": float((yt == 1).float().mean().item())}
        for kind in ("fk", "configurations"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if kind == "fk":
                out = api.train_points(P, y, GAMMA_TRAIN_7DOF)
            else:
                out = api.rbf_train(q, y, GAMMA_CONFIG_7DOF)
            torch.cuda.synchronize()
            t_train = time.perf_counter() - t0
            sup = out["support"].long()
            sx, sa = q[sup].contiguous(), out["alpha"][sup].contiguous()
            if kind == "fk":
                model = api.support_prep(arm, sx, sa, GAMMA_TRAIN_7DOF)
                _, lt = api.fk_score_prepared(arm, model, qt)
                ms = _event_ms(lambda: api.fk_score_prepared(arm, model, qq, out=(f, lab)), reps)
            else:
                _, lt = api.rbf_score(sx, sa, GAMMA_CONFIG_7DOF, qt)
                ms = _event_ms(lambda: api.rbf_score(sx, sa, GAMMA_CONFIG_7DOF, qq, out=(f, lab)), reps)
            row[kind] = {"support": int(sup.numel()), "converged": bool(out["converged"]), "updates": out["updates"],
                         "train_ms": t_train * 1e3, "accuracy": float(np.mean(lt.cpu().numpy() == yt_np)),
                         "query_ms_1M": ms, "us_per_query": ms * 1e3 / NQ}
            if c == counts[-1]:  # FP64 check of the last models' scores on 1,000 of the timed queries
                idx = np.linspace(0, NQ - 1, 1000).astype(np.int64)
                chk = {"sq": sx.cpu().numpy(), "al": sa.cpu().numpy(), "q": qq[idx].cpu().numpy(),
                       "f": f[idx].cpu().numpy(), "lab": lab[idx].cpu().numpy(), "into": row[kind]}
                if kind == "fk":
                    checks.append({"arm": arm, "gamma": GAMMA_TRAIN_7DOF, **chk})
                else:
                    checks.append({"kind": "configurations", "gamma": GAMMA_CONFIG_7DOF, **chk})
        rows.append(row)
    return {"N_train": N, "N_heldout": NT, "N_queries": NQ, "rows": rows}


def active_run(api, wl, arm, dev, steps=10, n_init=20_000, k=2, sigma=0.1, n_explore=2_000, n_test=20_000):
    """The moving-obstacle experiment (Section III-B's update, Section IV): a single randomly sized cube moves
    0.05 m along a random direction per step; after each move the model is updated once after two-stage
    active learning (k samples near each support point with N(0, sigma^2) joint noise, n_explore uniform
    samples, geometric labels, F = K alpha, Algorithm 1 warm start) and checked against the labels of n_test
    held-out configurations at the cube's new position. Both kernels; update time from device-synchronised
    host timers around the whole update."""
    import torch

    g = wl.rng("active/draws")
    lo, hi = wl.cubes("active/cube", 1, 0.1, 0.25)
    centre = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)
    q0 = torch.from_numpy(wl.configs("active/init", n_init, arm.n)).to(dev)
    qt = torch.from_numpy(wl.configs("active/test", n_test, arm.n)).to(dev)
    dirs = g.standard_normal((steps, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    res = {"steps": steps, "n_init": n_init, "k": k, "sigma": sigma, "n_explore": n_explore, "n_test": n_test}
    for kind, gam in (("fk", GAMMA_TRAIN_7DOF), ("configurations", GAMMA_CONFIG_7DOF)):
        y0, _ = api.label_capsule_box(arm, q0, arm.radius, lo, hi, want_clearance=False)
        out = api.train_points(api.fk_points(arm, q0), y0, gam) if kind == "fk" else api.rbf_train(q0, y0, gam)
        sup = out["support"].long()
        sq, sa = q0[sup].contiguous(), out["alpha"][sup].contiguous()
        c = centre.copy()
        rows = []
        gk = wl.rng(f"active/{kind}")
        for step in range(steps):
            c = c + 0.05 * dirs[step]
            lo2, hi2 = c - half, c + half
            S = sq.shape[0]
            noise = torch.from_numpy((sigma * gk.standard_normal((S * k, arm.n))).astype(np.float32)).to(dev)
            explore = torch.from_numpy(gk.uniform(-np.pi, np.pi, (n_explore, arm.n)).astype(np.float32)).to(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if kind == "fk":
                o = api.active_update(arm, sq, sa, gam, noise, k, explore, lo2, hi2)
                X = o["X"]
            else:
                X, a0 = api.active_samples(sq, sa, noise, k, explore)
                yX, _ = api.label_capsule_box(arm, X, arm.radius, lo2, hi2, want_clearance=False)
                api.active_relabel(yX, a0, S)
                F0, _ = api.rbf_score(sq, a0[:S].contiguous(), gam, X, want_label=False)
                o = api.rbf_train(X, yX, gam, alpha=a0, F=F0)
            torch.cuda.synchronize()
            t_upd = time.perf_counter() - t0
            s2 = o["support"].long()
            sq, sa = X[s2].contiguous(), o["alpha"][s2].contiguous()
            yt, _ = api.label_capsule_box(arm, qt, arm.radius, lo2, hi2, want_clearance=False)
            if kind == "fk":
                _, lt = api.fk_score(arm, sq, sa, gam, qt, want_f=False)
            else:
                _, lt = api.rbf_score(sq, sa, gam, qt, want_f=False)
            yt_np, lt_np = yt.cpu().numpy(), lt.cpu().numpy()
            pos, neg = yt_np == 1, yt_np == -1
            rows.append({"rows": int(X.shape[0]), "support": int(s2.numel()), "updates": o["updates"],
                         "converged": bool(o["converged"]), "update_ms": t_upd * 1e3,
                         "accuracy": float(np.mean(lt_np == yt_np)),
                         "tpr": float(np.mean(lt_np[pos] == 1)) if pos.any() else None,
                         "tnr": float(np.mean(lt_np[neg] == -1))})
        res[kind] = {"gamma": gam, "initial_support": int(sup.numel()), "per_step": rows,
                     "mean_update_ms": float(np.mean([r["update_ms"] for r in rows[1:]])),
                     "mean_accuracy": float(np.mean([r["accuracy"] for r in rows])),
                     "mean_tpr": float(np.mean([r["tpr"] for r in rows if r["tpr"] is not None])),
                     "mean_tnr": float(np.mean([r["tnr"] for r in rows]))}
    return res


def batched_run(api, wl, arm, gamma, dev, checks, reps=5):
    """256 environments with lognormal support sets and uniform query batches: one persistent graph-replayed
    launch versus one plain launch per environment."""
    import torch

    envs = wl.batched_envs()
    S_tot, N_tot = int(envs.support_counts.sum()), int(envs.query_counts.sum())
    sq = torch.from_numpy(wl.configs("bench_batch/s", S_tot, arm.n)).to(dev)
    al = torch.from_numpy(wl.weights("bench_batch/a", S_tot)).to(dev)
    q = torch.from_numpy(wl.configs("bench_batch/q", N_tot, arm.n)).to(dev)
    b = api.Batch(arm, envs.support_counts, envs.query_counts, gamma)
    b.prepare(sq, al)
    f = torch.empty(N_tot, dtype=torch.float32, device=dev)
    lab = torch.empty(N_tot, dtype=torch.int8, device=dev)
    t0 = time.perf_counter()
    tq = b.autotune(q, (f, lab))
    t_tune = time.perf_counter() - t0
    tuned = b.shape
    b2 = api.Batch(arm, envs.support_counts, envs.query_counts, gamma)  # same kind: takes the cached shape
    b2.prepare(sq, al)
    t0 = time.perf_counter()
    b2.autotune(q, (f, lab))
    t_cached = time.perf_counter() - t0
    cached = b2.shape
    b2.close()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        b.capture(q, (f, lab))
        b.replay()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(side)
        for _ in range(reps):
            b.replay()
        e1.record(side)
    e1.synchronize()
    ms_batch = e0.elapsed_time(e1) / reps
    # plain form: one prepared model and one launch per environment
    so, qo = envs.support_offsets(), envs.query_offsets()
    models = [api.support_prep(arm, sq[so[e]:so[e + 1]], al[so[e]:so[e + 1]], gamma) for e in range(envs.E)]
    fp = torch.empty_like(f)
    lp = torch.empty_like(lab)

    def plain():
        for e in range(envs.E):
            api.fk_score_prepared(arm, models[e], q[qo[e]:qo[e + 1]], out=(fp[qo[e]:qo[e + 1]], lp[qo[e]:qo[e + 1]]))

    plain()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plain()
    e1.record()
    e1.synchronize()
    ms_plain = e0.elapsed_time(e1) / reps
    same = bool(torch.equal(f, fp) and torch.equal(lab, lp))
    kevals = float(np.sum(envs.support_counts.astype(np.float64) * envs.query_counts))
    Mm = int(np.sum(arm.frames > 0))
    res = {"E": envs.E, "queries": N_tot, "supports": S_tot, "tile_queries": tq, "shape": tuned,
           "autotune_s": t_tune, "autotune_cached_s": t_cached, "cached_shape_reused": bool(cached["from_cache"]),
           "ms_graph_replay": ms_batch,
           "checks_per_s": N_tot / (ms_batch * 1e-3), "kernel_evals_per_s": kevals / (ms_batch * 1e-3),
           "frac_alu": kevals * Mm / (ms_batch * 1e-3) / alu_peak(Mm, api.score_rational(arm, gamma)),
           "ms_plain_per_env_launches": ms_plain, "speedup_vs_plain": ms_plain / ms_batch,
           "identical_to_plain": same, "fp64_sample": {}}
    # FP64 comparison (CPU leg) on 2,000 evenly spaced queries of the largest and of the smallest environment
    for tag, e in (("largest_S", int(np.argmax(envs.support_counts))), ("smallest_S", int(np.argmin(envs.support_counts)))):
        idx = np.linspace(qo[e], qo[e + 1] - 1, 2000).astype(np.int64)
        res["fp64_sample"][tag] = {"env": e, "S": int(envs.support_counts[e])}
        checks.append({"arm": arm, "sq": sq[so[e]:so[e + 1]].cpu().numpy(), "al": al[so[e]:so[e + 1]].cpu().numpy(),
                       "gamma": gamma, "q": q[idx].cpu().numpy(), "f": f.cpu().numpy()[idx],
                       "lab": lab.cpu().numpy()[idx], "into": res["fp64_sample"][tag]})
    b.close()
    return res


def retrain_run(api, wl, arm, dev, n_env=16, N=20_000):
    """16 environments: label, train, shift every cube by 0.05 m in a random direction, relabel, warm-start.
    Once one environment after the other (fastron_train), once all 16 in one launch (fastron_train_batch), whose
    results must be identical."""
    import torch

    envs = wl.batched_envs()
    qs, y0s, y1s = [], [], []
    for e in range(n_env):
        q = torch.from_numpy(wl.configs(f"retrain/{e}/q", N, arm.n)).to(dev)
        lo, hi = wl.cubes(f"retrain/{e}/cubes", int(envs.cube_counts[e]), 0.1, 0.25)
        y0, _ = api.label_capsule_box(arm, q, arm.radius, lo, hi, want_clearance=False)
        shift = 0.05 * wl.unit_directions(f"retrain/{e}/shift", lo.shape[0])
        y1, _ = api.label_capsule_box(arm, q, arm.radius, lo + shift, hi + shift, want_clearance=False)
        qs.append(q)
        y0s.append(y0)
        y1s.append(y1)
    P = api.fk_points(arm, torch.cat(qs))
    Y0, Y1 = torch.cat(y0s), torch.cat(y1s)
    off = np.arange(n_env + 1, dtype=np.int64) * N
    rows = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    seq = []
    for e in range(n_env):
        sl = slice(e * N, (e + 1) * N)
        first = api.train_points(P[sl].contiguous(), Y0[sl].contiguous(), GAMMA_TRAIN_7DOF)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        second = api.train_points(P[sl].contiguous(), Y1[sl].contiguous(), GAMMA_TRAIN_7DOF, alpha=first["alpha"],
                           F=first["F"])
        torch.cuda.synchronize()
        seq.append(second)
        rows.append({"updates_first": first["updates"], "updates_warm": second["updates"],
                     "warm_ms": (time.perf_counter() - t0) * 1e3, "converged": bool(second["converged"])})
    t_seq = time.perf_counter() - t_all
    t0 = time.perf_counter()
    b0 = api.train_batch(P, Y0, off, GAMMA_TRAIN_7DOF)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    b1 = api.train_batch(P, Y1, off, GAMMA_TRAIN_7DOF, alpha=b0["alpha"], F=b0["F"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    same = all(torch.equal(b1["alpha"][e * N:(e + 1) * N], seq[e]["alpha"]) for e in range(n_env))
    return {"envs": n_env, "N_per_env": N, "total_ms_one_after_another": t_seq * 1e3,
            "warm_ms_mean": float(np.mean([r["warm_ms"] for r in rows])),
            "updates_warm_mean": float(np.mean([r["updates_warm"] for r in rows])),
            "updates_first_mean": float(np.mean([r["updates_first"] for r in rows])),
            "all_converged": all(r["converged"] for r in rows),
            "one_launch": {"first_ms": (t1 - t0) * 1e3, "warm_ms": (t2 - t1) * 1e3,
                           "warm_speedup_vs_one_after_another": sum(r["warm_ms"] for r in rows) / ((t2 - t1) * 1e3),
                           "converged": bool(b0["converged"] and b1["converged"]), "identical": bool(same)}}


BF16_PEAK_TFLOPS = 2500.0


def mlp_train_flops(d_in, H):
    """Algorithmic FLOP to train the screening network on one sample: forward (both layers and the head, bias
    adds included) 2 (d_in H + H H + H), dH1 2 H H, and the two weight gradients 2 H H + 2 d_in H."""
    return 2 * (d_in * H + H * H + H) + 2 * H * H + 2 * H * H + 2 * d_in * H


def mlp_run(api, wl, arm, dev, epochs=3, n_train=1_900_000):
    """The screening network's training step alone (no Fastron training in this leg): epochs over n_train
    labelled configurations of the 20-cube environment, batch 8,192, each epoch timed with HIP events; FLOP per
    epoch from mlp_train_flops against the dense BF16 peak."""
    import torch

    lo, hi = wl.cubes("bench7/cubes", 20, 0.1, 0.25)
    q_tr = torch.from_numpy(wl.configs("bench7/screen_train", n_train, arm.n)).to(dev)
    y_tr, _ = api.label_capsule_box(arm, q_tr, arm.radius, lo, hi, want_clearance=False)
    P_tr = api.fk_points(arm, q_tr)
    del q_tr
    d_in = 3 * arm.M
    net = api.MLP(d_in, 256, max_rows=8192)
    net.set_params(torch.from_numpy(wl.mlp_init(d_in, 256, name="bench7/mlp_init")).to(dev))
    net.fit_standardisation(P_tr)
    perms = [torch.from_numpy(wl.rng(f"bench7/mlp_perm{ep}").permutation(n_train).astype(np.int32)).to(dev)
             for ep in range(epochs)]
    ms, losses = [], []
    for ep in range(epochs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        losses.append(net.train_epoch(P_tr, y_tr, perms[ep], batch=8192, lr=1e-3))
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    net.close()
    flops = mlp_train_flops(d_in, 256) * n_train
    best = float(np.median(ms))
    return {"samples": n_train, "batch": 8192, "epochs": epochs, "epoch_ms": ms, "epoch_ms_median": best,
            "samples_per_s": n_train / (best * 1e-3), "flop_per_epoch": flops,
            "tflops": flops / (best * 1e-3) / 1e12, "frac_bf16_peak": flops / (best * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
            "losses": losses}


def screen_run(api, wl, arm, dev, epochs=6, n_train=2_000_000, n_query=4_194_304, taus=(0.0, 0.5, 1.0, 2.0, 4.0)):
    """Screening network trained on 2,000,000 geometrically labelled configurations (first 1,900,000 train, last
    100,000 held out); fallback model = Algorithm 1 on 50,000 labelled samples with S_max = 4,000; 4,194,304
    queries scored plain (Fastron FK only) and screened for each tau; accuracy against geometric labels."""
    import torch

    lo, hi = wl.cubes("bench7/cubes", 20, 0.1, 0.25)
    sync = torch.cuda.synchronize
    # training data for the network
    q_tr = torch.from_numpy(wl.configs("bench7/screen_train", n_train, arm.n)).to(dev)
    y_tr, _ = api.label_capsule_box(arm, q_tr, arm.radius, lo, hi, want_clearance=False)
    P_tr = api.fk_points(arm, q_tr)
    del q_tr
    n_fit = n_train - 100_000
    net = api.MLP(3 * arm.M, 256, max_rows=8192)
    net.set_params(torch.from_numpy(wl.mlp_init(3 * arm.M, 256, name="bench7/mlp_init")).to(dev))
    P_fit, y_fit = P_tr[:n_fit], y_tr[:n_fit]
    net.fit_standardisation(P_fit)
    perms = [torch.from_numpy(wl.rng(f"bench7/mlp_perm{ep}").permutation(n_fit).astype(np.int32)).to(dev)
             for ep in range(epochs)]  # drawn on the host before the timed training
    sync()
    t0 = time.perf_counter()
    losses = []
    for ep in range(epochs):
        losses.append(net.train_epoch(P_fit, y_fit, perms[ep], batch=8192, lr=1e-3))
    sync()
    train_s = time.perf_counter() - t0
    del perms
    z_ho = net.forward(P_tr[n_fit:].contiguous())
    acc_ho = float((torch.where(z_ho >= 0, 1, -1).to(torch.int8) == y_tr[n_fit:]).float().mean())
    del P_tr, y_tr
    # fallback Fastron model (S_max = 4,000)
    q50 = torch.from_numpy(wl.configs("bench7/train", 50_000, arm.n)).to(dev)
    y50, _ = api.label_capsule_box(arm, q50, arm.radius, lo, hi, want_clearance=False)
    fit = api.train_points(api.fk_points(arm, q50), y50, GAMMA_TRAIN_7DOF, s_max=4000)
    sup = fit["support"].long()
    model = api.support_prep(arm, q50[sup].contiguous(), fit["alpha"][sup].contiguous(), GAMMA_TRAIN_7DOF)
    # queries and their geometric labels
    q = torch.from_numpy(wl.configs("bench7/screen_q", n_query, arm.n)).to(dev)
    truth, _ = api.label_capsule_box(arm, q, arm.radius, lo, hi, want_clearance=False)

    def timed(fn, reps=3):
        fn()
        sync()
        t = time.perf_counter()
        for _ in range(reps):
            out = fn()
        sync()
        return out, (time.perf_counter() - t) / reps

    (_, lab_plain), t_plain = timed(lambda: api.fk_score_prepared(arm, model, q, want_f=False))
    acc_plain = float((lab_plain == truth).float().mean())
    rows = []
    for tau in taus:
        (lab, _, fb, nfb), t = timed(lambda: net.screen(arm, model, q, tau))
        rows.append({"tau": tau, "fallback_rate": nfb / n_query, "checks_per_s": n_query / t,
                     "accuracy": float((lab == truth).float().mean()), "speedup_vs_plain": t_plain / t})
    net.close()
    train_tflops = mlp_train_flops(3 * arm.M, 256) * n_fit * epochs / train_s / 1e12
    return {"train_samples": n_fit, "epochs": epochs, "train_s": train_s, "losses": losses,
            "train_tflops": train_tflops, "train_frac_bf16_peak": train_tflops / BF16_PEAK_TFLOPS,
            "heldout_accuracy_mlp_only": acc_ho, "fallback_support": int(sup.numel()),
            "fallback_converged": bool(fit["converged"]), "queries": n_query,
            "plain": {"checks_per_s": n_query / t_plain, "accuracy": acc_plain}, "screened": rows}


def cpu_baseline(arm, sq, al, q, gamma, f_gpu, lab_gpu, seconds, extras, checks):
    """FP64 oracle on a bounded, evenly spaced sample of the queries (all host threads); also the FP64
    comparisons queued by the other legs (max |df|, sign agreement, queries inherently ambiguous at that
    error: |f_fp64| < max |df|)."""
    import oracle

    for c in checks:
        if c.get("kind") == "configurations":
            ref = oracle.rbf_score(c["sq"].astype(np.float64), c["al"].astype(np.float64), c["gamma"],
                                   c["q"].astype(np.float64))
        else:
            a = c["arm"]
            dh_c = oracle.dh_table(a.a, a.alpha, a.d, a.theta, a.joint_type)
            ref = oracle.score(dh_c, a.frames, c["sq"].astype(np.float64), c["al"].astype(np.float64),
                               c["gamma"], c["q"].astype(np.float64), offset=a.offsets)
        df = float(np.max(np.abs(c["f"].astype(np.float64) - ref)))
        c["into"]["vs_fp64"] = {"queries": int(ref.size), "max_abs_df": df,
                                "sign_agreement": float(np.mean(c["lab"] == np.where(ref < 0, -1, 1))),
                                "ambiguous": int(np.sum(np.abs(ref) < df))}

    dh = oracle.dh_table(arm.a, arm.alpha, arm.d, arm.theta, arm.joint_type)
    sq64, al64 = sq.astype(np.float64), al.astype(np.float64)
    probe = np.linspace(0, q.shape[0] - 1, 4096).astype(np.int64)
    t0 = time.perf_counter()
    oracle.score(dh, arm.frames, sq64, al64, gamma, q[probe].astype(np.float64))
    rate = probe.shape[0] / (time.perf_counter() - t0)
    n = int(min(q.shape[0], max(1024, rate * seconds)))
    idx = np.linspace(0, q.shape[0] - 1, n).astype(np.int64)
    t0 = time.perf_counter()
    ref = oracle.score(dh, arm.frames, sq64, al64, gamma, q[idx].astype(np.float64))
    dt = time.perf_counter() - t0
    sign_ref = np.where(ref < 0, -1, 1)
    agree = {"sign_agreement_vs_fp64": float(np.mean(lab_gpu[idx] == sign_ref)),
             "max_abs_df_vs_fp64": float(np.max(np.abs(f_gpu[idx] - ref))),
             "fp64_sample": int(n)}
    for name, form in extras.get("forms", {}).items():
        form["sign_agreement_vs_fp64"] = float(np.mean(form["labels"][idx] == sign_ref))
    cpu = {"value": n / dt, "unit": "checks/s", "cores": oracle.num_threads(), "kind": "oracle",
           "build": oracle.BUILD_FLAGS,
           "sample": f"{n} evenly spaced queries of the same workload (S={sq.shape[0]}), {dt:.1f} s",
           "logical_cpus": os.cpu_count(), "physical_cores": _physical_cores(), "cpu_model": _cpu_model()}
    # one thread on a 10,000-query subset (the paper's thread count is not stated)
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    sub = np.linspace(0, q.shape[0] - 1, 10_000).astype(np.int64)
    t0 = time.perf_counter()
    oracle.score(dh, arm.frames, sq64, al64, gamma, q[sub].astype(np.float64))
    dt1 = time.perf_counter() - t0
    oracle.set_num_threads(threads)
    cpu["single_thread"] = {"value": sub.size / dt1, "unit": "checks/s", "us_per_check": dt1 * 1e6 / sub.size,
                            "sample": "10,000 evenly spaced queries"}
    cpu["rows"] = cpu_rows(oracle, arm, dh, extras)
    return cpu, agree


def cpu_rows(oracle, arm, dh, extras):
    """The oracle timed on the other steps of the path, each beside the GPU figure of the same step when the
    corresponding leg ran: FK (a1), Gram column (a4), Algorithm 1 (a5, 3-DOF workload), labels (a9), the
    screening network's forward pass (a8) and the score with the kernel on configurations."""
    from oracle import mlp_oracle
    from paper_1910_06451_amd import workloads as wl

    rows = {}
    kern = extras.get("kernels", {})

    def timed(fn):
        t0 = time.perf_counter()
        out = fn()
        return out, time.perf_counter() - t0

    qs = wl.configs("kern/q", 262_144, arm.n).astype(np.float64)
    P, t = timed(lambda: oracle.control_points(dh, arm.frames, qs))
    rows["fk_points"] = {"oracle_configs_per_s": qs.shape[0] / t, "sample": "262,144 configurations",
                         "gpu_configs_per_s": kern.get("fk_points", {}).get("configs_per_s")}
    _, t = timed(lambda: oracle.score_points(P[:1], np.ones(1), 10.0, P))
    rows["gram_column"] = {"oracle_points_per_s": P.shape[0] / t, "sample": "one column over 262,144 points",
                           "gpu_points_per_s": kern.get("gram_update", {}).get("points_per_s")}
    lo, hi = wl.cubes("bench7/cubes", 20, 0.1, 0.25)
    _, t = timed(lambda: oracle.capsule_box_labels(dh, qs[:65_536], arm.radius, lo, hi))
    rows["labels"] = {"oracle_configs_per_s": 65_536 / t, "sample": "65,536 configurations, 20 cubes",
                      "gpu_configs_per_s": kern.get("label_capsule_box", {}).get("configs_per_s")}
    d3 = extras.get("dof3")
    if d3:
        a3 = wl.arm_3dof()
        dh3 = oracle.dh_table(a3.a, a3.alpha, a3.d, a3.theta, a3.joint_type)
        q3 = wl.configs("train3", 2000, a3.n, seed=d3["seed"]).astype(np.float64)
        lo3, hi3 = wl.cubes("train3/cubes", 5, 0.15, None, seed=d3["seed"])
        y3, _ = oracle.capsule_box_labels(dh3, q3, a3.radius, lo3, hi3)
        P3 = oracle.control_points(dh3, a3.frames, q3).astype(np.float32).astype(np.float64)
        r3, t = timed(lambda: oracle.fastron_update(P3, y3, 10.0))
        rows["train_3dof"] = {"oracle_ms": t * 1e3, "oracle_updates": r3["updates"],
                              "gpu_ms_fp64": d3["train_ms_fp64"], "gpu_updates": d3["updates"],
                              "sample": "2,000 labelled 3-DOF configurations, gamma = 10"}
    cmp_ = extras.get("compare", {}).get("configurations")
    if cmp_:
        sx, sa = wl.model("cpu_rows/config", cmp_["support"], arm.n)
        qc = qs[:4096, : arm.n]
        _, t = timed(lambda: oracle.rbf_score(sx.astype(np.float64), sa.astype(np.float64), GAMMA_CONFIG_7DOF, qc))
        rows["configuration_score"] = {"oracle_kernel_evals_per_s": qc.shape[0] * sx.shape[0] / t,
                                       "sample": f"4,096 queries against {cmp_['support']:,} supports",
                                       "gpu_kernel_evals_per_s": cmp_["kernel_evals_per_s"]}
    params = [p.astype(np.float64) for p in wl.split_mlp_params(wl.mlp_init(24, 256, name="cpu_rows"), 24)]
    X = P[:65_536].reshape(-1, 24)
    _, t = timed(lambda: mlp_oracle.forward(params, X, X.mean(axis=0), X.std(axis=0) + 1e-9))
    scr = extras.get("screen", {})
    tau0 = next((r for r in scr.get("screened", []) if r["tau"] == 0.0), {})
    rows["mlp_forward"] = {"oracle_queries_per_s": X.shape[0] / t, "sample": "65,536 queries (NumPy FP64)",
                           "gpu_screen_tau0_checks_per_s": tau0.get("checks_per_s")}
    return rows


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _physical_cores():
    """Distinct (package, core) pairs among the CPUs this process may run on, from /proc/cpuinfo."""
    try:
        allowed = os.sched_getaffinity(0)
        cores, cpu, pkg = set(), None, None
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "processor":
                    cpu, pkg = int(val), None
                elif key == "physical id":
                    pkg = val
                elif key == "core id" and cpu in allowed:
                    cores.add((pkg, val))
        return len(cores) or None
    except (OSError, ValueError):
        return None


if __name__ == "__main__":
    main()
