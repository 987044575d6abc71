#!/usr/bin/env python3
"""Benchmark of the GA-CIR advance on one MI355X.

Workload (the 2048^2 single-level-set case): 2049^2 nodes on [0,1]^2, phi =
signed distance to the union of 4 seeded circles, velocity from an 8-mode sine
stream function modulated by cos(pi t / 2), 1024 steps of dt = 2/1024 (CFL
0.8); the flow reverses so the final state should return to the initial one.

One benchmark step = one pass of the whole path over the workload: the full
1024-step advance (every step: trace, split, gather, Hermite, gradient update,
write-back) followed by the FP64 shape-error reduction against the initial
state. The FP32-state path is timed (foot coordinates and split in FP64); the
FP64 path runs once beside it for the matched-error comparison.

Prints one JSON line. Options: --gpus (only 1 is supported), --steps K,
--warmup W, --no-cpu (skip the oracle baseline), --inner (time steps per
benchmark step, default the workload's 1024).

--workload adjoint times one gradient of the shape loss with respect to 16
stream-function amplitudes on 1024^2 cells: a 200-step FP32 advance that
keeps a checkpoint every 20 steps, the loss and its seed, and the reverse
sweep (each segment recomputed from its checkpoint, then 20 adjoint steps).

--workload variants times the 2048^2 advance (FP32) for each cross-derivative
reconstruction (central (A), cell-based (B), zero) with the superconsistent
and with Heun's gradient update, and on a box shifted by 0.1 (the flow then
enters through parts of every face) with the projection of feet alone,
Dirichlet inflow data, and the homogeneous Neumann face scheme.

--workload volume runs the 3D deformation test of the paper's volume-loss
tables (LeVeque's field x cos(pi t / 2.5), dt = h, to t = 2.5; a sphere and a
cube at n = 50, 100, 150, 200, FP64) and reports the relative volume change
beside the paper's GA-CIR rows, and the 200^3 advance's throughput.

--workload table runs every configuration once and prints the per-configuration
results (GPU rate, algorithmic HBM rate, the oracle's rate on all host threads
and on one core, shape errors, the distance to the oracle) as one JSON line
and, on stderr, as a markdown table: the 64^2 rotation (FP64, 128 steps), the
2048^2 workload in FP64 and FP32, the 256^3 vector-potential workload (FP32),
and the two bandwidth probes.

--workload batched times the many-problem case instead: 512 independent
grids of round(2^U(5,9)) cells per side, each with its own circles and
stream function, 256 steps of dt = 2/256 per benchmark step, advanced
together (one launch per step over a work list of tiles, the whole advance
replayed from a captured hipGraph, wave shapes chosen by the autotuner
first).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GALS node-updates/s + HBM GB/s, FP32 vs FP64 GPU at matched L1 shape error"
HBM_PEAK_GBPS = 8000.0
# Non-packed FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.
# (The 157.3 TFLOP/s datasheet figure needs packed FP32 instructions, which this
# build does not emit.)
VALU_F32_PEAK_TFLOPS = 78.6
SIMDS = 256 * 4
CLOCK_GHZ = 2.4
VALU_F32_PACKED_PEAK_TFLOPS = 157.3  # reported beside it, for comparison only
# Floating-point operations per node of the FP32 stream-function step as
# formulated, FMA = 2, on a lane whose stages take the degree-3 Taylor
# polynomials: jet 98 (14 dot products of 4), stage 1 0 (signs only: dt and
# the time factors sit in the stage weights), stage 2 75 (offset 2, Taylor
# test 3, offset scalings 4, Taylor polynomials 66), stage 3 79 (offset 6),
# Jacobian chain 66, foot (displacement in FP32, position in FP64) and split
# 16, cross derivatives 8, Hermite weights 40, bicubic value and gradient 80,
# gradient update 6.
ALG_FLOPS_PER_NODE = 468
# A lane whose two stage offsets are both in the degree-2 tier: each stage's
# polynomials cost 32 with 2 scalings (36 fewer a stage), and the jet skips
# its 5 order-4 entries (35 fewer). A lower bound of the step's count; the
# headline reports the hardware count from the counter summary instead.
ALG_FLOPS_PER_NODE_LOW = ALG_FLOPS_PER_NODE - 2 * 36 - 35
BYTES_PER_NODE = 24  # FP32 state: 3 planes read once + 3 planes written once
# The cell-based (B) cross derivatives replace the 8 flops of the central
# differences by 4 edge differences and 4 weighted vertex sums (28 flops).
VARIANT_B_FLOPS_PER_NODE = ALG_FLOPS_PER_NODE - 8 + 28
# FP32 3D step, 6-mode vector potential, central cross derivatives, as the
# kernel formulates it (FMA = 2; the time factors sit in the stage weights):
# velocity and Jacobian at the node from the per-axis tables (multiples 36,
# 6 modes x 59: 390) and at the two off-node stages with the angles shifted by
# angle addition (shift 36, multiples 36, modes 354: 426 each), stage offsets
# and displacement 30, Jacobian chain 180, foot and split 30, cross
# derivatives 120, Hermite weights 60, tricubic value and gradient 384,
# gradient update 18.
FLOPS_PER_NODE_3D = 390 + 2 * 426 + 30 + 180 + 30 + 120 + 60 + 384 + 18
BYTES_PER_NODE_3D = 32  # FP32 state: 4 planes read once + 4 planes written once
# Bandwidth probe (rigid rotation, the cheapest field). The three stages of an
# affine field compose to one affine map that the host forms once per step,
# so a node's foot costs D^2 FP64 multiply-adds (in cell units), and its
# Jacobian is uniform: 2D foot 8 + split 4 + cross derivatives 8 + Hermite
# weights 40 + bicubic 80 + update 6; 3D foot 18 + split 6 + cross 120 +
# weights 60 + tricubic 384 + update 18.
PROBE_FLOPS_PER_NODE_2D = 8 + 4 + 8 + 40 + 80 + 6
PROBE_FLOPS_PER_NODE_3D = 18 + 6 + 120 + 60 + 384 + 18


# The Infinity Cache (MALL) in front of HBM: working sets below it are not HBM-bound.
MALL_BYTES = 256 << 20
# FP64 grid whose L1 shape error after the time-reversed run equals the FP32
# path's at 2048^2 (measured: FP64 1.243e-9 at 1728^2, 1.116e-9 at 1792^2;
# FP32 at 2048^2 1.237e-9).
MATCHED_FP64_CELLS = 1728
# The paper's only throughput figure (sec. 6.2, computational effort): the
# superconsistent GA-CIR run of the vortex test on a 64^2 grid, 512 steps, in
# about 9 s on one core of an unnamed desktop computer.
PAPER_CPU_CONTEXT = {"value": 512 * 65 * 65 / 9.0, "unit": "node-updates/s", "cores": 1,
                     "hardware": "one core of an unnamed desktop computer (the paper's, 2009)",
                     "sample": "512 steps of 65^2 nodes in 9 s (sec. 6.2)"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Sources each timed kernel is compiled from (plus the build flags): a
# committed traffic record applies only while these are unchanged.
STEP_HEADERS = ["gals_internal.h", "velocity.h", "hermite.h", "stream2d.h"]
SINGLE_KERNEL_SOURCES = ["kernels_step.hip"] + STEP_HEADERS
BATCH_KERNEL_SOURCES = ["batch.hip", "batch_shape.h", "gals_batch_api.hip"] + STEP_HEADERS
ADJ_KERNEL_SOURCES = ["adjoint.hip", "reduce.h"] + STEP_HEADERS
# Floating-point operations per node of the FP32 adjoint step (FMA = 2):
# trace 346 (the forward step's jet, stages, chain and foot, 334, plus the 12
# products that restore the time factors of the stage Jacobians), cross
# derivatives 8, Hermite weights with second derivatives 60, bicubic value,
# gradient and Hessian 132, the state adjoint's cell shares 156, seeds 28,
# reverse Jacobian chain 128, sin/cos multiples at the 3 stage points 112
# (from the node's table entries, shifted by angle addition at the two
# off-node stages), mode terms 438 (146 a stage: y factors per n, M cos per
# m, three multiply-adds per mode), third derivatives 376 (188 at each of two
# stages), stage-position adjoints 72, accumulation and block reduction 44
# (FP64: 16 accumulations, 12 adds of the two halving swaps, 16 of the row
# sums).
ADJ_FLOPS_PER_NODE = 1900
# read the state (3 x 4 B) and lam_next (3 x 8 B); zero-fill and
# accumulate lam_prev (3 x 8 B written, and the atomics' read-modify-write)
ADJ_BYTES_PER_NODE = 12 + 24 + 24 + 24


def kernel_source_hash(files):
    """Hash of the code a kernel is built from: its sources and the build
    script, with comments and whitespace removed (an edit of a comment does
    not change the kernel)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in sorted(files) + ["../build.py"]:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_0905_3409_amd", "csrc", name), encoding="utf-8") as fh:
            text = fh.read()
        if name.endswith(".py"):
            text = re.sub(r"#[^\n]*", "", text)
        else:
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def profile_record(profile_md, files, kind):
    """The fields of a `<kind>-record:` line of a committed rocprofv3 summary
    under profiles/, as floats; None if the summary or the line is missing, or
    if the kernel has changed since the counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", profile_md)
    if not os.path.exists(path):
        return None
    m = re.search(kind + r"-record: src_hash=(\w+)((?: \w+=[\d.]+)+)", open(path).read())
    if not m or m.group(1) != kernel_source_hash(files):
        return None
    return {k: float(v) for k, v in re.findall(r"(\w+)=([\d.]+)", m.group(2))}


def traffic_record(profile_md, files):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE/WRITE_SIZE summary,
    scaled by the counters' reading of a plain copy; None if the kernel has
    changed since the counters were taken."""
    r = profile_record(profile_md, files, "traffic")
    if r is None:
        return None
    kib = r["fetch_kib"] * r["fetch_scale"] + r["write_kib"] * r["write_scale"]
    return kib * 1024.0


def valu_issue(profile_md, files, kernel_us):
    """The vector-issue side of a kernel from its rocprofv3 counter summary:
    VALU instructions per wave (SQ_INSTS_VALU / SQ_WAVES), hardware flops per
    node (SQ_INSTS_VALU_FLOPS_FP32 + _FP64, x64 lanes, over the nodes), and
    the time the chip needs to issue those instructions at 4 cycles per wave64
    instruction (16 lanes per SIMD) on 1024 SIMDs at 2.4 GHz, as a fraction
    of the kernel's measured time. None if the kernel has changed since."""
    r = profile_record(profile_md, files, "valu")
    if r is None:
        return None
    issue_us = r["valu_per_wave"] * r["waves"] * 4 / (SIMDS * CLOCK_GHZ * 1e3)
    tflops = r["hw_flops_per_node"] * r["nodes"] / (kernel_us * 1e-6) / 1e12
    return {"valu_instr_per_wave": r["valu_per_wave"], "waves": int(r["waves"]),
            "issue_us_at_4_cycles": issue_us, "issue_frac": issue_us / kernel_us,
            "hw_flops_per_node": r["hw_flops_per_node"], "hw_tflops": tflops,
            "hw_frac_of_nonpacked_fp32_peak": tflops / VALU_F32_PEAK_TFLOPS,
            "hw_frac_of_packed_fp32_peak": tflops / VALU_F32_PACKED_PEAK_TFLOPS,
            "source": "profiles/" + profile_md}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--inner", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--workload",
                    choices=["single", "batched", "adjoint", "variants", "volume", "3d",
                             "probe", "table"],
                    default="single")
    ap.add_argument("--tiles", default="",
                    help="batched only: wave widths per size class, e.g. 64,0,16,64, "
                         "instead of the autotuner's choice")
    ap.add_argument("--profile", action="store_true",
                    help="short FP32 advance plus a plain device copy of known size "
                         "(for calibrating rocprofv3 byte counters); prints no JSON")
    ap.add_argument("--probe-case", choices=["2d", "3d"], default="2d",
                    help="probe workload with --profile: the case to run")
    ap.add_argument("--profile-fp64", action="store_true",
                    help="single workload with --profile: advance the FP64 state instead")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU; sharding a grid over several GPUs is "
              "described in the design notes, not implemented. Run with --gpus 1.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_0905_3409_amd as pkg
    from paper_0905_3409_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "adjoint":
        return bench_adjoint(args)
    if args.workload == "variants":
        return bench_variants(args)
    if args.workload == "volume":
        return bench_volume(args)
    if args.workload == "3d":
        return bench_3d(args)
    if args.workload == "probe":
        return bench_probe(args)
    if args.workload == "table":
        return bench_table(args)
    dev = torch.device("cuda", 0)
    w = inputs.stream_circles()
    inner = args.inner or w["steps"]
    n = w["ncell"][0]
    h = 1.0 / n
    nodes = (n + 1) ** 2
    eps, band = 1.5 * h, 3 * h
    log(f"workload {w['name']} {n}^2 cells, {inner} steps/bench step, dt={w['dt']:.6g}")

    def setup(dtype):
        g = pkg.Grid(w["ncell"], w["lo"], w["hi"], dtype=dtype)
        g.set_velocity(w["kind"], w["params"], w["period"])
        ref = g.from_numpy(w["phi0"], w["psi0"])
        return g, ref, ref.clone()

    def bench_step(g, st, ref, ev=None):
        if ev is not None:
            ev[0].record()
        g.advance(st, 0.0, w["dt"], inner)
        if ev is not None:
            ev[1].record()
        return g.norms(st, ref, eps, band)  # synchronises

    # ---------------------------------------------------------------- FP32
    if args.profile:
        prec = "float64" if args.profile_fp64 else "float32"
        gp, _, stp = setup(prec)
        steps = args.inner or 64
        gp.advance(stp, 0.0, w["dt"], steps)
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)  # plain copy: reads and writes exactly 256 MiB
        torch.cuda.synchronize()
        log(f"profile: {steps} {prec} steps on {nodes} nodes, then a {nbytes} B device copy")
        return 0
    g32, ref32, st32 = setup("float32")
    for _ in range(args.warmup):
        bench_step(g32, st32, ref32)
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        bench_step(g32, st32, ref32, events[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    adv_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    kernel_us = adv_ms * 1e3 / inner  # average step-kernel duration (launches back to back)
    value = nodes * inner / (ms_per_step * 1e-3)
    log(f"fp32: {ms_per_step:.2f} ms/bench step, advance {adv_ms:.2f} ms, "
        f"step kernel {kernel_us:.2f} us, {value / 1e9:.2f} G node-upd/s")

    # ---------------------------------------------- full-run errors, FP32 vs FP64
    st32.copy_(ref32)
    n32 = bench_step(g32, st32, ref32)  # one fresh full run
    res = {}
    if not args.no_fp64:
        g64, ref64, st64 = setup("float64")
        bench_step(g64, st64, ref64)          # warm-up
        st64.copy_(ref64)
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        torch.cuda.synchronize()
        a = time.perf_counter()
        n64 = bench_step(g64, st64, ref64, ev)
        b = time.perf_counter()
        adv64 = ev[0].elapsed_time(ev[1])
        res["fp64"] = {"value": nodes * inner / (b - a), "advance_ms": adv64,
                       "step_kernel_us": adv64 * 1e3 / inner,
                       "l1_shape_error": n64[2], "linf_band_error": n64[3],
                       "volume_change": n64[4] - n64[5]}
        res["l1_shape_error_ratio_fp32_over_fp64"] = n32[2] / n64[2] if n64[2] > 0 else None
        # the FP32 final state against the FP64 one (the FP64 path matches the
        # oracle to 1e-12), both after the whole run
        d = state_errors(g64, st32.double(), st64, h, eps, band)
        res["fp32_vs_fp64_final"] = d
        log(f"fp64: {res['fp64']['value'] / 1e9:.2f} G node-upd/s, L1 shape err {n64[2]:.3e}; "
            f"fp32 L1 shape err {n32[2]:.3e} (ratio {res['l1_shape_error_ratio_fp32_over_fp64']:.3f}); "
            f"fp32 vs fp64 final: phi {d['phi']:.2e} psi {d['psi']:.2e} L1 {d['l1_shape']:.2e}")
        del g64, ref64, st64
        res["matched_error"] = matched_error(args, w, n32[2], ms_per_step, value)
    res["fp32_l1_shape_error"] = n32[2]
    res["fp32_linf_band_error"] = n32[3]

    gbps = nodes * BYTES_PER_NODE / (kernel_us * 1e-6) / 1e9
    state_bytes = 3 * g32.plane * 4
    # the vector-issue side, from the kernel's committed counter summary
    alu = {"nonpacked_fp32_peak_tflops": VALU_F32_PEAK_TFLOPS,
           "packed_fp32_peak_tflops": VALU_F32_PACKED_PEAK_TFLOPS}
    alu.update(valu_issue("k_step2d_f32_stream_2048.md", SINGLE_KERNEL_SOURCES, kernel_us)
               or {"source": None})
    roofline = {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": gbps / HBM_PEAK_GBPS,
                "traffic": traffic_record("k_step2d_f32_stream_2048.md", SINGLE_KERNEL_SOURCES),
                "kernel": "k_step2d_stream<float, CENTRAL, taylor>",
                "bytes_per_launch": nodes * BYTES_PER_NODE, "bytes_per_node": BYTES_PER_NODE,
                "avg_launch_us": kernel_us,
                "working_set_bytes": 2 * state_bytes,
                "mall_resident": 2 * state_bytes < MALL_BYTES,
                "note": "the two 50 MB state copies fit the 256 MB Infinity Cache, so these "
                        "bytes are not all HBM traffic; the kernel is bound by vector "
                        "instruction issue (alu.issue_frac: the time its VALU instructions "
                        "need at 4 cycles each, over its measured time)",
                "alu": alu}

    # ------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu:
        import oracle
        k_cpu = 64  # about 15 s on 16 host threads
        a = time.perf_counter()
        ophi, opsi = oracle.advance(2, w["ncell"], w["lo"], w["hi"], w["kind"], w["params"],
                                    w["period"], w["phi0"], w["psi0"], 0.0, w["dt"], k_cpu)
        b = time.perf_counter()
        cpu = {"value": nodes * k_cpu / (b - a), "unit": "node-updates/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"first {k_cpu} of the {w['steps']} steps of the same 2048^2 workload "
                         f"(FP64 oracle, OpenMP), {b - a:.1f} s"}
        log(f"cpu oracle: {cpu['value'] / 1e6:.2f} M node-upd/s on {cpu['cores']} threads")
        # and on one core: the first 4 steps
        threads = oracle.num_threads()
        oracle.set_threads(1)
        k1 = 4
        a = time.perf_counter()
        oracle.advance(2, w["ncell"], w["lo"], w["hi"], w["kind"], w["params"], w["period"],
                       w["phi0"], w["psi0"], 0.0, w["dt"], k1)
        b = time.perf_counter()
        oracle.set_threads(threads)
        cpu["single_core"] = {"value": nodes * k1 / (b - a), "unit": "node-updates/s",
                              "cores": 1, "sample": f"the first {k1} steps, {b - a:.1f} s"}
        cpu["paper_context"] = PAPER_CPU_CONTEXT
        log(f"cpu oracle, 1 core: {nodes * k1 / (b - a) / 1e6:.3f} M node-upd/s")
        # every GPU result of the same 64 steps against the oracle's
        res["vs_oracle_64_steps"] = vs_oracle(w, k_cpu, ophi, opsi, h, eps, band)

    line = {
        "metric": METRIC, "value": value, "unit": "node-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "stream_circles: 2048^2 cells, 4 seeded circles, 8-mode sine "
                               "stream function x cos(pi t/2), 1024 steps, CFL 0.8",
                   "grid_nodes": [n + 1, n + 1], "time_steps_per_step": inner,
                   "state": "f32", "foot_coordinates": "f64", "seed": w["seed"]},
        "hbm_gbps_algorithmic": gbps,
        "roofline": roofline,
        "cpu_baseline": cpu,
        **res,
    }
    print(json.dumps(line), flush=True)
    return 0


def state_errors(g, st, ref, h, eps, band):
    """Normwise errors of a state against a reference state of the same FP64
    context: phi over max|phi_ref|, psi over max|psi_ref| and over
    max(max|psi_ref|, max|phi_ref|/h), and the L1 shape error between them."""
    import numpy as np  # noqa: F401
    import torch
    out = g.norms(st, ref, eps, band)
    grid = lambda t: g._grid_view(t)  # noqa: E731  (the valid nodes of a plane)
    max_psi = max(float(grid(ref[1 + a]).abs().max()) for a in range(g.dim))
    max_phi = out[7]
    return {"phi": out[0] / max_phi, "psi": out[1] / max_psi,
            "psi_scaled": out[1] / max(max_psi, max_phi / h), "l1_shape": out[2],
            "linf_band": out[3], "nonfinite": out[6], "max_abs_phi_ref": max_phi,
            "max_abs_psi_ref": max_psi}


def vs_oracle(w, steps, ophi, opsi, h, eps, band):
    """The FP32 and FP64 GPU states after `steps` steps against the oracle's."""
    import numpy as np  # noqa: F401
    import torch

    import paper_0905_3409_amd as pkg
    g64 = pkg.Grid(w["ncell"], w["lo"], w["hi"], dtype="float64")
    oref = g64.from_numpy(ophi, opsi)
    out = {"steps": steps}
    for dtype in ("float32", "float64"):
        g = pkg.Grid(w["ncell"], w["lo"], w["hi"], dtype=dtype)
        g.set_velocity(w["kind"], w["params"], w["period"])
        st = g.from_numpy(w["phi0"], w["psi0"])
        g.advance(st, 0.0, w["dt"], steps)
        torch.cuda.synchronize()
        e = state_errors(g64, st.double(), oref, h, eps, band)
        out["fp32" if dtype == "float32" else "fp64"] = e
        log(f"{dtype} after {steps} steps vs oracle: phi {e['phi']:.2e} psi {e['psi']:.2e} "
            f"(scaled {e['psi_scaled']:.2e}) L1 {e['l1_shape']:.2e}")
        del g, st
    return out


def matched_error(args, w, e32, ms32, value32):
    """FP64 throughput at the FP32 path's L1 shape error: the same physical
    problem (circles, stream function, T = 2, CFL 0.8) on the coarser grid at
    which the FP64 error equals the FP32 error at 2048^2, timed the same way."""
    import numpy as np  # noqa: F401
    import torch

    import paper_0905_3409_amd as pkg
    from paper_0905_3409_amd import inputs
    n = MATCHED_FP64_CELLS
    wm = inputs.stream_circles(n=n, steps=n // 2)
    g = pkg.Grid(wm["ncell"], wm["lo"], wm["hi"], dtype="float64")
    g.set_velocity(wm["kind"], wm["params"], wm["period"])
    ref = g.from_numpy(wm["phi0"], wm["psi0"])
    st = ref.clone()
    h = 1.0 / n
    times = []
    for k in range(1 + max(1, min(args.steps, 3))):
        st.copy_(ref)
        torch.cuda.synchronize()
        a = time.perf_counter()
        g.advance(st, 0.0, wm["dt"], wm["steps"])
        out = g.norms(st, ref, 1.5 * h, 3 * h)  # synchronises
        if k > 0:
            times.append((time.perf_counter() - a) * 1e3)
    ms = float(np.median(times))
    nodes = (n + 1) ** 2
    ratio = e32 / out[2]
    r = {"fp64_cells": [n, n], "fp64_steps": wm["steps"], "fp64_l1_shape_error": out[2],
         "fp32_l1_shape_error": e32, "ratio_fp32_over_fp64": ratio,
         "matched": bool(1 / 1.1 <= ratio <= 1.1),
         "fp64_ms_per_solution": ms, "fp32_ms_per_solution": ms32,
         "fp64_node_updates_per_s": nodes * wm["steps"] / (ms * 1e-3),
         "fp32_node_updates_per_s": value32,
         "fp32_speedup_at_matched_error": ms / ms32,
         "how": f"FP64 on {n}^2 cells with {wm['steps']} steps (CFL 0.8, T = 2) reaches the "
                "L1 shape error the FP32 path reaches on 2048^2; both times are one whole "
                "solution (advance and the shape-error reduction)"}
    log(f"matched error: fp64 {n}^2 L1 {out[2]:.3e} vs fp32 2048^2 {e32:.3e} (ratio "
        f"{ratio:.3f}); fp64 {ms:.1f} ms vs fp32 {ms32:.1f} ms per solution: fp32 "
        f"{ms / ms32:.2f}x faster")
    return r


def _oracle_rates(dim, w, steps_all, sample_nodes=20000):
    """The oracle's node-updates/s on all host threads (`steps_all` whole
    steps) and on one core (a step of `sample_nodes` nodes: the whole-grid
    cross-derivative pass plus the sampled nodes, scaled to the grid)."""
    import numpy as np

    import oracle
    nodes = int(np.prod([c + 1 for c in w["ncell"]]))
    a = time.perf_counter()
    res = oracle.advance(dim, w["ncell"], w["lo"], w["hi"], w["kind"], w["params"], w["period"],
                         w["phi0"], w["psi0"], 0.0, w["dt"], steps_all)
    t_all = time.perf_counter() - a
    threads = oracle.num_threads()
    oracle.set_threads(1)
    try:
        rng = np.random.default_rng(0)
        k = min(sample_nodes, nodes)
        pick = np.sort(rng.choice(nodes, k, replace=False))
        args = (dim, w["ncell"], w["lo"], w["hi"], w["kind"], w["params"], w["period"],
                w["phi0"], w["psi0"], 0.0, w["dt"])
        a = time.perf_counter()
        oracle.step_nodes(*args, np.zeros(0, dtype=np.int64))
        t0 = time.perf_counter() - a
        a = time.perf_counter()
        oracle.step_nodes(*args, pick)
        tk = time.perf_counter() - a
    finally:
        oracle.set_threads(threads)
    one = nodes / (t0 + max(tk - t0, 0.0) * nodes / k)
    return res, nodes * steps_all / t_all, threads, one


def bench_table(args):
    """Per-configuration results in one run (see the module docstring)."""
    import numpy as np
    import torch

    import paper_0905_3409_amd as pkg
    from paper_0905_3409_amd import inputs

    rows = []

    def gpu_run(w, dtype, steps, reps=3):
        g = pkg.Grid(w["ncell"], w["lo"], w["hi"], dtype=dtype)
        g.set_velocity(w["kind"], w["params"], w["period"])
        ref = g.from_numpy(w["phi0"], w["psi0"])
        st = ref.clone()
        g.advance(st, 0.0, w["dt"], min(steps, 8))
        times = []
        for _ in range(reps):
            st.copy_(ref)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            g.advance(st, 0.0, w["dt"], steps)
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        return g, st, ref, float(np.median(times))

    def row(name, prec, w, dtype, bpn, oracle_steps, full_errors=True):
        dim = len(w["ncell"])
        nodes = int(np.prod([c + 1 for c in w["ncell"]]))
        h = 1.0 / w["ncell"][0]
        g, st, ref, ms = gpu_run(w, dtype, w["steps"])
        rate = nodes * w["steps"] / (ms * 1e-3)
        out = g.norms(st, ref, 1.5 * h, 3 * h) if full_errors else None
        r = {"config": name, "prec": prec, "cells": list(w["ncell"]), "steps": w["steps"],
             "gpu_ms": ms, "gpu_node_updates_per_s": rate,
             "hbm_gbps_algorithmic": rate * bpn / 1e9,
             "hbm_frac": rate * bpn / 1e9 / HBM_PEAK_GBPS}
        if out is not None:
            r.update({"l1_shape_error": out[2], "linf_band_error": out[3]})
        if oracle_steps and not args.no_cpu:
            (ophi, opsi), r_all, thr, r_one = _oracle_rates(dim, w, oracle_steps)
            r.update({"oracle_node_updates_per_s": r_all, "oracle_threads": thr,
                      "oracle_node_updates_per_s_1core": r_one, "oracle_steps": oracle_steps})
            g64 = pkg.Grid(w["ncell"], w["lo"], w["hi"], dtype="float64")
            g64.set_velocity(w["kind"], w["params"], w["period"])
            s2 = g64.from_numpy(w["phi0"], w["psi0"]) if dtype == "float64" else None
            gg = g if dtype == "float64" else pkg.Grid(w["ncell"], w["lo"], w["hi"], dtype=dtype)
            if dtype != "float64":
                gg.set_velocity(w["kind"], w["params"], w["period"])
            s1 = gg.from_numpy(w["phi0"], w["psi0"])
            gg.advance(s1, 0.0, w["dt"], oracle_steps)
            torch.cuda.synchronize()
            e = state_errors(g64, s1.double(), g64.from_numpy(ophi, opsi), h, 1.5 * h, 3 * h)
            r.update({"vs_oracle_phi": e["phi"], "vs_oracle_psi": e["psi"],
                      "vs_oracle_psi_scaled": e["psi_scaled"]})
            del g64, s1, s2
        rows.append(r)
        log(f"{name} {prec}: {rate / 1e9:.3f} G node-upd/s, {r['hbm_gbps_algorithmic']:.0f} GB/s "
            f"algorithmic" + (f", oracle {r['oracle_node_updates_per_s'] / 1e6:.2f} M/s on "
                             f"{r['oracle_threads']} threads, {r['oracle_node_updates_per_s_1core'] / 1e6:.3f} M/s on 1 core"
                             if "oracle_threads" in r else ""))
        del g, st, ref
        torch.cuda.empty_cache()

    c1 = inputs.rotation_circle()
    row("C1 64^2 rotation", "FP64", c1, "float64", 48, c1["steps"])
    c2 = inputs.stream_circles()
    row("C2 2048^2 stream function", "FP64", c2, "float64", 48, 16)
    row("C2 2048^2 stream function", "FP32", c2, "float32", BYTES_PER_NODE, 16)
    c3 = inputs.vecpot_spheres()
    row("C3 256^3 vector potential", "FP32", c3, "float32", BYTES_PER_NODE_3D, 1)
    # bandwidth probes: rotation, random state (no shape error, no oracle)
    for name, ncell, steps, bpn in (("probe 2D 8192^2 rotation", (8192, 8192), 32, BYTES_PER_NODE),
                                    ("probe 3D 384^3 rotation", (384, 384, 384), 16,
                                     BYTES_PER_NODE_3D)):
        dim = len(ncell)
        A = np.zeros((dim, dim))
        A[0, 1], A[1, 0] = -2.0 * np.pi, 2.0 * np.pi
        g = pkg.Grid(ncell, dtype="float32")
        g.set_velocity(inputs.AFFINE, inputs.affine_params(np.zeros(dim), np.full(dim, 0.5), A), 0.0)
        st = torch.zeros((1 + dim, g.plane), dtype=torch.float32, device="cuda")
        st[0].normal_()
        st[1:].normal_()
        dt = 0.9 / ncell[0] / (np.pi * np.sqrt(2.0))
        g.advance(st, 0.0, dt, 2)
        times = []
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            g.advance(st, 0.0, dt, steps)
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        ms = float(np.median(times))
        nodes = int(np.prod([c + 1 for c in ncell]))
        rate = nodes * steps / (ms * 1e-3)
        rows.append({"config": name, "prec": "FP32", "cells": list(ncell), "steps": steps,
                     "gpu_ms": ms, "gpu_node_updates_per_s": rate,
                     "hbm_gbps_algorithmic": rate * bpn / 1e9,
                     "hbm_frac": rate * bpn / 1e9 / HBM_PEAK_GBPS})
        log(f"{name}: {rate / 1e9:.3f} G node-upd/s, {rate * bpn / 1e9:.0f} GB/s algorithmic")
        del g, st
        torch.cuda.empty_cache()

    def fmt(v, f):
        return "-" if v is None else format(v, f)
    log("| config | prec | GPU node-upd/s | HBM GB/s algorithmic (of 8 TB/s) | oracle node-upd/s "
        "(threads / 1 core) | E_L1 / E_Linf band | vs oracle phi / psi (psi scaled) |")
    log("|---|---|---|---|---|---|---|")
    for r in rows:
        orc = (f"{r['oracle_node_updates_per_s'] / 1e6:.2f} M ({r['oracle_threads']}) / "
               f"{r['oracle_node_updates_per_s_1core'] / 1e6:.3f} M" if "oracle_threads" in r else "-")
        err = (f"{r['l1_shape_error']:.3e} / {r['linf_band_error']:.3e}"
               if "l1_shape_error" in r else "-")
        vso = (f"{r['vs_oracle_phi']:.1e} / {r['vs_oracle_psi']:.1e} ({r['vs_oracle_psi_scaled']:.1e}) "
               f"after {r['oracle_steps']} steps" if "vs_oracle_phi" in r else "-")
        log(f"| {r['config']} | {r['prec']} | {r['gpu_node_updates_per_s'] / 1e9:.3f} G | "
            f"{r['hbm_gbps_algorithmic']:.0f} ({r['hbm_frac']:.2f}) | {orc} | {err} | {vso} |")
    line = {"metric": "per-configuration results (GPU, oracle, errors)",
            "value": rows[2]["gpu_node_updates_per_s"], "unit": "node-updates/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": rows[2]["gpu_ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "every configuration once (table)"},
            "rows": rows, "roofline": None, "cpu_baseline": None,
            "paper_context": PAPER_CPU_CONTEXT}
    print(json.dumps(line), flush=True)
    return 0


def bench_batched(args):
    import numpy as np
    import torch

    import paper_0905_3409_amd as pkg
    from paper_0905_3409_amd import inputs

    dev = torch.device("cuda", 0)
    w = inputs.batched_stream_circles()
    probs = w["problems"]
    inner = args.inner or w["steps"]
    nodes = sum((p["ncell"][0] + 1) * (p["ncell"][1] + 1) for p in probs)
    log(f"workload {w['name']}: {len(probs)} grids, {nodes} nodes, {inner} steps/bench step")
    b = pkg.Batch([p["ncell"] for p in probs], dtype="float32")
    for k, p in enumerate(probs):
        b.set_velocity(k, w["kind"], p["params"], w["period"])
    ref = b.from_numpy([(p["phi0"], p["psi0"]) for p in probs])
    st = ref.clone()
    s = torch.cuda.Stream()
    if args.profile:
        # the shapes the timed run would use, then a short advance
        if args.tiles:
            b.set_tiles([int(v) for v in args.tiles.split(",")])
        else:
            scratch = ref.clone()
            b.autotune(scratch, w["dt"], steps=8)
            del scratch
        torch.cuda.synchronize()
        log(f"profile: wave widths per class {b.get_tiles()}; the last "
            f"{args.inner or 16} step launches are the measured ones")
        b.advance(st, 0.0, w["dt"], args.inner or 16)
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        log(f"profile: batched FP32 steps on {nodes} nodes, then a {nbytes} B device copy")
        return 0
    if args.tiles:
        b.set_tiles([int(v) for v in args.tiles.split(",")])
        log(f"wave widths per class {b.get_tiles()} (given)")
    else:
        scratch = ref.clone()
        tune_ms = b.autotune(scratch, w["dt"], steps=8)
        del scratch
        log(f"autotune: wave widths per class {b.get_tiles()}, {tune_ms:.3f} ms for 8 steps")

    def bench_step(ev=None):
        with torch.cuda.stream(s):
            if ev is not None:
                ev[0].record(s)
            b.advance(st, 0.0, w["dt"], inner, graph=True, stream=s)
            if ev is not None:
                ev[1].record(s)
        s.synchronize()

    torch.cuda.synchronize()  # the state was made on the current stream; steps run on s
    for _ in range(args.warmup):
        bench_step()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        bench_step(events[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    adv_ms = float(np.mean([a.elapsed_time(c) for a, c in events]))
    kernel_us = adv_ms * 1e3 / inner  # per step launch (the table launch is < 0.1 %)
    value = nodes * inner / (ms_per_step * 1e-3)
    log(f"batched fp32: {ms_per_step:.2f} ms/bench step, advance {adv_ms:.2f} ms, "
        f"{kernel_us:.2f} us per step launch, {value / 1e9:.2f} G node-upd/s")
    # flops per node: the hardware count of the committed counter summary
    # while it matches the kernel's source, else the formulated lower bound
    issue = valu_issue("k_batch_step_f32_512grids.md", BATCH_KERNEL_SOURCES, kernel_us)
    fpn = issue["hw_flops_per_node"] if issue else ALG_FLOPS_PER_NODE_LOW
    tflops = nodes * fpn / (kernel_us * 1e-6) / 1e12
    gbps = nodes * BYTES_PER_NODE / (kernel_us * 1e-6) / 1e9
    roofline = {"bound": "alu", "achieved": tflops, "peak": VALU_F32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": tflops / VALU_F32_PEAK_TFLOPS,
                "traffic": traffic_record("k_batch_step_f32_512grids.md", BATCH_KERNEL_SOURCES),
                "kernel": "k_batch_step<float, CENTRAL, taylor>",
                "flops_per_node": fpn,
                "flops_counted": "hardware (rocprofv3)" if issue else "formulated lower bound",
                "flops_per_launch": nodes * fpn, "avg_launch_us": kernel_us,
                "hbm_gbps": gbps, "hbm_frac": gbps / HBM_PEAK_GBPS,
                "bytes_per_launch": nodes * BYTES_PER_NODE, "valu": issue}
    # the FP32 final states of every 8th grid against an FP64 batched run of
    # the same steps (the FP64 batch matches the oracle; its grids are
    # checked against FP64 single grids bit for bit in the tests)
    res = {}
    if not args.no_fp64:
        # one advance of `inner` steps from the initial state, as timed (the
        # copy runs on the current stream and the advance on s: wait for it)
        st.copy_(ref)
        torch.cuda.synchronize()
        bench_step()
        torch.cuda.synchronize()
        fin32 = {k: b.to_numpy(st, k) for k in range(0, len(probs), 8)}
        b64 = pkg.Batch([p["ncell"] for p in probs], dtype="float64")
        for k, p in enumerate(probs):
            b64.set_velocity(k, w["kind"], p["params"], w["period"])
        st64 = b64.from_numpy([(p["phi0"], p["psi0"]) for p in probs])
        b64.advance(st64, 0.0, w["dt"], inner)
        torch.cuda.synchronize()
        rows = []
        for k, f32 in fin32.items():
            p = probs[k]
            gk = pkg.Grid(p["ncell"], (0.0, 0.0), (1.0, 1.0), dtype="float64")
            hk = 1.0 / max(p["ncell"])
            ref = gk.from_numpy(*b64.to_numpy(st64, k))
            d = state_errors(gk, gk.from_numpy(*f32), ref, hk, 1.5 * hk, 3 * hk)
            n0 = gk.norms(ref, gk.from_numpy(p["phi0"], p["psi0"]), 1.5 * hk, 3 * hk)
            # resolved: the FP64 run returns phi to within twice its initial
            # range (on the coarsest grids the flow's filaments are not
            # resolved, |psi| grows by orders of magnitude in both precisions,
            # and the two runs differ at O(1))
            resolved = d["max_abs_phi_ref"] <= 2.0 * float(np.max(np.abs(p["phi0"])))
            rows.append((max(p["ncell"]), resolved, d["phi"], d["psi"], d["psi_scaled"],
                         d["l1_shape"] / n0[2] if n0[2] > 0 else 0.0))
            del gk, ref
        ok = [r for r in rows if r[1]]
        cols = ("phi", "psi", "psi_scaled", "l1_shape_rel")
        res["fp32_vs_fp64_final"] = {
            "grids": len(rows), "resolved_grids": len(ok),
            "smallest_resolved_cells": min(r[0] for r in ok) if ok else None,
            "largest_unresolved_cells": max((r[0] for r in rows if not r[1]), default=None),
            "median_resolved": {c: float(np.median([r[2 + i] for r in ok])) for i, c in enumerate(cols)} if ok else None,
            "worst_resolved": {c: float(max(r[2 + i] for r in ok)) for i, c in enumerate(cols)} if ok else None,
            "how": "every 8th grid, FP32 final state against an FP64 batched run of the same steps; "
                   "l1_shape_rel: the L1 shape distance between the two final states over the FP64 "
                   "run's own L1 shape error against the initial state"}
        f = res["fp32_vs_fp64_final"]
        if ok:
            log(f"fp32 vs fp64 final ({f['resolved_grids']} of {f['grids']} sampled grids resolved, "
                f"the smallest {f['smallest_resolved_cells']} cells): median phi "
                f"{f['median_resolved']['phi']:.2e} psi {f['median_resolved']['psi']:.2e}, worst phi "
                f"{f['worst_resolved']['phi']:.2e} psi {f['worst_resolved']['psi']:.2e}, L1 shape "
                f"distance {f['worst_resolved']['l1_shape_rel']:.2e} of the FP64 shape error")
        del b64, st64
    cpu = None
    if not args.no_cpu:
        import oracle
        k_cpu, sample = 8, list(range(0, len(probs), 8))
        a = time.perf_counter()
        for k in sample:
            p = probs[k]
            oracle.advance(2, p["ncell"], (0.0, 0.0), (1.0, 1.0), w["kind"], p["params"],
                           w["period"], p["phi0"], p["psi0"], 0.0, w["dt"], k_cpu)
        c = time.perf_counter()
        snodes = sum((probs[k]["ncell"][0] + 1) * (probs[k]["ncell"][1] + 1) for k in sample)
        cpu = {"value": snodes * k_cpu / (c - a), "unit": "node-updates/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"first {k_cpu} steps of every 8th of the 512 grids "
                         f"({len(sample)} grids, {snodes} nodes; FP64 oracle, OpenMP), "
                         f"{c - a:.1f} s"}
        log(f"cpu oracle: {cpu['value'] / 1e6:.2f} M node-upd/s on {cpu['cores']} threads")
        # and on one core: the same sample, one step
        threads = oracle.num_threads()
        oracle.set_threads(1)
        a = time.perf_counter()
        for k in sample:
            p = probs[k]
            oracle.advance(2, p["ncell"], (0.0, 0.0), (1.0, 1.0), w["kind"], p["params"],
                           w["period"], p["phi0"], p["psi0"], 0.0, w["dt"], 1)
        c = time.perf_counter()
        oracle.set_threads(threads)
        cpu["single_core"] = {"value": snodes / (c - a), "unit": "node-updates/s", "cores": 1,
                              "sample": f"the first step of the same {len(sample)} grids, "
                                        f"{c - a:.1f} s"}
        log(f"cpu oracle, 1 core: {snodes / (c - a) / 1e6:.3f} M node-upd/s")
    line = {
        "metric": "GALS batched node-updates/s (512 uneven 2D grids, one launch per step)",
        "value": value, "unit": "node-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched_stream_circles: 512 grids, round(2^U(5,9)) cells per "
                               "side, 4 circles and an 8-mode sine stream function each, "
                               "256 steps of dt 2/256, CFL 0.8",
                   "grids": len(probs), "nodes": nodes, "time_steps_per_step": inner,
                   "wave_widths_per_class": b.get_tiles(),
                   "wave_widths_from": "given" if args.tiles else "autotuner",
                   "graph": True, "seed": w["seed"]},
        "hbm_gbps_algorithmic": gbps,
        "roofline": roofline,
        "cpu_baseline": cpu,
        **res,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_adjoint(args):
    import numpy as np
    import torch

    import paper_0905_3409_amd as pkg
    from paper_0905_3409_amd import inputs
    from paper_0905_3409_amd.autograd import stream_params

    w = inputs.adjoint_circles()
    n = w["ncell"][0]
    nodes = (n + 1) ** 2
    steps, every, dt, eps = w["steps"], 20, w["dt"], w["eps"]
    g = pkg.Grid(w["ncell"], dtype="float32")
    g.set_velocity(pkg.STREAM_SIN, stream_params(w["target_amps"], w["modes"]), 0.0)
    tgt = g.from_numpy(w["phi0"], w["psi0"])
    g.advance(tgt, 0.0, dt, steps)
    g.set_velocity(pkg.STREAM_SIN, stream_params(w["amps"], w["modes"]), 0.0)
    st0 = g.from_numpy(w["phi0"], w["psi0"])
    st = st0.clone()
    ckpt = torch.empty(g.checkpoint_bytes(steps, every), dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    log(f"workload {w['name']}: {n}^2 cells, {len(w['amps'])} amplitudes, {steps} steps, "
        f"checkpoints every {every}")
    if args.profile:
        k = args.inner or 8
        g.advance_save(st, 0.0, dt, k, k, ckpt)
        _, lam = g.shape_loss(st, tgt, eps)
        g.adjoint(ckpt, 0.0, dt, k, k, lam)
        torch.cuda.synchronize()
        log(f"profile: {k} forward steps, {k - 1} recomputed, {k} adjoint steps")
        return 0

    def gradient(ev=None):
        st.copy_(st0)
        if ev is not None:
            ev[0].record(s)
        g.advance_save(st, 0.0, dt, steps, every, ckpt)
        if ev is not None:
            ev[1].record(s)
        loss, lam = g.shape_loss(st, tgt, eps)  # synchronises
        if ev is not None:
            ev[2].record(s)
        dS = g.adjoint(ckpt, 0.0, dt, steps, every, lam)
        if ev is not None:
            ev[3].record(s)
        torch.cuda.synchronize()
        return loss, dS

    for _ in range(args.warmup):
        gradient()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        loss, dS = gradient(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    rev_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    # the reverse sweep recomputes steps - ceil(steps / every) forward steps;
    # the rest of it is the adjoint launches (and their zero fills)
    recompute = steps - (steps + every - 1) // every
    step_us = fwd_ms * 1e3 / steps
    adj_us = (rev_ms * 1e3 - recompute * step_us) / steps
    log(f"gradient: {ms:.2f} ms (forward {fwd_ms:.2f} ms, reverse sweep {rev_ms:.2f} ms); "
        f"forward step {step_us:.1f} us, adjoint step {adj_us:.1f} us; loss {loss:.6e}")
    flops = nodes * ADJ_FLOPS_PER_NODE / (adj_us * 1e-6) / 1e12
    roofline = {"bound": "alu", "achieved": flops, "peak": VALU_F32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": flops / VALU_F32_PEAK_TFLOPS,
                "traffic": traffic_record("k_adjoint2d_stream_f32_1024.md", ADJ_KERNEL_SOURCES),
                "kernel": "k_adjoint2d_stream<float, CENTRAL, taylor>",
                "flops_per_launch": nodes * ADJ_FLOPS_PER_NODE, "avg_launch_us": adj_us,
                "avg_launch_us_from": "reverse-sweep events minus the recomputed forward steps",
                "bytes_per_launch": nodes * ADJ_BYTES_PER_NODE,
                "hbm_gbps": nodes * ADJ_BYTES_PER_NODE / (adj_us * 1e-6) / 1e9}
    cpu = None
    if not args.no_cpu:
        import oracle
        k_cpu = 2
        a = time.perf_counter()
        oracle.grad_cs(w["ncell"], (0.0, 0.0), (1.0, 1.0), stream_params(w["amps"], w["modes"]),
                       0.0, w["phi0"], w["psi0"], 0.0, dt, k_cpu,
                       phi_target=w["phi0"], eps=eps)
        b = time.perf_counter()
        per_grad = (b - a) * steps / k_cpu
        cpu = {"value": 1.0 / per_grad, "unit": "gradients/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"complex-step gradient (16 complex advances) over the first {k_cpu} of "
                         f"the {steps} steps at 1024^2, {b - a:.1f} s, scaled to {steps} steps"}
        log(f"cpu oracle: {per_grad:.0f} s per gradient on {cpu['cores']} threads")
    line = {
        "metric": "GALS gradient evaluations/s (dL/da, 16 stream-function amplitudes)",
        "value": 1e3 / ms, "unit": "gradients/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "adjoint_circles: 1024^2 cells, 4 seeded circles, steady 16-mode "
                               "sine stream function, 200 steps at CFL 0.8, checkpoints every "
                               "20, smoothed-Heaviside loss against a seeded target",
                   "grid_nodes": [n + 1, n + 1], "time_steps": steps, "checkpoint_every": every,
                   "state": "f32", "adjoint_state": "f64", "seed": w["seed"]},
        "forward_ms": fwd_ms, "reverse_ms": rev_ms, "forward_step_us": step_us,
        "adjoint_step_us": adj_us,
        "node_steps_per_s": nodes * (2 * steps + recompute) / (ms * 1e-3),
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_variants(args):
    import numpy as np
    import torch

    import paper_0905_3409_amd as pkg
    from paper_0905_3409_amd import inputs

    w = inputs.stream_circles()
    inner = args.inner or w["steps"]
    n = w["ncell"][0]
    nodes = (n + 1) ** 2
    s = torch.cuda.current_stream()
    names = {pkg.MIXED_CENTRAL: "central (A)", pkg.MIXED_CELL: "cell-based (B)",
             pkg.MIXED_ZERO: "zero"}
    table = {}
    for mixed in (pkg.MIXED_CENTRAL, pkg.MIXED_CELL, pkg.MIXED_ZERO):
        g = pkg.Grid(w["ncell"], w["lo"], w["hi"], dtype="float32", mixed=mixed)
        g.set_velocity(w["kind"], w["params"], w["period"])
        ref = g.from_numpy(w["phi0"], w["psi0"])
        st = ref.clone()
        for psi, pname in ((pkg.PSI_SUPERCONSISTENT, "superconsistent"), (pkg.PSI_HEUN, "heun")):
            g.set_psi_update(psi)
            times = []
            for k in range(args.warmup + args.steps):
                st.copy_(ref)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(s)
                g.advance(st, 0.0, w["dt"], inner)
                b.record(s)
                torch.cuda.synchronize()
                if k >= args.warmup:
                    times.append(a.elapsed_time(b))
            ms = float(np.mean(times))
            norms = g.norms(st, ref, 1.5 / n, 3.0 / n)
            us = ms * 1e3 / inner
            table[f"{names[mixed]}, {pname}"] = {
                "step_us": us, "node_updates_per_s": nodes / (us * 1e-6),
                "l1_shape_error": norms[2]}
            log(f"{names[mixed]:15s} {pname:15s}: {us:6.2f} us/step, "
                f"{nodes / us / 1e3:.1f} G node-upd/s, L1 shape error {norms[2]:.3e}")
        del g, ref, st
    for m in names.values():
        table[f"{m}, heun / superconsistent time"] = (table[f"{m}, heun"]["step_us"] /
                                                     table[f"{m}, superconsistent"]["step_us"])
    # inflow boundary conditions (sec. 4.1): the same field on a box shifted
    # so that the flow enters through parts of every face
    lo, hi = (-0.1, -0.1), (1.1, 1.1)
    coords = inputs.node_grid(w["ncell"], lo, hi)
    phi_b, psi_b = inputs.sdf_union(coords, w["centres"], w["radii"])
    bcs = {pkg.BC_NEUMANN: "projection", pkg.BC_INFLOW: "Dirichlet data",
           pkg.BC_INFLOW_NEUMANN: "Neumann face scheme"}
    for bc, bname in bcs.items():
        g = pkg.Grid(w["ncell"], lo, hi, dtype="float32", bc=bc)
        g.set_velocity(w["kind"], w["params"], w["period"])
        ref = g.from_numpy(phi_b, psi_b)
        st = ref.clone()
        if bc == pkg.BC_INFLOW:
            data = ref.clone()  # fixed data: the initial state, phi_t = 0
            phit = torch.zeros(g.plane, dtype=torch.float32, device="cuda")
            g.set_inflow_data(data, phit)
        times = []
        for k in range(args.warmup + args.steps):
            st.copy_(ref)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            g.advance(st, 0.0, w["dt"], inner)
            b.record(s)
            torch.cuda.synchronize()
            if k >= args.warmup:
                times.append(a.elapsed_time(b))
        us = float(np.mean(times)) * 1e3 / inner
        table[f"inflow box, {bname}"] = {"step_us": us, "node_updates_per_s": nodes / (us * 1e-6)}
        log(f"inflow box {bname:20s}: {us:6.2f} us/step")
        del g, ref, st
    for bname in ("Dirichlet data", "Neumann face scheme"):
        table[f"inflow box, {bname} / projection time"] = (
            table[f"inflow box, {bname}"]["step_us"] / table["inflow box, projection"]["step_us"])
    main = table["cell-based (B), superconsistent"]
    flops = nodes * VARIANT_B_FLOPS_PER_NODE / (main["step_us"] * 1e-6) / 1e12
    line = {
        "metric": "GALS node-updates/s, cell-based (B) cross derivatives (2048^2, FP32)",
        "value": main["node_updates_per_s"], "unit": "node-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main["step_us"] * inner / 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "stream_circles: 2048^2 cells, 4 seeded circles, 8-mode sine "
                               "stream function x cos(pi t/2), 1024 steps, CFL 0.8",
                   "time_steps_per_step": inner, "seed": w["seed"]},
        "roofline": {"bound": "alu", "achieved": flops, "peak": VALU_F32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": flops / VALU_F32_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_step2d_stream<float, CELL, taylor, superconsistent>",
                     "flops_per_launch": nodes * VARIANT_B_FLOPS_PER_NODE,
                     "avg_launch_us": main["step_us"]},
        "variants": table,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_volume(args):
    import numpy as np
    import torch

    import paper_0905_3409_amd as pkg
    from paper_0905_3409_amd import inputs

    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "volume_loss.json")))
    table = {}
    timing = None
    for shape in ("sphere", "cube"):
        for n in golden["n"]:
            w = inputs.leveque_shape(shape, n)
            g = pkg.Grid(w["ncell"], w["lo"], w["hi"], dtype="float64")
            g.set_velocity(w["kind"], w["params"], w["period"])
            ref = g.from_numpy(w["phi0"], w["psi0"])
            st = ref.clone()
            s = torch.cuda.current_stream()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            g.advance(st, 0.0, w["dt"], w["steps"])
            b.record(s)
            out = g.norms(st, ref, 1.5 / n, 3.0 / n)
            ms = a.elapsed_time(b)
            loss = 100.0 * (out[4] - out[5]) / out[5]
            paper = golden[shape][golden["n"].index(n)]
            table[f"{shape} n={n}"] = {"volume_change_percent": loss, "paper_percent": paper,
                                       "steps": w["steps"], "advance_ms": ms}
            log(f"{shape:6s} n={n:3d}: volume change {loss:+.2f} % (paper {paper:+.1f} %), "
                f"{w['steps']} steps in {ms:.1f} ms")
            if n == golden["n"][-1] and shape == "sphere":
                nodes = (n + 1) ** 3
                timing = (nodes, w["steps"], ms)
            del g, ref, st
            torch.cuda.empty_cache()
    nodes, steps, ms = timing
    value = nodes * steps / (ms * 1e-3)
    line = {
        "metric": "GALS node-updates/s, 3D deformation test (200^3, FP64), and volume change "
                  "against the paper's tables",
        "value": value, "unit": "node-updates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "leveque_shape: LeVeque 3D deformation x cos(pi t/2.5), dt = h, "
                               "t = 0..2.5; sphere r 0.15 and cube 0.3 at (0.35,0.35,0.35)",
                   "grids": golden["n"], "volume": "prod(h) sum H_eps(-phi), eps = 1.5 h"},
        "volume_table": table,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    return 0


def device_copy_rate(nbytes=1 << 30, reps=10):
    """What a plain device-to-device copy attains on this GPU in this run
    (torch's copy_ of a 1 GiB FP32 tensor: the runtime's copy kernel), as
    context for the probe's bandwidth: read + written bytes over the median
    time of reps copies."""
    import numpy as np
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    ms = float(np.median(times))
    del src, dst
    torch.cuda.empty_cache()
    return {"gbps": 2 * nbytes / (ms * 1e-3) / 1e9, "bytes_moved": 2 * nbytes, "ms": ms,
            "how": "torch copy_ of a 1 GiB FP32 tensor, median of 10"}


def bench_probe(args):
    """Labelled bandwidth probe, not one of the workloads: rigid rotation (the
    cheapest velocity) on working sets far beyond the 256 MB Infinity Cache,
    2D 8192^2 and 3D 384^3, FP32."""
    import numpy as np
    import torch

    import paper_0905_3409_amd as pkg
    from paper_0905_3409_amd import inputs

    table = {}
    cases = [("2d", (8192, 8192), 32, BYTES_PER_NODE, PROBE_FLOPS_PER_NODE_2D),
             ("3d", (384, 384, 384), 16, BYTES_PER_NODE_3D, PROBE_FLOPS_PER_NODE_3D)]
    if args.profile:  # one case (--probe-case) for a few steps, then a plain copy
        cases = [(name, ncell, args.inner or 4, bpn, fpn)
                 for name, ncell, _, bpn, fpn in cases if name == args.probe_case]
    for name, ncell, steps, bpn, fpn in cases:
        dim = len(ncell)
        A = np.zeros((dim, dim))
        A[0, 1], A[1, 0] = -2.0 * np.pi, 2.0 * np.pi
        params = inputs.affine_params(np.zeros(dim), np.full(dim, 0.5), A)
        dt = 0.9 / ncell[0] / (np.pi * np.sqrt(2.0))  # CFL 0.9 at the corners
        g = pkg.Grid(ncell, dtype="float32")
        g.set_velocity(inputs.AFFINE, params, 0.0)
        st = torch.zeros((1 + dim, g.plane), dtype=torch.float32, device="cuda")
        st[0].normal_()
        st[1:].normal_()
        g.advance(st, 0.0, dt, 2)  # warm-up
        times = []
        for _ in range(1 if args.profile else max(args.steps, 1)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            g.advance(st, 0.0, dt, steps)
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        us = float(np.median(times)) * 1e3 / steps
        nodes = int(np.prod([c + 1 for c in ncell]))
        gbps = nodes * bpn / (us * 1e-6) / 1e9
        tflops = nodes * fpn / (us * 1e-6) / 1e12
        table[name] = {"cells": list(ncell), "step_us": us,
                       "node_updates_per_s": nodes / (us * 1e-6),
                       "state_bytes": int(st.numel() * 4), "hbm_gbps_algorithmic": gbps,
                       "hbm_frac": gbps / HBM_PEAK_GBPS, "tflops": tflops,
                       "valu_frac": tflops / VALU_F32_PEAK_TFLOPS}
        log(f"probe {name} {ncell}: {us:.1f} us/step, {nodes / us / 1e3:.1f} G node-upd/s, "
            f"{gbps:.0f} GB/s algorithmic ({gbps / HBM_PEAK_GBPS:.2f} of HBM), "
            f"{tflops:.1f} TFLOP/s ({tflops / VALU_F32_PEAK_TFLOPS:.2f} of VALU)")
        del g, st
        torch.cuda.empty_cache()
    if args.profile:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        torch.empty_like(src).copy_(src)  # plain copy: reads and writes exactly 256 MiB
        torch.cuda.synchronize()
        return 0
    main = table["2d"]
    copy = device_copy_rate()
    log(f"plain device copy: {copy['gbps']:.0f} GB/s; the 2D probe step moves its bytes at "
        f"{main['hbm_gbps_algorithmic'] / copy['gbps']:.2f} of that rate")
    line = {
        "metric": "bandwidth probe (not a workload): rigid rotation, FP32, 2D 8192^2 and "
                  "3D 384^3", "value": main["node_updates_per_s"], "unit": "node-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": main["step_us"] / 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "probe: rotation about the centre at 2 pi per unit time, CFL 0.9 "
                               "at the corners, random state"},
        "probe": table,
        "roofline": {"bound": "hbm", "achieved": main["hbm_gbps_algorithmic"],
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": main["hbm_frac"],
                     "traffic": traffic_record("k_step2d_affine_probe_8192.md",
                                               SINGLE_KERNEL_SOURCES),
                     "kernel": "k_step2d_affine<float, CENTRAL, superconsistent>",
                     "bytes_per_launch": (8193 ** 2) * BYTES_PER_NODE,
                     "avg_launch_us": main["step_us"],
                     "alu": {"flops_per_node": PROBE_FLOPS_PER_NODE_2D,
                             "achieved_tflops": main["tflops"],
                             "frac_of_nonpacked_fp32_peak": main["valu_frac"]},
                     "device_copy": dict(copy, probe_frac_of_copy=main["hbm_gbps_algorithmic"]
                                         / copy["gbps"])},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_3d(args):
    import numpy as np
    import torch

    import paper_0905_3409_amd as pkg
    from paper_0905_3409_amd import inputs

    w = inputs.vecpot_spheres()
    inner = args.inner or w["steps"]
    n = w["ncell"][0]
    h = 1.0 / n
    nodes = (n + 1) ** 3
    eps, band = 1.5 * h, 3 * h
    log(f"workload {w['name']} {n}^3 cells, {inner} steps/bench step, dt={w['dt']:.6g}")
    pts = inputs.random_points(7, 1_000_000, 3)

    def run(dtype, steps, timed):
        g = pkg.Grid(w["ncell"], w["lo"], w["hi"], dtype=dtype)
        g.set_velocity(w["kind"], w["params"], w["period"])
        ref = g.from_numpy(w["phi0"], w["psi0"])
        st = ref.clone()
        times = []
        for k in range(timed):
            st.copy_(ref)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            g.advance(st, 0.0, w["dt"], steps)
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        return g, st, ref, times

    if args.profile:
        steps = args.inner or 8
        g, st, _, _ = run("float32", steps, 1)
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        torch.empty_like(src).copy_(src)  # plain copy: reads and writes exactly 256 MiB
        torch.cuda.synchronize()
        log(f"profile: {steps} FP32 steps on {nodes} nodes, then a {nbytes} B device copy")
        return 0
    g32, st32, ref32, _ = run("float32", min(inner, 8), max(args.warmup, 1))  # warm-up
    del g32, st32, ref32
    torch.cuda.empty_cache()
    g32, st32, ref32, times = run("float32", inner, args.steps)
    adv_ms = float(np.mean(times))
    kernel_us = adv_ms * 1e3 / inner
    value = nodes * inner / (adv_ms * 1e-3)
    n32 = g32.norms(st32, ref32, eps, band)
    # curvature at 1e6 points at t = T
    dpts = torch.from_numpy(np.ascontiguousarray(pts)).to("cuda")
    g32.eval_points(st32, dpts)  # warm-up
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    g32.eval_points(st32, dpts)
    b.record()
    torch.cuda.synchronize()
    eval_ms = a.elapsed_time(b)
    log(f"fp32: advance {adv_ms:.1f} ms, step kernel {kernel_us:.1f} us, "
        f"{value / 1e9:.2f} G node-upd/s, L1 shape err {n32[2]:.3e}; 1e6 point evals "
        f"{eval_ms:.3f} ms")
    fin32 = g32.to_numpy(st32)  # the FP32 final state, for the comparison with FP64
    del g32, st32, ref32
    torch.cuda.empty_cache()
    res = {}
    if not args.no_fp64:
        g64, st64, ref64, t64 = run("float64", inner, 1)
        n64 = g64.norms(st64, ref64, eps, band)
        res["fp64"] = {"value": nodes * inner / (t64[0] * 1e-3), "advance_ms": t64[0],
                       "l1_shape_error": n64[2], "linf_band_error": n64[3]}
        res["l1_shape_error_ratio_fp32_over_fp64"] = n32[2] / n64[2] if n64[2] > 0 else None
        # the FP32 final state against the FP64 one (the FP64 path matches the
        # oracle to 1e-12), both after the whole run
        d = state_errors(g64, g64.from_numpy(*fin32), st64, h, eps, band)
        res["fp32_vs_fp64_final"] = d
        log(f"fp64: advance {t64[0]:.1f} ms, {res['fp64']['value'] / 1e9:.2f} G node-upd/s, "
            f"L1 shape err {n64[2]:.3e}; fp32 vs fp64 final: phi {d['phi']:.2e} "
            f"psi {d['psi']:.2e} L1 {d['l1_shape']:.2e}")
        del g64, st64, ref64
    gbps = nodes * BYTES_PER_NODE_3D / (kernel_us * 1e-6) / 1e9
    tflops = nodes * FLOPS_PER_NODE_3D / (kernel_us * 1e-6) / 1e12
    line = {
        "metric": "GALS node-updates/s, 3D tricubic step (256^3, FP32)", "value": value,
        "unit": "node-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": adv_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "vecpot_spheres: 256^3 cells, 8 seeded spheres, curl of a "
                               "6-mode sine vector potential x cos(pi t/3), 512 steps, CFL 0.9",
                   "time_steps_per_step": inner, "seed": w["seed"],
                   "curvature_points": int(pts.shape[0])},
        "fp32_l1_shape_error": n32[2], "fp32_linf_band_error": n32[3],
        "eval_points_ms": eval_ms,
        "roofline": {"bound": "alu", "achieved": tflops, "peak": VALU_F32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / VALU_F32_PEAK_TFLOPS,
                     "traffic": traffic_record("k_step3d_vecpot_f32_256.md",
                                               SINGLE_KERNEL_SOURCES),
                     "kernel": "k_step3d_vecpot<float, CENTRAL, shift, superconsistent>",
                     "flops_per_launch": nodes * FLOPS_PER_NODE_3D, "avg_launch_us": kernel_us,
                     "hbm_gbps": gbps, "hbm_frac": gbps / HBM_PEAK_GBPS},
        "cpu_baseline": None,
        **res,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
