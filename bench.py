#!/usr/bin/env python3
"""Throughput of the weighted Gerchberg-Saxton hologram loop on one MI355X.

A step is one call of the library's WGS loop: the workload's iterations of
forward transform -> farfield weight update -> adjoint transform -> phase
projection, on synthetic inputs already resident in HBM.  The default
workload is the full-field 2D stand-in (1024 x 1024 SLM, 400 spots from 50
bilinearly interpolated isoplanatic patches x 8 Zernike modes, 100 WGS
iterations per step).

Printed (one JSON line): spot x pixel kernel evaluations per second over
forward + adjoint (value), WGS iterations per second, the fraction of the
FP32 vector peak, the roofline of the dominant kernel from HIP events on
the library's stream, and the FP64 CPU oracle timed on a bounded sample of
the same workload on the host cores (with the GPU's error against it).
"""

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X FP32 vector, AMD specification
METRIC = ("spot·pixel kernel evals/s (fwd+adj) and WGS iters/s; "
          "% FP32 VALU peak")


def flops_per_eval(D):
    # D phase multiply-adds (2 flops each), range reduction (1), sin and
    # cos (1 each), complex multiply-accumulate as 4 FMAs (8 flops)
    return 2 * D + 11


# Issue costs of the instructions every evaluation needs, in cycles of the
# nominal 2.4 GHz clock per wave64 instruction per SIMD: an FP32 FMA, a
# hardware sine or cosine, and one 32x32x16 bf16 matrix-core product.  They
# are measured when the benchmark starts, by the committed microbenchmark
# (libash_ubench.so, include/ash_ubench.h), not typed in.  A 32 x 32 block
# of evaluations needs 32 sines and cosines, 32 FMAs and `groups`
# matrix-core products at the least (vector and matrix-core issue do not
# overlap on this chip).
ISSUE = {}
SIMDS, CLOCK_HZ = 256 * 4, 2.4e9
# FP32 issue slots of the vector units: 256 CUs x 64 lanes x 2.4 GHz
SLOT_RATE = 256 * 64 * 2.4e9


MIX = {}   # (groups, reduce, moments) -> (evals/s, waves per SIMD)


def measure_issue_costs(device=0):
    from paper_2505_08777_amd.ubench import issue_rates
    r = issue_rates(device)
    ISSUE.clear()
    ISSUE.update(r)
    return r


def mix_ceiling(groups, reduce=False, moments=False):
    """The transforms' issue ceiling: evaluations/s of their irreducible
    instruction mix on every SIMD (libash_ubench's k_mix, measured on first
    use), and the occupancy it was reached at."""
    key = (int(groups), bool(reduce), bool(moments))
    if key not in MIX:
        from paper_2505_08777_amd.ubench import mix_ceiling as measure
        MIX[key] = measure(*key)
    return MIX[key]


def issue_ceiling(groups, cycles=None):
    """Evaluations/s if every SIMD issued only the irreducible work."""
    c = cycles or ISSUE
    per_block = 32 * c["trans"] + 32 * c["fma"] + groups * c["mfma"]
    return SIMDS * CLOCK_HZ * 1024 / per_block


def dtype_label(info):
    """The arithmetic of the path: FP32 values and sums, with the phase a
    sum of exact products of bf16 pieces on the matrix cores."""
    return ("f32 (phase: bf16-piece products on the matrix cores with FP32 "
            "accumulation, remainder terms in %s pieces, offsets / slopes / "
            "nearfield phases in 3; FP64 tile offsets at set-up)"
            % (info["pieces"],))


def alu_roofline(kernel, evals_per_launch, ms_avg, launches, D, groups,
                 traffic=None, traffic_src=None, reduce=False, moments=False,
                 flops=None, ceiling=None):
    """Roofline of a transform kernel in algorithmic FP32 flops.

    The peak is the issue ceiling: the evaluations per second of the
    transform's irreducible instruction mix (per 32 x 32 block: `groups`
    matrix-core products for the phases, 32 sines and cosines, 32 FMAs, or
    for the moment transform 8 more products instead of the FMAs) measured
    on all 1024 SIMDs at start-up, expressed in the same algorithmic flops
    per evaluation.  The FP32 vector peak is given beside it: part of each
    evaluation runs on the matrix cores, so the fraction of the vector peak
    alone can pass 1.
    """
    F = flops if flops is not None else flops_per_eval(D)
    ceil, occ = ceiling or mix_ceiling(groups, reduce, moments)
    achieved = evals_per_launch * F / (ms_avg * 1e-3) / 1e12
    peak = F * ceil / 1e12
    return {"bound": "alu", "kernel": kernel, "achieved": achieved,
            "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": traffic, "traffic_unit": "bytes/launch",
            "traffic_source": traffic_src, "avg_launch_ms": ms_avg,
            "launches": launches, "flops_per_eval": F,
            "evals_per_launch": evals_per_launch,
            "peak_basis": "issue ceiling: the irreducible instruction mix of "
                          "a 32x32 block (%d matrix-core products, 32 "
                          "sines/cosines, %s) measured on all SIMDs at "
                          "start-up (libash_ubench k_mix, %d waves/SIMD): "
                          "%.4g evaluations/s"
                          % (groups, "8 more products" if moments
                             else "32 FMAs", occ, ceil),
            "ceiling_evals_per_s": ceil,
            "fp32_vector_peak": FP32_VECTOR_PEAK_TFLOPS,
            "frac_of_fp32_vector_peak": achieved / FP32_VECTOR_PEAK_TFLOPS}


def issue_model(evals_per_s, groups, cycles=None):
    """The additive model: the separate issue costs of the block's sines,
    cosines, FMAs and matrix-core products summed (an upper bound on the
    block's cost, since the three units overlap partly)."""
    c = cycles or ISSUE
    ceil = issue_ceiling(groups, c)
    return {"additive_ceiling_evals_per_s": ceil,
            "achieved_evals_per_s": evals_per_s,
            "frac_of_additive": evals_per_s / ceil, "groups": groups,
            "cycles": {k: c[k] for k in ("fma", "trans", "mfma")}}


def slot_model(evals_per_s, D, cycles=None):
    """The vector-unit slot model of '% FP32 VALU peak': per evaluation
    (D + 4)/2 packed-FMA slots + 1 range reduction + r_sin + r_cos, r = the
    measured transcendental cost in FMA slots, against 256 x 64 x 2.4e9
    slots/s (it prices the phase multiply-adds on the vector unit)."""
    c = cycles or ISSUE
    r = c["trans"] / c["fma"]
    s_eval = (D + 4) / 2.0 + 1.0 + 2.0 * r
    return {"pct": 100.0 * evals_per_s * s_eval / SLOT_RATE,
            "slots_per_eval": s_eval, "r_trans": r,
            "note": "prices the D phase multiply-adds on the vector unit; "
                    "here they run on the matrix cores, so this reads above "
                    "100 %"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="volume1920",
                    choices=["plain256", "field1024", "volume1920",
                             "grad1024", "batch64", "batch64small",
                             "principal1024", "coefgrad1024", "feedback1024",
                             "quality1024"],
                    help="grad1024 times the differentiable form (Adam steps "
                         "of the spot-amplitude loss with TV); principal1024 "
                         "the WGS loop on 8 principal isoplanatic modes of a "
                         "27-mode calibration; coefgrad1024 the gradient in "
                         "the kernel coefficients (moment transform) on the "
                         "grad1024 inputs; feedback1024 a closed WGS loop on "
                         "simulated spot measurements with phase fixing; "
                         "quality1024 the windowed Strehl proxy of three "
                         "corrections; "
                         "batch64 the batched form (64 holograms' WGS "
                         "loops together), batch64small the same for 64 "
                         "small holograms (256..512, 5..200 spots)")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch64: skip the autotuner (default range length)")
    ap.add_argument("--form", choices=["tuned", "one_launch", "per_phase"],
                    default="tuned",
                    help="batch workloads: run the form the tuner chose, or "
                         "force one (after tuning)")
    ap.add_argument("--iters", type=int, default=None,
                    help="WGS iterations per step (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="also time the WGS step captured once in a HIP graph "
                         "and replayed (default for plain256, whose loop is "
                         "launch-bound)")
    ap.add_argument("--event-stride", type=int, default=8,
                    help="WGS workloads: bracket one transform launch in "
                         "every this many with HIP events (each event pair "
                         "costs stream time)")
    ap.add_argument("--ubench", action="store_true",
                    help="only measure the issue costs (libash_ubench) and "
                         "print them, then exit")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many "
                         "MiB (for scaling HBM byte counters), then exit")
    return ap.parse_args()


def calibrate_copy(mib):
    """A plain copy of known size: reads and writes mib MiB once each."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}),
          flush=True)


def kernel_source_sha256():
    src = os.path.join(ROOT, "paper_2505_08777_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def profiled_traffic(workload, kernel, summary="wgs_kernels", profiles=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summary
    of this workload (FETCH_SIZE and WRITE_SIZE, scaled by what they read
    for a plain copy), or None when the summary was taken on other kernel
    source than the one built here."""
    profiles = profiles or os.path.join(ROOT, "profiles")
    path = os.path.join(profiles, "%s_%s.txt" % (summary, workload))
    if not os.path.exists(path):
        return None, None
    sha = kernel_source_sha256()
    rec, val = None, None
    for line in open(path):
        if line.startswith("kernels_hip_sha256:"):
            rec = line.split(":", 1)[1].strip()
        if line.startswith("traffic_bytes_per_launch[%s]:" % kernel):
            val = float(line.split(":", 1)[1].split()[0])
    if rec != sha or val is None:
        return None, os.path.relpath(path, ROOT)
    return val, os.path.relpath(path, ROOT)


def profiled_counters(workload, kernel, summary="wgs_kernels", profiles=None):
    """Per-dispatch counters of `kernel` (display name, e.g.
    'k_forward<3, false>') from the committed summary's counter table, or
    None when the summary was taken on other kernel source."""
    profiles = profiles or os.path.join(ROOT, "profiles")
    path = os.path.join(profiles, "%s_%s.txt" % (summary, workload))
    if not os.path.exists(path):
        return None
    rec, cols, vals = None, None, {}
    for line in open(path):
        if line.startswith("kernels_hip_sha256:"):
            rec = line.split(":", 1)[1].strip()
        cells = [x.strip() for x in line.strip().strip("|").split("|")]
        if cells and cells[0] == "counter":
            cols = [c.replace("ash::", "") for c in cells[1:]]
        elif cols and len(cells) == len(cols) + 1 and cells[0].isupper() \
                and kernel in cols:
            try:
                vals[cells[0]] = float(cells[1 + cols.index(kernel)])
            except ValueError:
                pass
    if rec != kernel_source_sha256() or not vals:
        return None
    return vals


def issue_utilisation(counters, evals_per_launch, ms_avg, cycles=None):
    """Instructions per evaluation from the counters, and the fraction of
    the SIMDs' issue cycles (1024 SIMDs at 2.4 GHz over the measured launch
    time) that they take at the measured issue costs."""
    if not counters:
        return None
    c = cycles or ISSUE
    valu = counters.get("SQ_INSTS_VALU", 0.0)
    trans = counters.get("SQ_INSTS_VALU_TRANS_F32", 0.0)
    mfma = counters.get("SQ_INSTS_MFMA", 0.0)
    need = trans * c["trans"] + (valu - trans) * c["fma"] + mfma * c["mfma"]
    avail = SIMDS * CLOCK_HZ * ms_avg * 1e-3
    return {"valu_per_eval": valu / evals_per_launch,
            "trans_per_eval": trans / evals_per_launch,
            "mfma_per_eval": mfma / evals_per_launch,
            "minimum_valu_per_eval": 64.0 / 1024,
            "issue_utilisation": need / avail,
            "trans_issue_share": trans * c["trans"] / avail,
            "mfma_issue_share": mfma * c["mfma"] / avail,
            "source": "rocprofv3 counters of the committed summary, costs "
                      "measured at start-up"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


CPU_MIN_S, CPU_MAX_S, CPU_MAX_PAIRS = 10.0, 30.0, 8
# evaluations per sample pair: forward of sampled spots over every pixel,
# adjoint of every spot at sampled pixels
SAMPLE_FWD_EVALS, SAMPLE_ADJ_EVALS = 6e8, 1.5e8


def cpu_baseline(ctx, d, w=None, basis=None, full_ctx=None):
    """The FP64 oracle on a bounded sample of the same workload.

    Sample pairs: the forward transform of the workload's seeded start phase
    for a random subset of spots (all of them when spots x pixels is at
    most 6e8) over every pixel, and the adjoint of a farfield shaped like
    the loop's projection (target amplitudes, random phases) over every
    spot at a random subset of pixels (at most 1.5e8 evaluations); pairs
    repeat until CPU_MIN_S seconds have passed (at most CPU_MAX_PAIRS).
    Every output of a transform depends on one spot or one pixel, so the
    sampled outputs are exact references: the GPU's transforms of the same
    inputs are compared with the first pair (with `full_ctx`, also those of
    a context in full precision)."""
    import numpy as np
    import torch
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from tolerance import field_errors
    geom = oracle.Geometry(d["nx"], d["ny"])
    if basis is None:
        basis = oracle.ZernikeBasis(d["modes"])
    if w is None:
        w = d["w"]
    cores = len(os.sched_getaffinity(0))
    amp32 = d["amp"].astype(np.float32).astype(np.float64)
    phi32 = d["phi0"].astype(np.float32)
    f = amp32 * np.exp(1j * phi32.astype(np.float64))
    N, P = w.shape[0], geom.P
    S = min(N, max(1, int(SAMPLE_FWD_EVALS // P)))
    Q = min(P, max(1, int(SAMPLE_ADJ_EVALS // N)))
    rng = np.random.default_rng(2505)
    evals, pairs, first = 0, 0, None
    t0 = time.perf_counter()
    while pairs < CPU_MAX_PAIRS:
        sel = np.sort(rng.choice(N, S, replace=False)) if S < N else np.arange(N)
        pix = np.sort(rng.choice(P, Q, replace=False)) if Q < P else np.arange(P)
        y = (d["t"] * np.exp(1j * rng.uniform(-np.pi, np.pi, N))).astype(np.complex64)
        Eref = oracle.forward(f, w, basis, geom, spots=sel, workers=cores)
        gref = oracle.adjoint(y.astype(np.complex128), w, basis, geom,
                              pixels=pix, workers=cores)
        evals += S * P + N * Q
        pairs += 1
        if first is None:
            first = (sel, pix, y, Eref, gref)
        if time.perf_counter() - t0 >= CPU_MIN_S:
            break
    T = time.perf_counter() - t0
    sel, pix, y, Eref, gref = first
    dev = torch.device("cuda:0")

    def errors(c):
        E = c.forward(phase=torch.tensor(phi32, device=dev)).cpu().numpy()[sel]
        g = c.adjoint(torch.tensor(y, device=dev)).cpu().numpy().reshape(-1)[pix]
        fe, ge = field_errors(E, Eref), field_errors(g, gref)
        return {"forward_max_rel": fe[0], "forward_norm_rel": fe[1],
                "adjoint_max_rel": ge[0], "adjoint_norm_rel": ge[1],
                "pieces": c.info()["pieces"]}

    obj = {"value": evals / T, "unit": "evals/s", "cores": cores,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": "%d sample pair(s), each the forward of %d of %d spots "
                     "over all %d pixels and the adjoint of all spots at %d "
                     "pixels: %.3g evals in %.1f s, FP64 numpy on %d threads"
                     % (pairs, S, N, P, Q, evals, T, cores)}
    parity = errors(ctx)
    parity.update({"spots_sampled": S, "pixels_sampled": Q, "bar": 1e-4,
                   "precision": "auto"})
    if full_ctx is not None:
        parity["full_precision"] = errors(full_ctx)
    return obj, parity


def graph_replay(ctx, d, n_iter, steps):
    """The WGS step captured in a HIP graph (through torch's capture on the
    library's stream) and replayed `steps` times: the loop without host
    launch costs.  No compute call of the library allocates, synchronises
    or records a memset, so the step can be captured as it is."""
    import torch
    dev = torch.device("cuda:0")
    N = d["w"].shape[0]
    ph = torch.tensor(d["phi0"], dtype=torch.float32, device=dev)
    W = torch.ones(N, dtype=torch.float32, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ctx.wgs(ph, n_iter, weights=W, want_E=False, want_stats=False)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ctx.wgs(ph, n_iter, weights=W, want_E=False, want_stats=False)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    return {"wgs_iters_per_s": n_iter * steps / T,
            "ms_per_step": 1e3 * T / steps,
            "evals_per_s": 2.0 * N * d["nx"] * d["ny"] * n_iter * steps / T}


def bench_coef(args, d):
    """Gradient in the kernel coefficients on the 1024 x 1024, 1000-spot
    inputs: a step is `iters` calls of ash_coef_grad (moment transform and
    the gradient finish) for a fixed field gradient G."""
    import numpy as np
    import torch
    import paper_2505_08777_amd as A

    n_calls = args.iters or 20
    nx, ny = d["nx"], d["ny"]
    N, D = d["w"].shape
    P = nx * ny
    dev = torch.device("cuda:0")
    ctx = A.Context(0)
    ctx.set_basis(nx, ny, modes=d["modes"],
                  amp=torch.tensor(d["amp"], dtype=torch.float32, device=dev))
    ctx.set_spots(d["w"], d["t"])
    info = ctx.info()
    phase = torch.tensor(d["phi0"], dtype=torch.float32, device=dev)
    rng = np.random.default_rng(1024)
    G = torch.tensor((rng.normal(size=N) + 1j * rng.normal(size=N))
                     .astype(np.complex64), device=dev)
    grad = torch.empty((N, D), dtype=torch.float32, device=dev)

    def run():
        for _ in range(n_calls):
            ctx.coef_grad(phase, G, out=grad)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    ctx.profile(True, categories=("forward",))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    T = t1 - t0
    value = N * P * n_calls * args.steps / T
    ms_avg = prof["forward"][0] / max(prof["forward"][1], 1)
    groups = info["groups"]
    kname = "k_moments<%d, %d, %s>" % (groups, 2 if 2 * D > 32 else 1,
                                        "true" if info["range_reduce"] else "false")
    F = 6 * D + 3       # phase 2D, reduction 1, sin + cos, 4D moment flops
    traffic, traffic_src = profiled_traffic("coefgrad1024", kname,
                                            "coef_grad_kernels")
    out = {
        "metric": "spot·pixel moment evals/s (gradient in the kernel "
                  "coefficients)", "value": value, "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype_label(info),
        "data": "synthetic",
        "config": {"workload": "coefgrad1024", "slm": "%dx%d" % (nx, ny),
                   "spots": N, "modes": D, "calls_per_step": n_calls},
        "coef_grads_per_s": n_calls * args.steps / T,
        "roofline": alu_roofline(kname, N * P, ms_avg, prof["forward"][1], D,
                                 groups, traffic, traffic_src,
                                 reduce=bool(info["range_reduce"]),
                                 moments=True, flops=F),
        "kernels": {k: {"total_ms": v[0], "launches": v[1],
                        "avg_ms": v[0] / v[1] if v[1] else None}
                    for k, v in prof.items()},
        "layout": info,
    }
    if not args.no_cpu_baseline:
        import oracle
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from tolerance import field_errors
        geom = oracle.Geometry(nx, ny)
        basis = oracle.ZernikeBasis(d["modes"])
        cores = len(os.sched_getaffinity(0))
        sel = np.sort(rng.choice(N, size=8, replace=False))
        amp = d["amp"].astype(np.float32).astype(np.float64)
        phi = d["phi0"].astype(np.float32).astype(np.float64)
        Gh = G.cpu().numpy().astype(np.complex128)
        t2 = time.perf_counter()
        gref = oracle.coef_grad(amp * np.exp(1j * phi), d["w"], basis, geom,
                                Gh[sel], spots=sel, workers=cores)
        t3 = time.perf_counter()
        ctx.coef_grad(phase, G, out=grad)
        ge = field_errors(grad.cpu().numpy()[sel], gref)
        out["cpu_baseline"] = {
            "value": len(sel) * P / (t3 - t2), "unit": "evals/s",
            "cores": cores, "kind": "oracle",
            "sample": "coefficient gradient of %d spots over all %d pixels "
                      "and %d modes (%.2f s), FP64 numpy on %d threads"
                      % (len(sel), P, D, t3 - t2, cores)}
        out["parity"] = {"coef_grad_max_rel": ge[0],
                         "coef_grad_norm_rel": ge[1], "bar": 1e-4}
        out["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_feedback(args, d):
    """Closed-loop weighted GS with experimental feedback on a simulated
    system (1024 x 1024, 400 spots): each loop iteration measures the spot
    amplitudes of the current hologram on the 'true' system (a forward
    transform with perturbed aberrations, times per-spot gains) and runs one
    ash_wgs_feedback iteration on the model; the farfield phases are fixed
    after the first iterations.  A step is the workload's loop iterations."""
    import numpy as np
    import torch
    import paper_2505_08777_amd as A

    n_iter = args.iters or d["n_iter"]
    fix = d["fix_phase_after"]
    nx, ny = d["nx"], d["ny"]
    N, D = d["w"].shape
    P = nx * ny
    dev = torch.device("cuda:0")
    amp = torch.tensor(d["amp"], dtype=torch.float32, device=dev)
    model = A.Context(0)
    model.set_basis(nx, ny, modes=d["modes"], amp=amp)
    model.set_spots(d["w"], d["t"])
    system = A.Context(0)
    system.set_basis(nx, ny, modes=d["modes"], amp=amp)
    system.set_spots(d["w_true"], d["t"])
    gain = torch.tensor(d["gain"], dtype=torch.float32, device=dev)
    t = torch.tensor(d["t"], dtype=torch.float32, device=dev)

    def uniformity(E):
        I = (gain * torch.abs(E)) ** 2 / t ** 2
        return float(1.0 - (I.max() - I.min()) / (I.max() + I.min()))

    def loop(phase, W):
        for it in range(n_iter):
            meas = gain * torch.abs(system.forward(phase=phase))
            mode = 0 if it < fix - 1 else (1 if it == fix - 1 else -1)
            model.wgs_feedback(phase, meas, weights=W, fix_phase_after=mode,
                               want_E=False, want_stats=False)

    phase = torch.tensor(d["phi0"], dtype=torch.float32, device=dev)
    W = torch.ones(N, dtype=torch.float32, device=dev)
    for _ in range(args.warmup):
        loop(phase.clone(), W.clone())
    torch.cuda.synchronize()
    model.profile(True, categories=("forward", "adjoint"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ph = torch.tensor(d["phi0"], dtype=torch.float32, device=dev)
        Ws = torch.ones(N, dtype=torch.float32, device=dev)
        loop(ph, Ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = model.profile_read()
    model.profile(False)
    T = t1 - t0
    value = 3.0 * N * P * n_iter * args.steps / T
    u_fb = uniformity(system.forward(phase=ph))
    # the same number of model-only WGS iterations, for comparison
    ph2 = torch.tensor(d["phi0"], dtype=torch.float32, device=dev)
    model.wgs(ph2, n_iter, want_E=False, want_stats=False)
    u_model = uniformity(system.forward(phase=ph2))
    info = model.info()
    dom = max(("forward", "adjoint"), key=lambda k: prof[k][0])
    ms_avg = prof[dom][0] / max(prof[dom][1], 1)
    kname = "k_%s<%d, %s>" % (dom, info["groups"],
                              "true" if info["range_reduce"] else "false")
    out = {
        "metric": "spot·pixel kernel evals/s of the closed loop (measurement "
                  "forward + WGS forward + adjoint)",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype_label(info), "data": "synthetic",
        "config": {"workload": "feedback1024", "slm": "%dx%d" % (nx, ny),
                   "spots": N, "modes": D, "loop_iters_per_step": n_iter,
                   "fix_phase_after": fix},
        "loop_iters_per_s": n_iter * args.steps / T,
        "system_uniformity": {"feedback_loop": u_fb,
                              "model_only_wgs": u_model},
        "roofline": alu_roofline(kname, N * P, ms_avg, prof[dom][1], D,
                                 info["groups"],
                                 reduce=bool(info["range_reduce"])),
        "kernels": {k: {"total_ms": v[0], "launches": v[1],
                        "avg_ms": v[0] / v[1] if v[1] else None}
                    for k, v in prof.items()},
        "layout": info,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["parity"] = cpu_baseline(model, d)
    model.close()
    system.close()
    print(json.dumps(out), flush=True)


def bench_quality(args, d):
    """In-silico spot quality on the 1024 x 1024, 400-spot field: WGS
    holograms for three corrections of the workload's aberrations
    (uncorrected: tilts only; isoplanatic: every spot gets the aberration of
    the spot nearest the centre; anisoplanatic: each its own) are seen
    through the true system, and S' = max I / sum I is taken over 21 x 21
    farfield windows sampled every 0.25 bins around every spot.  A step is
    one quality evaluation of the anisoplanatic hologram (window spots set
    on the camera context, forward over 400 x 441 kernels, per-window
    S')."""
    import numpy as np
    import torch
    import paper_2505_08777_amd as A

    win, step_bins = 21, 0.25
    nx, ny = d["nx"], d["ny"]
    truth = d["w"]
    N, D = truth.shape
    P = nx * ny
    dev = torch.device("cuda:0")
    amp = torch.tensor(d["amp"], dtype=torch.float32, device=dev)
    centre = int(np.argmin(d["u"] ** 2 + d["v"] ** 2))
    corr = {"uncorrected": truth.copy(), "isoplanatic": truth.copy(),
            "anisoplanatic": truth}
    corr["uncorrected"][:, 2:] = 0.0
    corr["isoplanatic"][:, 2:] = truth[centre, 2:]
    model = A.Context(0)
    model.set_basis(nx, ny, modes=d["modes"], amp=amp)
    holo = {}
    for name, w in corr.items():
        model.set_spots(w, d["t"])
        ph = torch.tensor(d["phi0"], dtype=torch.float32, device=dev)
        model.wgs(ph, d["n_iter"], want_E=False, want_stats=False)
        holo[name] = ph
    model.close()
    cam = A.Context(0)
    cam.set_basis(nx, ny, modes=d["modes"], amp=amp)

    def quality(ph):
        return A.spot_quality(cam, ph, truth, ix=1, iy=0, win=win,
                              step=step_bins)

    for _ in range(args.warmup):
        quality(holo["anisoplanatic"])
    torch.cuda.synchronize()
    cam.profile(True, categories=("forward",))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S = quality(holo["anisoplanatic"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = cam.profile_read()
    cam.profile(False)
    T = t1 - t0
    S_all = {name: quality(ph).cpu().numpy() for name, ph in holo.items()}
    top = max(float(v.max()) for v in S_all.values())
    info = cam.info()
    n_k = N * win * win
    ms_avg = prof["forward"][0] / max(prof["forward"][1], 1)
    kname = "k_forward<%d, %s>" % (info["groups"],
                                   "true" if info["range_reduce"] else "false")
    out = {
        "metric": "spot·pixel kernel evals/s of the windowed quality "
                  "evaluation (set-up, forward, S')",
        "value": n_k * P * args.steps / T, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype_label(info),
        "data": "synthetic",
        "config": {"workload": "quality1024", "slm": "%dx%d" % (nx, ny),
                   "spots": N, "modes": D, "window": win,
                   "window_step_bins": step_bins, "wgs_iters": d["n_iter"]},
        "relative_strehl_mean": {name: float(v.mean()) / top
                                 for name, v in S_all.items()},
        "relative_strehl_min": {name: float(v.min()) / top
                                for name, v in S_all.items()},
        "roofline": alu_roofline(kname, n_k * P, ms_avg, prof["forward"][1],
                                 D, info["groups"],
                                 reduce=bool(info["range_reduce"])),
        "kernels": {k: {"total_ms": v[0], "launches": v[1],
                        "avg_ms": v[0] / v[1] if v[1] else None}
                    for k, v in prof.items()},
        "layout": info,
    }
    if not args.no_cpu_baseline:
        # S' of two spots' windows of the anisoplanatic hologram, by the
        # oracle (441 kernels over every pixel each); the GPU's are in S
        import oracle
        geom = oracle.Geometry(nx, ny)
        basis = oracle.ZernikeBasis(d["modes"])
        f = (d["amp"].astype(np.float32).astype(np.float64)
             * np.exp(1j * holo["anisoplanatic"].cpu().numpy().astype(np.float64)))
        sel = [centre, int(np.argmax(d["u"] ** 2 + d["v"] ** 2))]
        t0 = time.perf_counter()
        Sref = oracle.spot_quality(f, truth, basis, geom, ix=1, iy=0, win=win,
                                   step=step_bins, spots=sel,
                                   workers=len(os.sched_getaffinity(0)))
        Tc = time.perf_counter() - t0
        Sg = S_all["anisoplanatic"][sel]
        out["cpu_baseline"] = {
            "value": len(sel) * win * win * P / Tc, "unit": "evals/s",
            "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
            "sample": "the windows of %d spots (%d kernels over all %d "
                      "pixels) in %.1f s, FP64 numpy"
                      % (len(sel), len(sel) * win * win, P, Tc)}
        out["parity"] = {"spots": sel,
                         "strehl_max_rel": float(np.max(np.abs(Sg - Sref) / Sref)),
                         "bar": 1e-4}
    cam.close()
    print(json.dumps(out), flush=True)


def autograd_descent(A, ctx, d, n_steps):
    """The same descent through torch autograd: the spot fields from
    `propagate` (its backward is the adjoint kernel with the gradient
    epilogue), the loss and its TV term in torch ops, torch.optim.Adam.
    Returns the rate and the loss at every step (before its update)."""
    import numpy as np
    import torch
    amp = np.asarray(d["amp"], np.float64)
    N = d["w"].shape[0]
    s = float(np.sqrt(amp.size * np.sum(amp ** 2) / N))
    t = torch.tensor(d["t"], dtype=torch.float32, device="cuda:0")
    two_pi = 2.0 * np.pi

    def wrap(x):
        return x - two_pi * torch.round(x / two_pi)

    def loss_of(ph):
        E = A.propagate(ph, ctx)
        spot = torch.sum((torch.abs(E / s) ** 2 - t) ** 2)
        dx = torch.nn.functional.pad(wrap(ph[:, 1:] - ph[:, :-1]), (0, 1))
        dy = torch.nn.functional.pad(wrap(ph[1:, :] - ph[:-1, :]), (0, 0, 0, 1))
        tv = torch.mean(torch.sqrt(dx * dx + dy * dy + d["tv_eps"] ** 2))
        return spot + d["lam"] * tv

    def run(k):
        ph = torch.tensor(d["phi0"], dtype=torch.float32, device="cuda:0",
                          requires_grad=True)
        opt = torch.optim.Adam([ph], lr=d["lr"], betas=d["betas"],
                               eps=d["adam_eps"])
        losses = []
        for _ in range(k):
            opt.zero_grad(set_to_none=False)
            L = loss_of(ph)
            L.backward()
            opt.step()
            losses.append(L.detach())
        return torch.stack(losses)

    run(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = run(n_steps)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    return n_steps / T, losses.cpu().numpy()


def bench_adam(args, d):
    """Adam descent of the 1024 x 1024, 1000-spot loss: a step is the
    workload's Adam updates (forward, loss, adjoint with the phase gradient
    and TV, update), timed like the WGS loop."""
    import numpy as np
    import torch
    import paper_2505_08777_amd as A

    n_steps = args.iters or d["n_iter"]
    nx, ny = d["nx"], d["ny"]
    N, D = d["w"].shape
    P = nx * ny
    dev = torch.device("cuda:0")
    ctx = A.Context(0)
    ctx.set_basis(nx, ny, modes=d["modes"],
                  amp=torch.tensor(d["amp"], dtype=torch.float32, device=dev))
    ctx.set_spots(d["w"], d["t"])
    info = ctx.info()
    phi0 = torch.tensor(d["phi0"], dtype=torch.float32, device=dev)
    kw = dict(lr=d["lr"], betas=d["betas"], eps=d["adam_eps"],
              tv_weight=d["lam"], tv_eps=d["tv_eps"])

    def run():
        ph = phi0.clone()
        return ctx.adam(ph, n_steps, **kw)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    ctx.profile(True, categories=("forward", "adjoint"),
                stride=args.event_stride)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, _, loss, _ = run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    T = t1 - t0
    F = flops_per_eval(D)
    value = 2.0 * N * P * n_steps * args.steps / T
    dom = max(("forward", "adjoint"), key=lambda k: prof[k][0])
    ms_avg = prof[dom][0] / max(prof[dom][1], 1)
    kname = "k_%s<%d, %s>" % (dom, info["groups"],
                              "true" if info["range_reduce"] else "false")
    traffic, traffic_src = profiled_traffic(args.workload, kname)
    L = loss.cpu().numpy()
    out = {
        "metric": METRIC, "value": value, "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype_label(info),
        "data": "synthetic",
        "config": {"workload": "grad1024", "slm": "%dx%d" % (nx, ny),
                   "spots": N, "modes": D, "adam_steps_per_step": n_steps},
        "adam_steps_per_s": n_steps * args.steps / T,
        "algorithmic_flops_pct_of_fp32_vector_peak":
            100.0 * value * F / (FP32_VECTOR_PEAK_TFLOPS * 1e12),
        "baseline_slot_model": slot_model(value, D),
        "roofline": alu_roofline(kname, N * P, ms_avg, prof[dom][1], D,
                                 info["groups"], traffic, traffic_src,
                                 reduce=bool(info["range_reduce"])),
        "kernels": {k: {"total_ms": v[0], "launches": v[1],
                        "avg_ms": v[0] / v[1] if v[1] else None}
                    for k, v in prof.items()},
        "issue_model": issue_model(N * P / (ms_avg * 1e-3), info["groups"]),
        "loss_first_last": [float(L[0]), float(L[-1])],
        "event_stride": args.event_stride,
        "layout": info,
    }
    # the same descent through torch autograd, and the plain WGS loop, on
    # this context
    rate, La = autograd_descent(A, ctx, d, n_steps)
    out["autograd"] = {
        "adam_steps_per_s": rate,
        "loss_first_last": [float(La[0]), float(La[-1])],
        "max_rel_loss_diff_vs_fused": float(np.max(np.abs(La - L) / L)),
        "fused_speedup": out["adam_steps_per_s"] / rate}
    ph = phi0.clone()
    W = torch.ones(N, dtype=torch.float32, device=dev)
    ctx.wgs(ph, 10, weights=W, want_E=False, want_stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.wgs(ph, n_steps, weights=W, want_E=False, want_stats=False)
    torch.cuda.synchronize()
    out["plain_wgs_iters_per_s"] = n_steps / (time.perf_counter() - t0)
    # the gradient alone (ash_phase_grad: the adjoint with the gradient
    # epilogue), as the autograd backward calls it
    G = torch.ones(N, dtype=torch.complex64, device=dev)
    gout = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    ctx.phase_grad(phi0, G, out=gout)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        ctx.phase_grad(phi0, G, out=gout)
    torch.cuda.synchronize()
    Tg = (time.perf_counter() - t0) / 20
    out["phase_grad"] = {"per_s": 1.0 / Tg, "ms": 1e3 * Tg,
                         "evals_per_s": N * P / Tg}
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["parity"] = cpu_baseline(ctx, d)
        out["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_batch(args, holos):
    """64 holograms (batch64: sides 512..2048, N log-uniform in [10, 5000];
    batch64small: sides 256..512, N in [5, 200]; 12 modes): a step is the
    workload's WGS iterations (50, 20) of every hologram in the batched
    persistent launches, continuing from the last phases; the same loops
    run one context at a time are timed beside it."""
    import numpy as np
    import torch
    import paper_2505_08777_amd as A

    n_iter = args.iters or holos[0]["n_iter"]
    dev = torch.device("cuda:0")
    ctxs = []
    for d in holos:
        c = A.Context(0)
        c.set_basis(d["nx"], d["ny"], modes=d["modes"],
                    amp=torch.tensor(d["amp"], dtype=torch.float32, device=dev))
        c.set_spots(d["w"], d["t"])
        ctxs.append(c)
    b = A.Batch(ctxs)
    phases = [torch.tensor(d["phi0"], dtype=torch.float32, device=dev)
              for d in holos]
    weights = [torch.ones(d["w"].shape[0], dtype=torch.float32, device=dev)
               for d in holos]
    tune_s, forms = None, None
    if not args.no_tune:
        import tempfile
        t0 = time.perf_counter()
        with tempfile.TemporaryDirectory() as tmp:
            table = os.path.join(tmp, "tune.txt")
            b.tune(phases, table_out=table)
            torch.cuda.synchronize()
            tune_s = time.perf_counter() - t0
            forms = {"table": [l.strip() for l in open(table)
                               if not l.startswith("#")]}
        for line in forms["table"]:
            f = line.split()
            if f[0] == "form":
                forms["chosen"] = "one_launch" if f[1] == "1" else "per_phase"
                forms["per_phase_ms_per_iteration"] = float(f[2])
            if f[0] == "one_launch":
                forms.setdefault("one_launch_ms_per_iteration", 0.0)
                forms["one_launch_ms_per_iteration"] += float(f[4])
    if args.form != "tuned":
        b.set_form(args.form == "one_launch")
    info = b.info()
    for _ in range(args.warmup):
        b.wgs(phases, n_iter, weights=weights)
    torch.cuda.synchronize()
    b.profile(True, categories=("forward", "adjoint"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.wgs(phases, n_iter, weights=weights)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = b.profile_read()
    b.profile(False)
    T = t1 - t0
    D = holos[0]["w"].shape[1]
    F = flops_per_eval(D)
    evals = info["evals_per_transform"]
    value = 2.0 * evals * n_iter * args.steps / T
    shapes = max(info["shapes"], 1)
    # the ceiling of the fewest matrix-core groups among the shapes (the
    # highest), so the fraction is a lower estimate when shapes differ
    groups = min(info["groups"]) if info["groups"] else 0
    if info["one_launch"]:
        # one launch per record shape runs every iteration of its
        # holograms (forward, update, adjoint): the unit timed is a call
        kname = "k_batch_persist<%d, false>" % groups
        calls = max(prof["forward"][1] // shapes, 1)
        ms_avg = prof["forward"][0] / calls
        evals_launch = 2.0 * evals * n_iter
        launches = calls
    elif info["fused"]:
        # every transform in fused launches, timed under the adjoint
        # category: per call and record shape n_iter + 1 launches holding
        # 2 n_iter transforms of its holograms (the first only a forward,
        # the last only an adjoint); the unit timed is a launch of all
        # shapes, with the work of the average launch
        kname = "k_batch_fused<%d, false, 1>" % groups
        launches = prof["adjoint"][1] // shapes
        ms_avg = prof["adjoint"][0] / max(launches, 1)
        evals_launch = 2.0 * evals * n_iter / (n_iter + 1)
    else:
        # a phase is one launch per record shape, each over all holograms
        # of that shape: the unit timed is the phase (all its launches)
        dom = max(("forward", "adjoint"), key=lambda k: prof[k][0])
        kname = "k_batch_%s<%d, false>" % (dom, groups)
        launches = prof[dom][1] // shapes
        ms_avg = prof[dom][0] / max(launches, 1)
        evals_launch = evals
    # the unit timed spans one launch of every record shape: its traffic is
    # the sum of the shapes' kernels' traffic per launch (fused: the first,
    # middle and last launches weighted 1 : n_iter - 1 : 1; one launch: the
    # whole call, from the one-launch form's own summary)
    parts = []
    for g in (info["groups"] or [groups]):
        name = re.sub(r"<\d+,", "<%d," % g, kname, count=1)
        if info["one_launch"]:
            parts.append(profiled_traffic(args.workload, name,
                                          summary="one_launch_kernels"))
        elif info["fused"]:
            modes = [profiled_traffic(args.workload, name[:-2] + "%d>" % m,
                                      summary="batch_kernels") for m in (0, 1, 2)]
            t = (None if any(x is None for x, _ in modes) else
                 (modes[0][0] + (n_iter - 1) * modes[1][0] + modes[2][0])
                 / (n_iter + 1))
            parts.append((t, modes[1][1]))
        else:
            parts.append(profiled_traffic(args.workload, name,
                                          summary="batch_kernels"))
    traffic = (sum(t for t, _ in parts)
               if parts and all(t is not None for t, _ in parts) else None)
    traffic_src = parts[0][1] if parts else None
    out = {
        "metric": METRIC, "value": value, "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype_label({"pieces": "-".join(
            str(p) for p in sorted({c.info()["pieces"] for c in ctxs}))}),
        "data": "synthetic",
        "config": {"workload": args.workload, "holograms": len(holos),
                   "sum_N_P": evals, "modes": D,
                   "wgs_iters_per_step": n_iter},
        "wgs_iters_per_s_per_hologram": n_iter * args.steps / T,
        "algorithmic_flops_pct_of_fp32_vector_peak":
            100.0 * value * F / (FP32_VECTOR_PEAK_TFLOPS * 1e12),
        "roofline": alu_roofline(kname, evals_launch, ms_avg, launches, D,
                                 groups, traffic, traffic_src),
        "kernels": {k: {"total_ms": v[0], "launches": v[1],
                        "avg_ms": v[0] / v[1] if v[1] else None}
                    for k, v in prof.items()},
        "issue_model": issue_model(evals_launch / (ms_avg * 1e-3), groups),
        "layout": info, "tune_s": tune_s, "forms": forms,
    }
    # the same holograms' loops run one context at a time (plain loop)
    ph2 = [p.clone() for p in phases]
    w2 = [w.clone() for w in weights]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, p, w in zip(ctxs, ph2, w2):
        c.wgs(p, n_iter, weights=w, want_E=False, want_stats=False)
    torch.cuda.synchronize()
    Tp = time.perf_counter() - t0
    out["plain_loop"] = {"ms_per_step": 1e3 * Tp,
                         "evals_per_s": 2.0 * evals * n_iter / Tp,
                         "batch_speedup": Tp / (T / args.steps)}
    b.close()
    if not args.no_cpu_baseline:
        # the oracle on the hologram with the fewest evaluations, its
        # context's transforms beside it (the batch runs the same kernels)
        h = int(np.argmin([x["w"].shape[0] * x["nx"] * x["ny"] for x in holos]))
        out["cpu_baseline"], out["parity"] = cpu_baseline(ctxs[h], holos[h])
        out["parity"]["hologram"] = {"index": h, "N": holos[h]["w"].shape[0],
                                     "side": holos[h]["nx"]}
    for c in ctxs:
        c.close()
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.calibrate_copy_mib:
        calibrate_copy(args.calibrate_copy_mib)
        return
    if args.ubench and args.gpus == 1:
        print(json.dumps({"issue_cycles": measure_issue_costs()}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU; there is no multi-GPU path "
              "(each GPU would run its own slab of pixel rows with the "
              "full spot table and one small all-reduce of E per iteration)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads
    import paper_2505_08777_amd as A

    measure_issue_costs()
    if args.workload == "coefgrad1024":
        return bench_coef(args, workloads.grad1024())
    if args.workload == "feedback1024":
        return bench_feedback(args, workloads.feedback1024())
    if args.workload == "quality1024":
        return bench_quality(args, workloads.field1024())
    d = workloads.make(args.workload)
    if args.workload == "grad1024":
        return bench_adam(args, d)
    if args.workload in ("batch64", "batch64small"):
        return bench_batch(args, d)
    n_iter = args.iters or d["n_iter"]
    nx, ny = d["nx"], d["ny"]
    N, D = d["w"].shape
    P = nx * ny
    dev = torch.device("cuda:0")
    amp_t = torch.tensor(d["amp"], dtype=torch.float32, device=dev)
    ctx = A.Context(0)
    principal = None
    if args.workload == "principal1024":
        # the WGS loop on the K leading principal modes; the full-basis loop
        # is timed beside it
        pw, cf = A.zernike_table(d["modes"])
        cfK, wK, sigma = A.principal_modes(pw, cf, d["w"], d["K"])
        ctx.set_basis(nx, ny, mono_pow=pw, mono_coef=cfK, amp=amp_t)
        ctx.set_spots(wK, d["t"])
        n_keep = wK.shape[1] - d["K"]
        rot = d["w"][:, n_keep:]
        # the Zernike modes are orthonormal over the pupil, so the norm of
        # the dropped coefficients is the rms phase change over the pupil
        drop = np.sqrt(np.maximum(0.0, np.sum(rot ** 2, axis=1)
                                  - np.sum(wK[:, n_keep:] ** 2, axis=1)))
        principal = {"K": d["K"], "modes_in": D, "modes_evaluated": wK.shape[1],
                     "sigma": [float(x) for x in sigma],
                     "rms_phase_change_rad": {"mean": float(drop.mean()),
                                              "max": float(drop.max())}}
        D = wK.shape[1]
    else:
        ctx.set_basis(nx, ny, modes=d["modes"], amp=amp_t)
        ctx.set_spots(d["w"], d["t"])
    # a spot update (new coefficient matrix, pixel tables untouched), as
    # between holograms of a dynamic display: host call to results ready
    set_spots_ms = None
    if principal is None:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            ctx.set_spots(d["w"], d["t"])
        torch.cuda.synchronize()
        set_spots_ms = 1e3 * (time.perf_counter() - t0) / 5
    info = ctx.info()
    phase = torch.tensor(d["phi0"], dtype=torch.float32, device=dev)
    weights = torch.ones(N, dtype=torch.float32, device=dev)

    for _ in range(args.warmup):
        ctx.wgs(phase, n_iter, weights=weights, want_E=False, want_stats=False)
    torch.cuda.synchronize()

    # timed region: K steps, one transform launch in every event_stride
    # bracketed by HIP events
    ctx.profile(True, categories=("forward", "adjoint"),
                stride=args.event_stride)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.wgs(phase, n_iter, weights=weights, want_E=False,
                want_stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)

    # the same loop without events, for the event overhead
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        ctx.wgs(phase, n_iter, weights=weights, want_E=False,
                want_stats=False)
    torch.cuda.synchronize()
    t3 = time.perf_counter()

    T = t1 - t0
    ms_step = 1e3 * T / args.steps
    evals_step = 2.0 * N * P * n_iter
    value = evals_step * args.steps / T
    F = flops_per_eval(D)
    # dominant kernel: the transform with the larger total time
    dom = max(("forward", "adjoint"), key=lambda k: prof[k][0])
    ms_avg = prof[dom][0] / max(prof[dom][1], 1)
    kname = "k_%s<%d, %s>" % (dom, info["groups"],
                              "true" if info["range_reduce"] else "false")
    traffic, traffic_src = profiled_traffic(args.workload, kname)
    roofline = alu_roofline(kname, N * P, ms_avg, prof[dom][1], D,
                            info["groups"], traffic, traffic_src,
                            reduce=bool(info["range_reduce"]))
    counters = issue_utilisation(profiled_counters(args.workload, kname),
                                 N * P, ms_avg)
    kernels = {k: {"total_ms": v[0], "launches": v[1],
                   "avg_ms": v[0] / v[1] if v[1] else None}
               for k, v in prof.items()}

    out = {
        "metric": METRIC, "value": value, "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype_label(info),
        "data": "synthetic",
        "config": {"workload": args.workload, "slm": "%dx%d" % (nx, ny),
                   "spots": N, "modes": D, "wgs_iters_per_step": n_iter},
        "wgs_iters_per_s": n_iter * args.steps / T,
        "algorithmic_flops_pct_of_fp32_vector_peak":
            100.0 * value * F / (FP32_VECTOR_PEAK_TFLOPS * 1e12),
        "baseline_slot_model": slot_model(value, D),
        "ms_per_step_without_events": 1e3 * (t3 - t2) / args.steps,
        "event_stride": args.event_stride,
        "roofline": roofline,
        "issue_model": issue_model(N * P / (ms_avg * 1e-3), info["groups"]),
        "counters": counters,
        "kernels": kernels, "layout": info, "set_spots_ms": set_spots_ms,
    }
    if args.graph or args.workload == "plain256":
        out["graph_replay"] = graph_replay(ctx, d, n_iter, args.steps)
    if principal is not None:
        out["config"].update(modes=principal["modes_in"],
                             principal_modes=principal["K"],
                             modes_evaluated=principal["modes_evaluated"])
        full = A.Context(0)
        full.set_basis(nx, ny, modes=d["modes"], amp=amp_t)
        full.set_spots(d["w"], d["t"])
        ph_f = torch.tensor(d["phi0"], dtype=torch.float32, device=dev)
        w_f = torch.ones(N, dtype=torch.float32, device=dev)
        full.wgs(ph_f, 2, weights=w_f, want_E=False, want_stats=False)
        torch.cuda.synchronize()
        n_ref = min(n_iter, 20)
        t4 = time.perf_counter()
        full.wgs(ph_f, n_ref, weights=w_f, want_E=False, want_stats=False)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        ms_full = 1e3 * (t5 - t4) / n_ref
        ms_princ = 1e3 * (t3 - t2) / args.steps / n_iter
        principal["full_basis"] = {"groups": full.info()["groups"],
                                   "ms_per_iter": ms_full,
                                   "evals_per_s": 2.0 * N * P / (ms_full * 1e-3)}
        principal["ms_per_iter"] = ms_princ
        principal["loop_speedup"] = ms_full / ms_princ
        full.close()
        out["principal"] = principal

    if not args.no_cpu_baseline:
        if principal is not None:
            import oracle
            wr, br, _ = oracle.principal_modes(
                d["w"], oracle.ZernikeBasis(d["modes"]), d["K"])
            out["cpu_baseline"], out["parity"] = cpu_baseline(
                ctx, d, w=wr, basis=br)
        else:
            # the same transforms in full precision (3 pieces for every
            # remainder term) beside the default
            full = A.Context(0)
            full.set_precision(True)
            full.set_basis(nx, ny, modes=d["modes"], amp=amp_t)
            full.set_spots(d["w"], d["t"])
            out["cpu_baseline"], out["parity"] = cpu_baseline(
                ctx, d, full_ctx=full)
            full.close()
        out["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
