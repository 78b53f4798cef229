"""Benchmark: element-field-point interactions per second (potential + field), FP64 and
mixed precision, on one MI355X; collocation product and serving latency beside it.

One step = one evaluation of the whole hot path over the cylinder workload
(100,000 cap triangles with the 33-point rule + 50,000 mantle rectangles with 7 x 7 Gauss,
1,000,000 field points of which 30 % lie at distance ratio < 3 of some element):
distance-ratio classification and near-pair compaction, far-field point-charge sums,
FP64 near-field subdivision.  Inputs are resident in HBM before the timed region.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--serving-queries Q] [--quick]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # 256 CU x 2.4 GHz x 64 FP64 FMA lanes x 2
PEAK_FP32_TFLOPS = 157.3  # 256 CU x 2.4 GHz x 128 FP32 FMA lanes x 2 (packed)
PEAK_HBM_GBPS = 8000.0    # HBM3E
FLOP_PER_NODE_INT = 20    # Phi + E per point-charge term
FLOP_PER_PAIR = 16        # distance-ratio test + charge scaling per element-point pair
GRAD_FLOP_PER_NODE_INT = 30  # field gradient (six components) per point-charge term
COLLOC_FLOP_PER_NODE_INT = 11  # potential only (collocation product) per point-charge term
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "hbm_counters_cylinder150k_nested200k.txt")
VALU_FILE = os.path.join(PROFILES, "valu_counters_cylinder150k_nested200k.txt")
TRACE_FILE = os.path.join(PROFILES, "kernel_trace_cylinder150k_nested200k.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1606_03743_amd", "csrc", "kernels.hip")
PROBE_LIB = os.path.join(ROOT, "paper_1606_03743_amd", "libissue_probe.so")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def profile_value(path, key):
    """A figure of a committed rocprofv3 summary, or None when the file is missing or the
    kernel source changed since the profile was taken."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*(\w+)", txt)
    b = re.search(r"^" + re.escape(key) + r":\s*([0-9.eE+-]+)", txt, re.M)
    if not m or not b or m.group(1) != kernel_hash():
        return None
    return float(b.group(1))


def traffic_from_profile(kernel="far_fp64"):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, calibrated by a 1 GiB copy)."""
    return profile_value(TRAFFIC_FILE, f"{kernel}_hbm_bytes_per_launch")


def counted_flops_from_profile(kernel="far_fp64"):
    """Hardware flops per launch: 64 x (2 FMA + MUL + ADD + TRANS) of the kernel's FP64
    instructions (FP32 for the mixed kernels)."""
    sfx = "f32" if kernel.endswith("mixed") else "f64"
    return profile_value(VALU_FILE, f"{kernel}_counted_{sfx}_flops_per_launch")


def trace_avg_ms(prefix):
    """Average duration of a kernel in the committed kernel trace (None if stale)."""
    if not os.path.exists(TRACE_FILE):
        return None
    txt = open(TRACE_FILE).read()
    m = re.search(r"kernel_source_sha256_16:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_hash():
        return None
    for line in txt.splitlines():
        if line.startswith(prefix):
            return float(line[86:].split()[1])
    return None


def issue_rates():
    """Issue rates measured on cuda:0 (wavefront instructions per second; csrc/issue_probe.hip),
    or None without the probe library."""
    if not os.path.exists(PROBE_LIB):
        return None
    import ctypes

    import torch  # noqa: F401  (one HIP runtime per process: torch's)

    lib = ctypes.CDLL(PROBE_LIB)
    lib.issue_probe_rates.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    r = (ctypes.c_double * 6)()
    if lib.issue_probe_rates(0, r) != 0:
        return None
    keys = ("fma_f64", "rsq_f64", "f64_one_rsq_in_nine", "fma_f32", "rsq_f32", "f32_one_rsq_in_nine")
    return dict(zip(keys, [float(v) for v in r]))


def issue_ceiling(rates, kernel, node_ints, far_ms):
    """The node-interaction rate an FP64 kernel's instruction mix allows, from its committed VALU
    counts per node interaction: the full-rate FP64 instructions at the measured FMA rate, each
    reciprocal square root at its measured cost inside an FMA stream (9 / rate of the one-in-nine
    stream - 8 / FMA rate).  None without the rates or with stale counters."""
    f = profile_value(VALU_FILE, f"{kernel}_f64_lane_instructions_per_node_interaction")
    tr = profile_value(VALU_FILE, f"{kernel}_trans_per_node_interaction")
    if rates is None or f is None or tr is None:
        return None
    t_rsq = 9.0 / rates["f64_one_rsq_in_nine"] - 8.0 / rates["fma_f64"]
    per_wave_interaction = (f - tr) / rates["fma_f64"] + tr * t_rsq
    ceiling = 64.0 / per_wave_interaction
    achieved = node_ints / (1e-3 * far_ms)
    return {"node_interactions_per_s": ceiling, "achieved_node_interactions_per_s": achieved,
            "frac": achieved / ceiling, "fp64_instructions_per_node_interaction": f,
            "rsq_per_node_interaction": tr, "rates_wave_instructions_per_s": rates,
            "note": "the rate the kernel's instructions allow at the issue rates measured on this device "
                    "(probe kernels of independent chains): frac is the kernel's share of that ceiling"}


def profiled(kernel, flops, far_ms, peak):
    """Counted flops and HBM traffic of a kernel from the committed profiles, per launch,
    over this run's launch time."""
    c = counted_flops_from_profile(kernel)
    t = traffic_from_profile(kernel)
    s = 1e-3 * far_ms
    return {"counted_tflops": None if c is None else c / s / 1e12,
            "counted_frac": None if c is None else c / s / 1e12 / peak,
            "traffic": t, "hbm_gbps": None if t is None else t / s / 1e9}


def nerr(phi, E, ref):
    ep = np.abs(phi - ref["phi"]) / ref["abs_phi"]
    ee = np.sum(np.abs(E - ref["E"]), axis=1) / ref["abs_E"]
    rp = np.abs(phi - ref["phi"]) / np.abs(ref["phi"])
    return ep, ee, rp


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--serving-queries", type=int, default=120, help="fixed-rule serving leg (queries)")
    ap.add_argument("--serving-queries-dr", type=int, default=2000, help="distance-ratio serving leg (queries)")
    ap.add_argument("--side-steps", type=int, default=5, help="timed steps of the side legs (at most --steps)")
    ap.add_argument("--cpu-sample", type=int, default=2000, help="oracle sample size (points)")
    ap.add_argument("--quick", action="store_true", help="skip collocation, serving and the CPU baseline")
    ap.add_argument("--profile-only", action="store_true",
                    help="calibration copies and one evaluation of each profiled kernel (for counter runs)")
    ap.add_argument("--icosphere-only", action="store_true",
                    help="only the small-evaluation leg (1,280-triangle icosphere, 1,000 evaluations)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (requested --gpus {args.gpus}); every box in this setup "
              "has one GPU and the path has no multi-GPU leg.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1606_03743_amd import bemc, workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    if args.icosphere_only:
        r = icosphere_bench(torch, bemc, W, reps=1000)
        log(f"icosphere: {r['us_per_eval']:.1f} us per evaluation")
        return

    log("building the cylinder workload (150,000 elements, 1,000,000 points)")
    w = W.cylinder_150k()
    ctx = bemc.Context(0)
    ctx.set_rules(w.tri_rule, w.rect_gl_n, 3.0, 24)
    t_up = time.perf_counter()
    ctx.upload_geometry(w.tri, w.rect)  # validation, frames and copies (host arrays)
    t_geom = time.perf_counter() - t_up
    t_up = time.perf_counter()
    ctx.upload_densities(w.sigma)
    t_dens = time.perf_counter() - t_up
    pts = torch.tensor(np.ascontiguousarray(w.points.T), dtype=torch.float64, device=dev)
    n = pts.shape[1]
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    E = torch.empty((3, n), dtype=torch.float64, device=dev)
    ctx.set_near_capacity(40_000_000)  # fixed: evaluations never wait on the host
    torch.cuda.synchronize()

    if args.profile_only:
        # calibration kernels of known size for the HBM byte counters: a 1 GiB fill
        # (writes 1 GiB) and a 1 GiB copy (reads 1 GiB, writes 1 GiB)
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        for dr in (False, True):
            ctx.set_dr_rules(dr)
            for prec in ("fp64", "mixed"):
                ctx.eval(pts, prec, phi=phi, E=E)
                torch.cuda.synchronize()
                log(f"profile run: {prec} evaluation (rule choice by DR {dr}) done: {ctx.stats()}")
        ctx.set_dr_rules(False)
        ctx.close()
        wc = W.nested_cylinders_workload()
        cctx = bemc.Context(0)
        cctx.upload_geometry(wc.tri, wc.rect)
        sig = torch.tensor(wc.sigma, dtype=torch.float64, device=dev)
        for prec in ("fp64", "mixed"):
            cctx.collocation(sig, prec)
            torch.cuda.synchronize()
            log(f"profile run: {prec} collocation product (200,000 elements, 8 densities) done: {cctx.stats()}")
        cctx.close()
        return

    def timed(precision, steps, warmup):
        for i in range(warmup):
            ctx.eval(pts, precision, phi=phi, E=E)
            log(f"{precision} warmup {i + 1}/{warmup} done")
        torch.cuda.synchronize()
        far_ms = []
        t0 = time.perf_counter()
        for i in range(steps):
            ctx.eval(pts, precision, phi=phi, E=E)
            far_ms.append(ctx.stats()["far_ms"])
            log(f"{precision} step {i + 1}/{steps} done")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, far_ms, ctx.stats()

    dt64, far64, st64 = timed("fp64", args.steps, args.warmup)
    phi64, E64 = phi.cpu().numpy(), E.cpu().numpy().T.copy()
    side = max(1, min(args.steps, args.side_steps))
    dtmx, farmx, stmx = timed("mixed", side, 1)
    phimx, Emx = phi.cpu().numpy(), E.cpu().numpy().T.copy()
    # rule choice by distance ratio (fewest Gaussian points at the accuracy floor per pair)
    ctx.set_dr_rules(True)
    dtdr, fardr, stdr = timed("fp64", side, 1)
    phidr, Edr = phi.cpu().numpy(), E.cpu().numpy().T.copy()
    dtdrm, fardrm, stdrm = timed("mixed", side, 1)
    phidrm, Edrm = phi.cpu().numpy(), E.cpu().numpy().T.copy()
    ctx.set_dr_rules(False)
    # Table B5 for the rectangles (33 points, degree 13) instead of 7 x 7 Gauss (49 points)
    ctx.set_rules(w.tri_rule, -33)
    dtb5, farb5, stb5 = timed("fp64", side, 1)
    phib5, Eb5 = phi.cpu().numpy(), E.cpu().numpy().T.copy()
    dtb5m, farb5m, stb5m = timed("mixed", side, 1)
    phib5m, Eb5m = phi.cpu().numpy(), E.cpu().numpy().T.copy()
    ctx.set_rules(w.tri_rule, w.rect_gl_n)

    # field gradient dE_i/dx_j (six rows) on the same workload
    G = torch.empty((6, n), dtype=torch.float64, device=dev)
    grad = {}
    for prec in ("fp64", "mixed"):
        ctx.eval_gradient(pts, prec, G=G)
        torch.cuda.synchronize()
        log(f"gradient {prec} warmup done")
        t0 = time.perf_counter()
        ctx.eval_gradient(pts, prec, G=G)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ctx.stats()
        grad[prec] = {"value": st["pairs"] / dt, "unit": "pairs/s", "ms": 1e3 * dt, "far_kernel_ms": st["far_ms"],
                      "near_kernel_ms": st["near_ms"], "G": G.cpu().numpy().T.copy()}
        log(f"gradient {prec} step done")

    rates = issue_rates()
    log(f"issue rates (wavefront instructions/s): {rates}")
    pairs = st64["pairs"]
    node_int = st64["node_interactions"]
    ms_step = 1e3 * dt64 / args.steps
    value = pairs * args.steps / dt64
    alg_flops = FLOP_PER_NODE_INT * node_int + FLOP_PER_PAIR * pairs
    far_avg_s = 1e-3 * float(np.mean(far64))
    achieved = alg_flops / far_avg_s / 1e12
    traffic = traffic_from_profile("far_fp64")
    counted = counted_flops_from_profile("far_fp64")
    prof_ms = trace_avg_ms("far_eval_kernel<false, 33, 49, 0, 0, 0, 0, 0, 0, false, 3, false>")
    out = {
        "metric": "element-fieldpoint interactions/s (phi+E) FP64 vs mixed @1e-6; p99 query ms",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded cylinder mesh and points; the paper's KATRIN meshes are not available)",
        "config": {"workload": w.name, "elements": w.n_elements, "points": n, "near_frac": 0.3,
                   "tri_rule": w.tri_rule, "rect_gauss": f"{w.rect_gl_n}x{w.rect_gl_n}", "precision": "fp64"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": "far_eval_kernel<33,49,fp64>",
                     "flops_per_launch": alg_flops, "avg_launch_ms": 1e3 * far_avg_s,
                     "counted_fp64_tflops": None if counted is None else counted / far_avg_s / 1e12,
                     "counted_frac": None if counted is None else counted / far_avg_s / 1e12 / PEAK_FP64_TFLOPS,
                     "hbm_gbps": None if traffic is None else traffic / far_avg_s / 1e9,
                     "hbm_frac": None if traffic is None else traffic / far_avg_s / 1e9 / PEAK_HBM_GBPS,
                     "rocprof_avg_launch_ms": prof_ms,
                     "rocprof_frac": None if prof_ms is None else alg_flops / (1e-3 * prof_ms) / 1e12 / PEAK_FP64_TFLOPS,
                     "issue_ceiling": issue_ceiling(rates, "far_fp64", node_int, 1e3 * far_avg_s),
                     "note": "achieved: algorithmic flops (20 per node interaction + 16 per pair) over the far "
                             "kernel's mean HIP-event time in this run; rocprof_frac: the same over the committed "
                             "kernel trace's average (profiling box)"},
        "node_interactions_per_s": node_int * args.steps / dt64,
        "near": {"pairs": st64["near_pairs"], "leaves": st64["leaves"], "max_depth": st64["max_depth"],
                 "cap_hits": st64["cap_hits"], "stage_ms": st64["near_ms"],
                 "near_kernel_rocprof_ms": trace_avg_ms("near_kernel<0, true>"),
                 "near_list_kernel_rocprof_ms": trace_avg_ms("near_list_kernel"),
                 "near_kernel_write_bytes": profile_value(TRAFFIC_FILE, "near_field_write_bytes_per_launch"),
                 "near_kernel_read_bytes": profile_value(TRAFFIC_FILE, "near_field_read_bytes_per_launch"),
                 "result_bytes": 32 * st64["near_pairs"],
                 "note": "stage_ms: chunk reduction, near-list regrouping, near kernel and ordered sums (HIP "
                         "events); the near-pair list pass runs before the far kernel"},
        "upload": {"elements": w.n_elements, "geometry_s": t_geom, "densities_s": t_dens,
                   "note": "host arrays: validation, centroids, frames, charges, copies to the device"},
    }
    mixed_ach = alg_flops / (1e-3 * float(np.mean(farmx))) / 1e12
    counted32 = counted_flops_from_profile("far_mixed")
    c32 = None if counted32 is None else counted32 / (1e-3 * float(np.mean(farmx))) / 1e12
    out["mixed"] = {"value": pairs * side / dtmx, "unit": "pairs/s", "ms_per_step": 1e3 * dtmx / side,
                    "speedup_vs_fp64": (dt64 / args.steps) / (dtmx / side), "far_kernel_ms": float(np.mean(farmx)),
                    "roofline": {"bound": "alu", "achieved": mixed_ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                 "frac": mixed_ach / PEAK_FP32_TFLOPS,
                                 "counted_fp32_tflops": c32,
                                 "counted_frac": None if c32 is None else c32 / PEAK_FP32_TFLOPS}}

    g_flops = GRAD_FLOP_PER_NODE_INT * node_int + FLOP_PER_PAIR * pairs
    for prec, peak in (("fp64", PEAK_FP64_TFLOPS), ("mixed", PEAK_FP32_TFLOPS)):
        a_ = g_flops / (1e-3 * grad[prec]["far_kernel_ms"]) / 1e12
        grad[prec]["roofline"] = {"bound": "alu", "achieved": a_, "peak": peak, "unit": "TFLOP/s", "frac": a_ / peak}
    out["gradient"] = {k: {kk: vv for kk, vv in v.items() if kk != "G"} for k, v in grad.items()}
    out["gradient"]["flops_per_node_interaction"] = GRAD_FLOP_PER_NODE_INT

    dr_flops = FLOP_PER_NODE_INT * stdr["node_interactions"] + FLOP_PER_PAIR * pairs
    dr_ach = dr_flops / (1e-3 * float(np.mean(fardr))) / 1e12
    out["dr_rules"] = {"value": pairs * side / dtdr, "unit": "pairs/s", "precision": "fp64",
                       "ms_per_step": 1e3 * dtdr / side, "far_kernel_ms": float(np.mean(fardr)),
                       "node_interactions": stdr["node_interactions"],
                       "node_interactions_per_pair_choice": stdr["node_interactions_pair_rule"],
                       "node_interactions_fixed_rules": node_int,
                       "roofline": {"bound": "alu", "achieved": dr_ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                    "frac": dr_ach / PEAK_FP64_TFLOPS,
                                    **profiled("far_dr_fp64", dr_flops, float(np.mean(fardr)), PEAK_FP64_TFLOPS),
                                    "issue_ceiling": issue_ceiling(rates, "far_dr_fp64", stdr["node_interactions"],
                                                                   float(np.mean(fardr))),
                                    "note": "20 flops per executed node interaction + 16 per pair"},
                       "mixed_value": pairs * side / dtdrm, "mixed_far_kernel_ms": float(np.mean(fardrm)),
                       "rules": "triangles 7/12/19/33 points for DR >= 100/25/10/3, rectangles Tables B2/B3/B4 "
                                "and 7x7 Gauss for DR >= 150/40/15/3"}
    out["rect_table_b5"] = {"value": pairs * side / dtb5, "unit": "pairs/s", "precision": "fp64",
                            "ms_per_step": 1e3 * dtb5 / side, "far_kernel_ms": float(np.mean(farb5)),
                            "node_interactions": stb5["node_interactions"],
                            "mixed_value": pairs * side / dtb5m, "mixed_far_kernel_ms": float(np.mean(farb5m)),
                            "rules": "33-point triangles, Table B5 (33 points) rectangles"}

    if not args.quick:
        import oracle

        # CPU baseline on a bounded sample; the same oracle values check both precisions
        rng = np.random.default_rng(7)
        isn = w.info["is_near"]
        k_near = int(round(0.3 * args.cpu_sample))
        idx = np.concatenate([rng.choice(np.nonzero(~isn)[0], args.cpu_sample - k_near, replace=False),
                              rng.choice(np.nonzero(isn)[0], k_near, replace=False)])
        log(f"oracle on {idx.size} sampled points")
        t0 = time.perf_counter()
        ref = oracle.evaluate(w.tri, w.rect, w.sigma[0], w.points[idx], oracle.params(33, 7), with_abs=True)
        tc = time.perf_counter() - t0
        sample_pairs = idx.size * w.n_elements
        out["cpu_baseline"] = {"value": sample_pairs / tc, "unit": "pairs/s", "cores": ref["threads"],
                               "kind": "oracle",
                               "sample": f"{idx.size} of the 1,000,000 points (30 % near), all 150,000 elements, "
                                         f"{tc:.1f} s"}
        acc = {}
        for name, (p_, E_) in {"fp64": (phi64, E64), "mixed": (phimx, Emx)}.items():
            ep, ee, rp = nerr(p_[idx], E_[idx], ref)
            acc[name] = {"max_norm_err_phi": float(ep.max()), "max_norm_err_E": float(ee.max()),
                         "median_norm_err_phi": float(np.median(ep)), "median_norm_err_E": float(np.median(ee)),
                         "max_rel_err_phi": float(rp.max()), "median_rel_err_phi": float(np.median(rp))}
        for name, (p_, E_) in {"dr_fp64": (phidr, Edr), "dr_mixed": (phidrm, Edrm)}.items():
            ep, ee, rp = nerr(p_[idx], E_[idx], ref)
            acc[name] = {"max_norm_err_phi": float(ep.max()), "max_norm_err_E": float(ee.max()),
                         "median_rel_err_phi": float(np.median(rp))}
        out["accuracy_vs_oracle"] = acc
        # Table B5: parity with the oracle on the same rules, and its distance to the 7 x 7 Gauss result
        log(f"oracle with Table B5 rectangles on {idx.size} sampled points")
        refb5 = oracle.evaluate(w.tri, w.rect, w.sigma[0], w.points[idx],
                                oracle.params(33, rect_gl_n=0, rect_table_n=33), with_abs=True)
        for name, (p_, E_) in {"fp64": (phib5, Eb5), "mixed": (phib5m, Eb5m)}.items():
            ep, ee, _ = nerr(p_[idx], E_[idx], refb5)
            out["rect_table_b5"][f"{name}_max_norm_err_phi"] = float(ep.max())
            out["rect_table_b5"][f"{name}_max_norm_err_E"] = float(ee.max())
        ep, ee, _ = nerr(phib5[idx], Eb5[idx], ref)
        out["rect_table_b5"]["fp64_vs_gauss7x7_max_norm_diff_phi"] = float(ep.max())
        out["rect_table_b5"]["fp64_vs_gauss7x7_max_norm_diff_E"] = float(ee.max())
        gidx = idx[::10]
        log(f"oracle gradient on {gidx.size} sampled points")
        gref = oracle.gradient(w.tri, w.rect, w.sigma[0], w.points[gidx], oracle.params(33, 7))
        for prec in ("fp64", "mixed"):
            e = np.abs(grad[prec]["G"][gidx] - gref["G"]).max(axis=1) / gref["abs_T"]
            out["gradient"][prec]["max_norm_err"] = float(e.max())
            out["gradient"][prec]["median_norm_err"] = float(np.median(e))
        out["mixed"]["within_1e-6"] = acc["mixed"]["max_norm_err_phi"] <= 1e-6 and acc["mixed"]["max_norm_err_E"] <= 1e-6
        # the paper's plain relative error where it is well conditioned: sigma = 1 on every
        # element (no cancellation between elements), same sampled points
        log("plain relative error with sigma = 1")
        ones = np.ones(w.n_elements)
        ref1 = oracle.evaluate(w.tri, w.rect, ones, w.points[idx], oracle.params(33, 7))
        ctx.upload_densities(ones)
        sub = torch.tensor(np.ascontiguousarray(w.points[idx].T), dtype=torch.float64, device=dev)
        plain = {}
        for prec in ("fp64", "mixed"):
            p1, _, _ = ctx.eval(sub, prec)
            r = np.abs(p1.cpu().numpy() - ref1["phi"]) / np.abs(ref1["phi"])
            plain[prec] = {"max_rel_err_phi": float(r.max()), "median_rel_err_phi": float(np.median(r))}
        ctx.upload_densities(w.sigma)
        acc["sigma_one_plain"] = plain
        out["mixed"]["plain_rel_err_sigma_one_within_1e-6"] = plain["mixed"]["max_rel_err_phi"] <= 1e-6

        # collocation product: nested cylinders, 200,000 elements, 8 right-hand sides
        log("collocation: nested cylinders, 200,000 elements, 8 right-hand sides")
        wc = W.nested_cylinders_workload()
        cctx = bemc.Context(0)
        cctx.upload_geometry(wc.tri, wc.rect)
        sig = torch.tensor(wc.sigma, dtype=torch.float64, device=dev)
        colloc = {}
        for prec in ("fp64", "mixed"):
            res = cctx.collocation(sig, prec)
            # a product that forms its near stage (setting the rules again ends the reuse)
            cctx.set_rules()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = cctx.collocation(sig, prec, out=res)
            torch.cuda.synchronize()
            dt_first = time.perf_counter() - t0
            # the next product reuses it (as every product of a solve after the first)
            t0 = time.perf_counter()
            res = cctx.collocation(sig, prec, out=res)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = cctx.stats()
            rhs = wc.sigma.shape[0]
            cflops = COLLOC_FLOP_PER_NODE_INT * st["node_interactions"] + 2 * rhs * st["pairs"]
            peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_TFLOPS
            ach = cflops / (1e-3 * st["far_ms"]) / 1e12
            colloc[prec] = {"ms": 1e3 * dt, "ms_forming_near_stage": 1e3 * dt_first,
                            "timing_note": "ms: a product after another with the same geometry and rules, which "
                                           "reuses its near-pair list and near records (every product of a "
                                           "solve after the first); ms_forming_near_stage: a product that "
                                           "lists, orders and walks the near pairs itself",
                            "pairs_per_s": st["pairs"] / dt, "near_pairs": st["near_pairs"],
                            "far_kernel_ms": st["far_ms"], "near_kernel_ms": st["near_ms"],
                            "node_interactions": st["node_interactions"],
                            "roofline": {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                                         "frac": ach / peak,
                                         **profiled("colloc_" + prec, cflops, st["far_ms"], peak),
                                         "issue_ceiling": None if prec != "fp64" else issue_ceiling(
                                             rates, "colloc_fp64", st["node_interactions"], st["far_ms"]),
                                         "note": "11 flops per node interaction + 2 per pair and density"}}
        rows = np.random.default_rng(3).choice(wc.n_elements, 64, replace=False)
        cref = oracle.collocation(wc.tri, wc.rect, wc.sigma, rows=rows)
        got64 = res  # last result is mixed; recompute fp64 for the check
        got64 = cctx.collocation(sig, "fp64").cpu().numpy()[:, rows]
        gotmx = cctx.collocation(sig, "mixed").cpu().numpy()[:, rows]
        scale = cref["abs"]  # each right-hand side's own sum of |sigma_j phi_j| per row
        colloc["fp64"]["max_norm_err"] = float(np.max(np.abs(got64 - cref["out"]) / scale))
        colloc["mixed"]["max_norm_err"] = float(np.max(np.abs(gotmx - cref["out"]) / scale))
        colloc["workload"] = wc.name
        colloc["rhs"] = wc.sigma.shape[0]
        out["collocation"] = colloc
        cctx.close()

        out["solver"] = solver_bench(torch, bemc, W)
        out["icosphere"] = icosphere_bench(torch, bemc, W, reps=1000)

        if args.serving_queries > 0 or args.serving_queries_dr > 0:
            # one stream for long batches, one for queries of <= 4096 points; fixed rules,
            # then the rule choice by distance ratio on a longer prefix of the same stream;
            # served results of sampled queries checked against the oracle
            g = W.serving_geometry()
            policy = dict(max_batch_points=1 << 16, small_query_points=4096, n_streams=2)
            if args.serving_queries > 0:
                out["serving"] = serving(args.serving_queries, torch, bemc, W, g=g, check=4, **policy)
            if args.serving_queries_dr > 0:
                out["serving_dr"] = serving(args.serving_queries_dr, torch, bemc, W, g=g, dr=True, check=8, **policy)
    ctx.close()
    print(json.dumps(out), flush=True)


def icosphere_bench(torch, bemc, W, reps):
    """The 1,280-triangle icosphere with 4,096 points and the 7-point rule (every pair far):
    a launch-bound evaluation, timed over `reps` evaluations enqueued back to back."""
    log(f"icosphere: {reps} evaluations")
    w = W.icosphere_workload()
    ctx = bemc.Context(0)
    ctx.set_rules(7, 7)
    ctx.upload_geometry(w.tri, w.rect)
    ctx.upload_densities(w.sigma)
    ctx.set_near_capacity(1 << 16)  # fixed (no near pairs on this workload)
    pts = torch.tensor(np.ascontiguousarray(w.points.T), dtype=torch.float64, device="cuda:0")
    n = pts.shape[1]
    phi = torch.empty(n, dtype=torch.float64, device="cuda:0")
    E = torch.empty((3, n), dtype=torch.float64, device="cuda:0")
    for _ in range(20):
        ctx.eval(pts, "fp64", phi=phi, E=E)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.eval(pts, "fp64", phi=phi, E=E)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.stats()
    ctx.close()
    return {"workload": "icosphere R=1, 1,280 triangles (7-point rule), 4,096 points in 2 <= r <= 10",
            "reps": reps, "us_per_eval": 1e6 * dt / reps, "pairs_per_s": st["pairs"] * reps / dt,
            "far_kernel_us": 1e3 * st["far_ms"], "near_pairs": st["near_pairs"],
            "note": "each evaluation: near-pair list, far field, near stage (cost order, walk, per-point "
                    "finish); at most 4,096 points are taken in the caller's order"}


def solver_bench(torch, bemc, W):
    """Densities of a coaxial capacitor (inner cylinder 1 V, outer 0 V; 50,000 elements) by
    GMRES on the matrix-free collocation product."""
    log("solver: nested cylinders, 50,000 elements")
    w = W.nested_cylinders_workload(inner=(100, 100, 5000), outer=(150, 100, 7500), n_rhs=1)
    ctx = bemc.Context(0)
    ctx.upload_geometry(w.tri, w.rect)
    n_in_t, n_in_r = 10_000, 10_000
    pot = np.zeros(w.n_elements)
    pot[:n_in_t] = 1.0
    pot[w.tri.shape[0]:w.tri.shape[0] + n_in_r] = 1.0
    V = torch.tensor(pot, device="cuda:0")
    res = {}
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-6), ("refine", 1e-10)):
        sig, info = ctx.solve(V, tol=tol, max_iter=600, restart=60, precision=prec)
        torch.cuda.synchronize()
        s = sig.cpu().numpy()
        tri, rect = w.tri, w.rect
        a = np.concatenate([0.5 * np.linalg.norm(np.cross(tri[:, 3:6] - tri[:, 0:3], tri[:, 6:9] - tri[:, 0:3]), axis=1),
                            np.linalg.norm(rect[:, 3:6], axis=1) * np.linalg.norm(rect[:, 6:9], axis=1)])
        q = s * a
        inner = np.concatenate([np.arange(n_in_t), w.tri.shape[0] + np.arange(n_in_r)])
        res[prec] = dict(info, tol=tol, inner_charge_C=float(q[inner].sum()), total_charge_C=float(q.sum()))
        if prec == "fp64":
            s64 = s
        else:
            res[prec]["rel_diff_to_fp64_solution"] = float(np.linalg.norm(s - s64) / np.linalg.norm(s64))
    res["refine"]["note"] = "corrections by GMRES on mixed products, residuals by FP64 products"
    ctx.close()
    res["workload"] = "nested cylinders R=1 (z in [-5,5], 1 V) and R=2 (z in [-6,6], 0 V), 25k triangles + 25k rectangles"
    return res


def serving(n_queries, torch, bemc, W, g=None, dr=False, small_query_points=4096, max_batch_points=1 << 16,
            n_streams=2, check=0):
    """Open-loop Poisson arrivals on the 1,000,000-element cylinder: saturation rate from a
    burst of (at most) the first 500 queries, then arrivals at 0.7 x that rate; latency =
    arrival -> results in host memory.  check > 0: that many served queries (32 points of
    each) are compared with the oracle."""
    log(f"serving: 1,000,000-element cylinder, {n_queries} queries, rule choice by DR {dr}, "
        f"short-query class {small_query_points}, batch {max_batch_points}, {n_streams} streams")
    g = g or W.serving_geometry()
    ctx = bemc.Context(0)
    ctx.set_dr_rules(dr)
    ctx.upload_geometry(g.tri, g.rect)
    ctx.upload_densities(g.sigma)
    sizes = W.serving_query_sizes(20_000)[:n_queries]
    qpts = [np.ascontiguousarray(W.serving_query(i, s)) for i, s in enumerate(sizes)]
    phis = [np.empty(s) for s in sizes]
    Es = [np.empty((s, 3)) for s in sizes]
    ctx.server_start(mem_budget_bytes=16 << 30, max_batch_points=max_batch_points, n_streams=n_streams,
                     precision="mixed", small_query_points=small_query_points)
    # warm-up and saturation rate (a burst of the first queries at once)
    n_burst = min(n_queries, 500)
    t0 = time.perf_counter()
    tickets = [ctx.server_submit(qpts[i], phis[i], Es[i]) for i in range(n_burst)]
    for t in tickets:
        ctx.server_wait(t)
    burst = time.perf_counter() - t0
    sat_rate = n_burst / burst
    log(f"serving burst: {burst:.2f} s ({sat_rate:.1f} queries/s)")
    rate = 0.7 * sat_rate
    arrivals = W.poisson_arrivals(n_queries, rate)
    t0 = time.perf_counter()
    tickets = []
    for i in range(n_queries):
        while time.perf_counter() - t0 < arrivals[i]:
            time.sleep(min(1e-3, max(0.0, arrivals[i] - (time.perf_counter() - t0))))
        tickets.append((i, ctx.server_submit(qpts[i], phis[i], Es[i])))
    infos = [(i, ctx.server_wait(t)) for i, t in tickets]
    total = time.perf_counter() - t0
    # latency: submission (at the scheduled arrival) -> results in the host buffers
    lat = [1e3 * (info["end_s"] - info["submit_s"]) for _, info in infos]
    ctx.server_stop()
    ctx.close()
    pairs = int(np.sum(sizes)) * g.n_elements
    lat = np.array(lat)
    log(f"serving open loop: p50 {np.percentile(lat, 50):.1f} ms p99 {np.percentile(lat, 99):.1f} ms")
    lat_small = lat[np.array(sizes) <= max(small_query_points, 4096)]
    accuracy = None
    if check > 0:
        import oracle

        rng = np.random.default_rng(11)
        qs = rng.choice(n_queries, check, replace=False)
        sel = [(q, rng.choice(sizes[q], min(32, sizes[q]), replace=False)) for q in qs]
        P = np.concatenate([qpts[q][i] for q, i in sel])
        log(f"serving: oracle on {P.shape[0]} served points of {check} queries")
        ref = oracle.evaluate(g.tri, g.rect, g.sigma[0], P, oracle.params(33, 7, dr_rules=dr), with_abs=True)
        ph = np.concatenate([phis[q][i] for q, i in sel])
        Ev = np.concatenate([Es[q][i] for q, i in sel])
        ep = np.abs(ph - ref["phi"]) / ref["abs_phi"]
        ee = np.sum(np.abs(Ev - ref["E"]), axis=1) / ref["abs_E"]
        accuracy = {"points": int(P.shape[0]), "queries": int(check), "max_norm_err_phi": float(ep.max()),
                    "max_norm_err_E": float(ee.max()), "within_1e-6": bool(ep.max() <= 1e-6 and ee.max() <= 1e-6)}
    return {"workload": g.name, "queries": int(n_queries), "points": int(np.sum(sizes)),
            "accuracy_vs_oracle": accuracy, "burst_queries": n_burst,
            "precision": "mixed far field, FP64 near field",
            "rules": "by distance ratio" if dr else "33-point triangles, 7x7 rectangles",
            "policy": {"max_batch_points": max_batch_points, "streams": n_streams,
                       "short_query_class_points": small_query_points},
            "p50_ms_queries_le_4096_points": float(np.percentile(lat_small, 50)),
            "saturation_queries_per_s": sat_rate, "arrival_rate_queries_per_s": rate,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "pairs_per_s": pairs / total, "wall_s": total,
            "note": f"prefix of the 20,000-query stream ({n_queries} queries), sizes round(2^U(0,16))"}


if __name__ == "__main__":
    main()
