"""Benchmark of the FR hot path on one MI355X.

Headline workload: the 128x128x8 periodic box (131,072 hexahedra, 29.6 M
DOF) at Re 60000, Pr 0.72, Mach 0.1 base flow plus seeded divergence-free
Fourier modes, vertices perturbed by 5 % of the element width, p in
{1,2,3,4} with weights .3/.3/.25/.15 (synthetic, seeded).  A step computes
the FR residual R(U) and the exact tangent J(U) v in float64 from one
forward-mode (dual-number) pass; `value` is n_dof / (median step time) in
GDOF/s, with every input resident in HBM.

The same run reports, on that workload:
  * every operator alone (residual, float64 / float32 / finite-difference
    tangents, adjoint), in the degree-bucketed (fused) and per-bucket launch
    modes, median of >= 20 calls;
  * per-stage times of the step (HIP events on the launching stream, median);
  * the roofline of the step: the algorithmic bytes and flops of the
    residual + tangent per DOF (compulsory traffic: U and v read, R and Jv
    written, 217 B of mesh data per element; sum-factorised flops) against
    the FP64 vector peak and the HBM peak;
  * the implicit ESDIRK2 stage solve at these settings (GMRES(30) to 1e-6,
    PTC to 1e-4, dt 0.002) in the mixed form (float32 exact tangent and
    Krylov basis, captured Arnoldi graphs), in float64 with the exact
    tangent, and in the plain form (float64, finite-difference tangent,
    per-bucket launches, no graph) with the state-scaled step;
  * the same quantities on the 32x32x4 Re 3900 workload (cache-resident:
    absolute numbers only), including the full ESDIRK2 and ESDIRK4 steps;
  * the CPU oracle on a bounded sample of the headline workload at one
    thread and at every host thread.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --study {c3,c5,c3adapt,g2,precond}
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6
FP32_VECTOR_TFLOPS = 157.3
MESH_BYTES_PER_ELEMENT = 217  # 8 vertices (192 B), 6 neighbour ids (24 B), the degree (1 B)
# counted floating-point operations of the method (the oracle's residual on
# counted scalars), written by tests/golden/make_flop_counts.py
FLOP_COUNTS = os.path.join(ROOT, "tests", "golden", "flop_counts.json")
HEADLINE_SAMPLE = "navier_stokes_128x128x8_slab_4x128x8"


def planning_flops_per_dof(n):
    """The planning estimate of the Navier-Stokes residual's flops per DOF at
    n = p + 1 (about 60 n^4 per element of contractions plus pointwise and
    face work), kept beside the counted work for reference."""
    return 12.0 * n + 165.0 + 200.0 / n


def work_model(elem_p, sample=None):
    """Algorithmic work of the hot path on a degree field: bytes (compulsory
    HBM traffic: U, v read, R, Jv written, mesh data) and flops of each
    operator.  Flops are counted operations of the method per DOF: those of a
    sample of the same workload (mortar faces included) if one is named, else
    per degree from uniform periodic boxes.  The residual costs the counted
    residual; the tangents and the one-pass step cost the counted
    forward-mode dual evaluation (value and derivative)."""
    with open(FLOP_COUNTS) as f:
        counts = json.load(f)
    n = elem_p.astype(np.int64) + 1
    dof = 5 * n ** 3
    n_dof, E = float(dof.sum()), float(len(n))
    if sample:
        fres = counts[sample]["residual_per_dof"] * n_dof
        fdual = counts[sample]["dual_per_dof"] * n_dof
    else:
        tab = counts["uniform_4x4x4_navier_stokes"]
        fres = float(sum(dof[n == k].sum() * tab[str(k - 1)]["residual_per_dof"] for k in set(n.tolist())))
        fdual = float(sum(dof[n == k].sum() * tab[str(k - 1)]["dual_per_dof"] for k in set(n.tolist())))
    mesh = MESH_BYTES_PER_ELEMENT * E
    return {
        "n_dof": n_dof,
        "residual": {"bytes": 16 * n_dof + mesh, "flops": fres},
        "jvp_f64": {"bytes": 24 * n_dof + mesh, "flops": fdual},
        "jvp_f32": {"bytes": 12 * n_dof + mesh, "flops": fdual},
        "residual_and_jvp": {"bytes": 32 * n_dof + mesh, "flops": fdual},
        "planning_residual_flops": float((dof * np.array([planning_flops_per_dof(k) for k in n])).sum()),
    }


def roofline(work, t_s, peak_tflops=FP64_VECTOR_TFLOPS):
    """Fractions of the FP64 vector peak and of the HBM peak; the bound is the
    roof that takes longer for this work."""
    flops, by = work["flops"], work["bytes"]
    t_alu = flops / (peak_tflops * 1e12)
    t_hbm = by / (HBM_PEAK_GBS * 1e9)
    alu = {"bound": "alu", "achieved": round(flops / t_s / 1e12, 3), "peak": peak_tflops, "unit": "TFLOP/s",
           "frac": round(flops / t_s / 1e12 / peak_tflops, 4)}
    hbm = {"achieved_gbs": round(by / t_s / 1e9, 1), "frac": round(by / t_s / 1e9 / HBM_PEAK_GBS, 4)}
    out = dict(alu) if t_alu >= t_hbm else {"bound": "hbm", "achieved": hbm["achieved_gbs"], "peak": HBM_PEAK_GBS,
                                            "unit": "GB/s", "frac": hbm["frac"]}
    out["alu_frac"] = alu["frac"]
    out["hbm_frac"] = hbm["frac"]
    out["hbm_achieved_gbs"] = hbm["achieved_gbs"]
    out["algorithmic_bytes"] = by
    out["algorithmic_flops"] = flops
    out["attainable_gdof_s"] = round(work_n_dof(work) / max(t_alu, t_hbm) / 1e9, 2)
    return out


def work_n_dof(work):
    return work.get("n_dof", 0.0)


def median_ms(fn, reps, warmup, stream, torch):
    """Median over `reps` calls of fn, each bracketed by HIP events on the
    launching stream."""
    for _ in range(max(1, warmup)):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    t = [a.elapsed_time(b) for a, b in evs]
    return float(np.median(t)), float(np.mean(t))


def stage_medians(ctx, U, op, reps=20):
    """Per-launch times of one operator's kernels (fr_profile, HIP events on
    the stream): medians over `reps` single runs."""
    runs = [ctx.profile(U, op=op, reps=1) for _ in range(reps)]
    out = []
    for i, k in enumerate(runs[0]):
        ms = float(np.median([r[i]["ms"] for r in runs]))
        out.append({"stage": k["stage"], "units": int(k["units"]), "ms": round(ms, 5)})
    return out


def measured_traffic(name, key="traffic_bytes"):
    """HBM bytes per call of an operator from a committed rocprofv3 counter
    summary under profiles/ (lines 'source_sha256: ...', 'traffic_bytes:
    ...', 'fetched_bytes: ...', 'written_bytes: ...'), or None if there is
    none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            kv = dict(line.split(":", 1) for line in f if line.count(":") >= 1 and not line.startswith(("#", "|")))
    except OSError:
        return None
    kv = {k.strip().strip("-* `"): v.strip().strip("`") for k, v in kv.items()}
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


# sources that define the residual and tangent kernels and their launch plans
# (tile tables, face-slot order): a counter summary is used only while they
# hash to the value recorded in it
KERNEL_SOURCES = ("frx_device.hpp", "frx_residual.hpp", "frx_launch.hpp", "frx_k_dual64.hip", "frx_runtime.hip")
TRAFFIC_PROFILE = "residual_jvp_dual64_ns_128x128x8_hbm_traffic.md"


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1910_03693_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def host_cpu():
    """lscpu's model name and the number of host cores."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-implicit", action="store_true", help="skip the implicit-step comparisons")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-small", action="store_true", help="skip the 32x32x4 workload")
    ap.add_argument("--no-ops", action="store_true", help="skip the table of single operators")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB five times (reference for the HBM byte counters)")
    ap.add_argument("--forms", default=None,
                    help="c3 / c5 studies: comma-separated subset of the step forms (f64_exact_graph, "
                         "mixed_f32_exact_graph, mixed_f32_exact_graph_cgs1, plain_f64_fd_scaled, plain_f64_fd)")
    ap.add_argument("--study", choices=("c3", "c5", "c3adapt", "g2", "precond"), default=None,
                    help="instead of the headline: implicit steps on the 64x64x8 vortex street (c3) or the "
                         "128x128x8 box (c5), the adaptive vortex-street loop (c3adapt), or the p / p_max "
                         "refinement study of the isentropic vortex, uniform against adaptive degrees (g2)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the hot path is built and "
              "measured on a single MI355X, with no collectives).", file=sys.stderr)
        sys.exit(2)
    if args.study:
        if args.study == "c3adapt":
            res = adaptive_study()
        elif args.study == "g2":
            res = g2_study()
        elif args.study == "precond":
            res = precond_study()
        else:
            res = step_study(args.study, args.forms.split(",") if args.forms else None)
        print(json.dumps(res), flush=True)
        return

    import torch

    from paper_1910_03693_amd import frx
    from paper_1910_03693_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    case = I.config(5)
    ctx = frx.Context.from_case(case, max_restart=30, graphs=frx.FR_GRAPHS_F64_EXACT | frx.FR_GRAPHS_F32_EXACT)
    U = torch.tensor(case.U, device=dev)
    v = torch.tensor(I.random_direction(case.U.size, 4005).reshape(case.U.shape), device=dev)
    n_dof = ctx.n_dof
    E = int(case.mesh["n_elem"])
    print(f"[bench] workload 128x128x8 Re 60000, {E} elements, {n_dof} DOF", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ctx.autotune(U)
    t_tune = time.perf_counter() - t0
    shapes = {name: ctx.launch_shapes(k) for k, name in enumerate(("float64", "dual_float64", "dual_float32"))}
    print(f"[bench] autotuned in {t_tune:.1f} s; fused shapes (stage, code, items per tile) of the float64 dual "
          f"kernels: {shapes['dual_float64']}", file=sys.stderr, flush=True)
    ctx.set_launch(True)  # the batched design: one degree-bucketed launch per stage
    R, Jv = torch.empty_like(U), torch.empty_like(U)

    def step():
        # R(U) and J(U) v in float64 from one forward-mode pass
        ctx.residual_jvp(U, v, R, Jv)

    ms_step, ms_mean = median_ms(step, args.steps, args.warmup, stream, torch)
    value = n_dof / (ms_step * 1e-3) / 1e9
    print(f"[bench] residual + exact Jv (one pass): median {ms_step:.4f} ms/step (mean {ms_mean:.4f}), "
          f"{value:.3f} GDOF/s", file=sys.stderr, flush=True)

    W = work_model(case.elem_p, sample=HEADLINE_SAMPLE)
    W["residual_and_jvp"]["n_dof"] = n_dof
    roof = roofline(W["residual_and_jvp"], ms_step * 1e-3)
    stages = stage_medians(ctx, U, op=3)
    roof["kernel"] = ("fr_residual_jvp: " + " + ".join(s["stage"] for s in stages) +
                      " (Dual<double>, navier-stokes, roe)")
    roof["launch_ms"] = round(ms_step, 5)
    roof["stages"] = [dict(s, share=round(s["ms"] / sum(x["ms"] for x in stages), 3)) for s in stages]
    roof["work_model"] = (f"{W['residual_and_jvp']['flops'] / n_dof:.1f} flop/DOF (the oracle's counted "
                          f"forward-mode dual evaluation on a 4x128x8 slab of this workload, "
                          f"tests/golden/flop_counts.json; the residual alone "
                          f"{W['residual']['flops'] / n_dof:.1f}, the planning estimate 12n + 165 + 200/n "
                          f"{W['planning_residual_flops'] / n_dof:.1f}), "
                          f"{W['residual_and_jvp']['bytes'] / n_dof:.2f} B/DOF (U, v, R, Jv + "
                          f"{MESH_BYTES_PER_ELEMENT} B/element)")
    roof["traffic"] = measured_traffic(TRAFFIC_PROFILE)
    peaks = memory_peaks(torch)
    roof["measured_memory_peaks_gbs"] = peaks
    if roof["traffic"] is not None:
        roof["traffic_over_algorithmic"] = round(roof["traffic"] / roof["algorithmic_bytes"], 2)
        fetched = measured_traffic(TRAFFIC_PROFILE, "fetched_bytes")
        written = measured_traffic(TRAFFIC_PROFILE, "written_bytes")
        if fetched is not None and written is not None:
            # the step's measured reads and writes at the measured read-only
            # and write-only rates: the memory roof of this staged design
            t_mem = fetched / (peaks["read"] * 1e9) + written / (peaks["write"] * 1e9)
            roof["traffic_time_at_measured_peaks_ms"] = round(t_mem * 1e3, 4)
            roof["frac_of_measured_memory_roof"] = round(t_mem / (ms_step * 1e-3), 4)
    print(f"[bench] roofline {roof}", file=sys.stderr, flush=True)

    reps = max(20, args.steps // 2)
    v32 = v.float()
    J32 = torch.empty_like(v32)
    per_op = {}
    for mode in () if args.no_ops else ("fused", "per_bucket"):
        ctx.set_launch(mode == "fused")
        ops = {
            "residual_f64": (lambda: ctx.residual(U, out=R), W["residual"]),
            "jvp_exact_f64": (lambda: ctx.jvp(U, v, out=Jv), W["jvp_f64"]),
            "jvp_exact_f32": (lambda: ctx.jvp(U, v32, precision=frx.FR_F32, out=J32), W["jvp_f32"]),
            "jvp_fd_f64": (lambda: ctx.jvp(U, v, jv_mode=frx.FR_JV_FD, out=Jv), None),
            "residual_and_jvp_one_pass": (lambda: ctx.residual_jvp(U, v, R, Jv), W["residual_and_jvp"]),
            "vjp_f64": (lambda: ctx.vjp(U, v, out=Jv), None),
        }
        res = {}
        for k, (fn, w) in ops.items():
            t, _ = median_ms(fn, reps, 2, stream, torch)
            r = {"ms": round(t, 4), "gdof_s": round(n_dof / (t * 1e-3) / 1e9, 3)}
            if w is not None:
                w = dict(w, n_dof=n_dof)
                rf = roofline(w, t * 1e-3, FP32_VECTOR_TFLOPS if k == "jvp_exact_f32" else FP64_VECTOR_TFLOPS)
                r.update(alu_frac=rf["alu_frac"], hbm_frac=rf["hbm_frac"])
            res[k] = r
        per_op[mode] = res
        print(f"[bench] operators ({mode}): {res}", file=sys.stderr, flush=True)
    ctx.set_launch(True)
    del J32, v32

    out = {
        "metric": "GDOF/s for FR residual + exact Jv; implicit step time, mixed vs plain FP64",
        "value": round(value, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "ms_per_step_mean": round(ms_mean, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded mesh, degrees and Fourier-mode flow field)",
        "config": {"workload": "navier-stokes mixed-degree 128x128x8 periodic hex (131072 elements), Re 60000, "
                               "Mach 0.1, p in {1,2,3,4} w .3/.3/.25/.15, perturbed vertices",
                   "n_elem": E, "n_dof": int(n_dof),
                   "step": "R(U) and exact J(U)v, float64, from one forward-mode pass (fr_residual_jvp), "
                           "median of the timed steps",
                   "parallelism": "single GPU"},
        "roofline": roof,
        "operators": per_op,
        "launch_shapes": {"source": "fr_autotune on this workload", "seconds": round(t_tune, 2),
                          "fused_items_per_tile": {k: [list(x) for x in v2] for k, v2 in shapes.items()},
                          "legend": "(stage 0 trace / 1 interior faces / 2 divergence, code n or 8 n_low + n_high, "
                                    "items per 256-thread tile)"},
    }
    if args.copy_calibration > 0:
        out["copy_calibration"] = copy_calibration(torch, args.copy_calibration)
    if not args.no_implicit:
        out["implicit_stage_128x128x8"] = implicit_stage_c5(ctx, case, U, frx, torch)
    del R, Jv, v
    ctx.close()
    del U
    torch.cuda.empty_cache()
    if not args.no_small:
        out["small_32x32x4"] = small_workload(frx, I, torch, args, stream, not args.no_implicit)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds, value)
    print(json.dumps(out), flush=True)


def memory_peaks(torch, mib=2048, reps=10):
    """Achievable HBM rates on this GPU (GB/s), median of `reps`: read only
    (a sum over a float64 buffer), write only (a fill) and copy (bytes read
    plus bytes written), on 2 GiB buffers, far above the 256 MB Infinity
    Cache."""
    n = mib * 1024 * 1024 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    out = {}
    for name, fn, nbytes in (("read", lambda: x.sum(), 8 * n), ("write", lambda: y.fill_(0.5), 8 * n),
                             ("copy", lambda: y.copy_(x), 16 * n)):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            t.append(a.elapsed_time(b))
        out[name] = round(nbytes / (float(np.median(t)) * 1e-3) / 1e9, 1)
    del x, y
    torch.cuda.empty_cache()
    return out


def copy_calibration(torch, mib):
    """A plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE
    counters give the scale from counter units to bytes."""
    n = mib * 1024 * 1024 // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / 5
    return {"bytes_read": n * 8, "bytes_written": n * 8, "ms": round(ms, 4),
            "gb_s": round(2 * n * 8 / (ms * 1e-3) / 1e9, 1)}


def _timed_step(ctx, U, dt, torch, **kw):
    Uw = U.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ctx.esdirk_step(Uw, dt, **kw)
    torch.cuda.synchronize()
    return Uw, (time.perf_counter() - t0) * 1e3, st


def implicit_stage_c5(ctx, case, U, frx, torch):
    """The first implicit stage of an ESDIRK2 step (dt 0.002; PTC from
    dtau 2e-4 up to 4e-3, to 1e-4; GMRES(30) to 1e-6 relative, at most 300
    products) in the forms: mixed (float32 exact tangent and basis, graph;
    Gram-Schmidt twice, and once as in PETSc's GMRES), float64 exact (graph)
    and plain (float64 finite differences with the step scaled to the state,
    per-bucket launches, no graph).  The plain form with
    the paper's absolute step (1e-6 along the unit direction, 29.6 M
    components) stagnates here: see the c5 study."""
    dt = 0.002
    common = dict(dtau_init=2e-4, dtau_max=4e-3, tol_pseudo=1e-4, max_ptc_iter=50, last_stage=2)
    g = dict(restart=30, max_iter=300, tol=1e-6)
    res = {"dt": dt, "settings": {**common, **g}}
    outs = {}
    for name, gv, fused in (("mixed_f32_exact_graph", dict(g, precision=frx.FR_F32, use_graph=True), True),
                            ("mixed_f32_exact_graph_cgs1", dict(g, precision=frx.FR_F32, use_graph=True,
                                                                orthog=frx.FR_ORTHO_CGS), True),
                            ("f64_exact_graph", dict(g, precision=frx.FR_F64, use_graph=True), True),
                            ("plain_f64_fd_scaled", dict(g, jv_mode=frx.FR_JV_FD_SCALED, precision=frx.FR_F64),
                             False)):
        ctx.set_launch(fused)
        Uw, ms, st = _timed_step(ctx, U, dt, torch, gmres=gv, **common)
        outs[name] = Uw
        res[name] = {"ms": round(ms, 1), **st, "launch": "fused" if fused else "per-bucket"}
        print(f"[bench] 128x128x8 stage {name}: {ms:.1f} ms {st}", file=sys.stderr, flush=True)
    ctx.set_launch(True)
    ref = outs["f64_exact_graph"]
    for name in ("mixed_f32_exact_graph", "mixed_f32_exact_graph_cgs1", "plain_f64_fd_scaled"):
        res[f"rel_diff_{name}_vs_f64_exact"] = (outs[name] - ref).norm().item() / ref.norm().item()
    res["rel_change_of_stage"] = (ref - U).norm().item() / U.norm().item()
    res["speedup_mixed_vs_plain"] = round(res["plain_f64_fd_scaled"]["ms"] / res["mixed_f32_exact_graph"]["ms"], 3)
    res["speedup_mixed_cgs1_vs_plain"] = round(res["plain_f64_fd_scaled"]["ms"] /
                                               res["mixed_f32_exact_graph_cgs1"]["ms"], 3)
    return res


def small_workload(frx, I, torch, args, stream, implicit):
    """The 32x32x4 Re 3900 workload: cache-resident (U is 6 MB), so its numbers
    are absolute, not HBM evidence."""
    case = I.config(2)
    ctx = frx.Context.from_case(case, max_restart=30, graphs=frx.FR_GRAPHS_F64_EXACT | frx.FR_GRAPHS_F32_EXACT)
    U = torch.tensor(case.U, device="cuda")
    v = torch.tensor(I.random_direction(case.U.size, 4002).reshape(case.U.shape), device="cuda")
    R, Jv = torch.empty_like(U), torch.empty_like(U)
    ctx.autotune(U)
    ctx.set_launch(True)
    t, tm = median_ms(lambda: ctx.residual_jvp(U, v, R, Jv), max(20, args.steps), args.warmup, stream, torch)
    res = {"n_dof": int(ctx.n_dof), "residual_and_jvp_one_pass": {"ms": round(t, 5), "ms_mean": round(tm, 5),
                                                                   "gdof_s": round(ctx.n_dof / (t * 1e-3) / 1e9, 3)}}
    ops = {"residual_f64": lambda: ctx.residual(U, out=R), "jvp_exact_f64": lambda: ctx.jvp(U, v, out=Jv),
           "jvp_fd_f64": lambda: ctx.jvp(U, v, jv_mode=frx.FR_JV_FD, out=Jv), "vjp_f64": lambda: ctx.vjp(U, v, out=Jv)}
    for k, fn in ops.items():
        tk, _ = median_ms(fn, 20, 2, stream, torch)
        res[k] = {"ms": round(tk, 5), "gdof_s": round(ctx.n_dof / (tk * 1e-3) / 1e9, 3)}
    print(f"[bench] 32x32x4: {res}", file=sys.stderr, flush=True)
    if implicit:
        res["implicit_step"] = implicit_steps_small(ctx, U, frx, torch)
    ctx.close()
    return res


def implicit_steps_small(ctx, U, frx, torch):
    """One ESDIRK2 step (dt 0.005, dtau from dt/10 to dt, PTC to 1e-4,
    GMRES(30) to 1e-1): plain (float64, finite-difference Jv with the paper's
    step, per-bucket launches, no graph) versus mixed (float32 exact Jv and
    basis, graph) and float64 exact (graph); and one ESDIRK4 step, mixed."""
    dt = 0.005
    common = dict(dtau_init=dt / 10, dtau_max=dt, tol_pseudo=1e-4, max_ptc_iter=50)
    base = dict(restart=30, max_iter=100, tol=1e-1)
    res = {"dt": dt, "settings": {**common, **base}}
    outs = {}
    for name, g, fused, scheme in (
            ("plain_f64_fd", dict(base, jv_mode=frx.FR_JV_FD), False, frx.FR_ESDIRK2),
            ("mixed_f32_exact_graph", dict(base, precision=frx.FR_F32, use_graph=True), True, frx.FR_ESDIRK2),
            ("f64_exact_graph", dict(base, precision=frx.FR_F64, use_graph=True), True, frx.FR_ESDIRK2),
            ("esdirk4_mixed_f32_exact_graph", dict(base, precision=frx.FR_F32, use_graph=True), True,
             frx.FR_ESDIRK4)):
        ctx.set_launch(fused)
        _timed_step(ctx, U, dt, torch, gmres=g, scheme=scheme, **common)  # warm-up
        Uw, ms, st = _timed_step(ctx, U, dt, torch, gmres=g, scheme=scheme, **common)
        outs[name] = Uw
        res[name] = {"ms": round(ms, 3), **st, "launch": "fused" if fused else "per-bucket"}
        print(f"[bench] 32x32x4 step {name}: {ms:.2f} ms {st}", file=sys.stderr, flush=True)
    ctx.set_launch(True)
    res["rel_diff_mixed_vs_plain"] = ((outs["plain_f64_fd"] - outs["mixed_f32_exact_graph"]).norm().item() /
                                      outs["plain_f64_fd"].norm().item())
    res["rel_change_of_step"] = (outs["plain_f64_fd"] - U).norm().item() / U.norm().item()
    res["speedup_mixed_vs_plain"] = round(res["plain_f64_fd"]["ms"] / res["mixed_f32_exact_graph"]["ms"], 3)
    return res


def slab_of(case, nx_slab):
    """The first nx_slab columns (in x) of a structured box workload: its
    elements, degrees and state, closed periodically in x (the sample the
    CPU oracle is timed on)."""
    from paper_1910_03693_amd import inputs as I

    nx, ny, nz = case.mesh["shape"]
    ix = np.arange(case.mesh["n_elem"]) % nx
    sel = np.nonzero(ix < nx_slab)[0]  # mesh order (x fastest) is kept
    L = case.mesh["lengths"]
    m = I.box_mesh(nx_slab, ny, nz, (L[0] * nx_slab / nx, L[1], L[2]))
    m["elem_xyz"] = case.mesh["elem_xyz"][sel]
    off = I.sp_offsets(case.elem_p)
    cols = np.concatenate([np.arange(off[e], off[e + 1]) for e in sel])
    sub = I.Case("slab", m, case.elem_p[sel].copy(), np.ascontiguousarray(case.U[:, cols]), case.physics,
                 case.flux, case.gamma, case.mu, case.prandtl, case.farfield, {})
    return sub


def cpu_baseline(case, seconds, gpu_value):
    """The CPU oracle as it stands (plain loops; OpenMP over elements and
    faces), timed on the host: residual + complex-step exact tangent (the
    headline step's two results) on a 16x128x8 slab of the headline workload
    (an eighth of its elements, same degrees and field), once at one thread and
    once at every host thread, each repeated until `seconds` have passed."""
    import oracle

    sub = slab_of(case, 16)
    orc = oracle.Oracle.from_case(sub)
    v = np.random.default_rng(4005).normal(size=sub.U.shape)
    model, _ = host_cpu()
    ncpu = oracle.threads()  # OpenMP's default: OMP_NUM_THREADS if set, else the cores it may use
    runs = {}
    for th in (1, ncpu):
        oracle.set_threads(th)
        t0 = time.perf_counter()
        ts = []
        while True:
            t1 = time.perf_counter()
            orc.residual(sub.U)
            orc.jvp(sub.U, v)
            ts.append(time.perf_counter() - t1)
            if time.perf_counter() - t0 >= seconds:
                break
        med = float(np.median(ts))
        runs[th] = {"gdof_s": round(sub.U.size / med / 1e9, 6), "seconds_per_step": round(med, 3), "reps": len(ts)}
        print(f"[bench] cpu oracle, {th} thread(s): {runs[th]}", file=sys.stderr, flush=True)
    oracle.set_threads(ncpu)
    best = runs[ncpu]
    return {"value": best["gdof_s"], "unit": "GDOF/s", "cores": ncpu, "kind": "oracle",
            "sample": f"residual + complex-step exact Jv on a 16x128x8 slab of the 128x128x8 workload "
                      f"({sub.U.size} DOF), median of {best['reps']} at {ncpu} threads",
            "single_thread": runs[1], "all_threads": best, "host_cpu": model,
            "gpu_over_cpu": round(gpu_value / best["gdof_s"], 1)}


def adaptive_study(steps=4):
    """The paper's loop on the 64x64x8 vortex street: starting from the
    indicator's degree field, each time step is one implicit ESDIRK2 step
    (mixed form) followed by one p-adaptation on the device (indicator,
    criteria with the maximum indicator of the same degree, face limiter, new
    degree buckets, projected state)."""
    import torch

    from paper_1910_03693_amd import adapt, frx
    from paper_1910_03693_amd import inputs as I

    p, _ = adapt.indicator_degree_field(lambda ep: I.case_street(elem_p=ep))
    case = I.case_street(elem_p=p)
    ctx = frx.Context.from_case(case, max_restart=30, graphs=frx.FR_GRAPHS_F32_EXACT, fused=True)
    U = torch.tensor(case.U, device="cuda")
    dt = 0.05
    common = dict(dtau_init=0.005, dtau_max=0.05, tol_pseudo=1e-4, max_ptc_iter=50)
    g = dict(restart=30, max_iter=100, tol=1e-1, precision=frx.FR_F32, use_graph=True)
    out = {"study": "c3adapt", "dt": dt, "settings": {**common, **g}, "steps": []}
    for k in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.esdirk_step(U, dt, gmres=g, **common)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        case, ctx2, U = adapt.adapt_step(case, ctx, U, reserve=dict(max_restart=30, graphs=frx.FR_GRAPHS_F32_EXACT),
                                         fused=True, eta_max_scope=frx.FR_ETA_MAX_SAME_DEGREE)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if ctx2 is not ctx:
            ctx.close()
        ctx = ctx2
        rec = {"step_ms": round((t1 - t0) * 1e3, 1), "adapt_ms": round((t2 - t1) * 1e3, 1), **st,
               "n_dof_after": int(ctx.n_dof),
               "degree_histogram_p1_to_p5_after": np.bincount(case.elem_p, minlength=6)[1:].tolist()}
        out["steps"].append(rec)
        print(f"[bench] c3adapt step {k}: {rec}", file=sys.stderr, flush=True)
    return out


def step_study(which, forms=None):
    """Implicit steps on a larger workload (not the headline): c3 = 64x64x8
    vortex street with the degree field chosen by the spectral-decay indicator
    (one full ESDIRK2 step, GMRES(30) to 1e-1); c5 = the 128x128x8 box at
    Re 60000, Mach 0.1 with the settings of the paper's SD7003 runs (one full
    ESDIRK2 step, GMRES(30) to 1e-6), including the plain form with the
    paper's absolute finite-difference step."""
    import torch

    from paper_1910_03693_amd import adapt, frx
    from paper_1910_03693_amd import inputs as I

    out = {"study": which}
    if which == "c3":
        p, hist = adapt.indicator_degree_field(lambda ep: I.case_street(elem_p=ep))
        case = I.case_street(elem_p=p)
        out["degree_histogram_p1_to_p5"] = np.bincount(p, minlength=6)[1:].tolist()
        dt, common = 0.05, dict(dtau_init=0.005, dtau_max=0.05, tol_pseudo=1e-4, max_ptc_iter=50)
        g = dict(restart=30, max_iter=100, tol=1e-1)
    else:
        case = I.config(5)
        dt, common = 0.002, dict(dtau_init=2e-4, dtau_max=4e-3, tol_pseudo=1e-4, max_ptc_iter=50)
        g = dict(restart=30, max_iter=300, tol=1e-6)
    ctx = frx.Context.from_case(case, max_restart=30, graphs=frx.FR_GRAPHS_F64_EXACT | frx.FR_GRAPHS_F32_EXACT)
    U = torch.tensor(case.U, device="cuda")
    ctx.autotune(U)
    out["n_dof"] = int(ctx.n_dof)
    out["dt"] = dt
    out["settings"] = {**common, **g}
    variants = (("f64_exact_graph", dict(g, precision=frx.FR_F64, use_graph=True), True),
                ("mixed_f32_exact_graph", dict(g, precision=frx.FR_F32, use_graph=True), True),
                ("mixed_f32_exact_graph_cgs1", dict(g, precision=frx.FR_F32, use_graph=True,
                                                    orthog=frx.FR_ORTHO_CGS), True),
                ("plain_f64_fd_scaled", dict(g, jv_mode=frx.FR_JV_FD_SCALED, precision=frx.FR_F64), False),
                ("plain_f64_fd", dict(g, jv_mode=frx.FR_JV_FD, precision=frx.FR_F64), False))
    if forms:
        variants = tuple(v for v in variants if v[0] in forms)
    outs = {}
    for name, gv, fused in variants:
        ctx.set_launch(fused)
        Uw, ms, st = _timed_step(ctx, U, dt, torch, gmres=gv, **common)
        outs[name] = Uw
        out[name] = {"ms": round(ms, 1), **st, "launch": "fused" if fused else "per-bucket"}
        print(f"[bench] {which} {name}: {ms:.1f} ms {st}", file=sys.stderr, flush=True)
    ref = outs.get("f64_exact_graph")
    for name in ("mixed_f32_exact_graph", "mixed_f32_exact_graph_cgs1", "plain_f64_fd_scaled", "plain_f64_fd"):
        if ref is not None and name in outs:
            out[f"rel_diff_{name}_vs_f64_exact"] = (outs[name] - ref).norm().item() / ref.norm().item()
    if "plain_f64_fd_scaled" in out and "mixed_f32_exact_graph" in out:
        out["speedup_mixed_vs_plain_scaled"] = round(out["plain_f64_fd_scaled"]["ms"] /
                                                     out["mixed_f32_exact_graph"]["ms"], 3)
    return out


def precond_study():
    """The element-Jacobi preconditioner (section 2.3) against none, in the
    mixed form (float32 exact tangent and basis, float32 blocks, and the same
    with the inverse kept in float16) and in float64, GMRES with one-pass
    Gram-Schmidt: on the 32x32x4 workload one full ESDIRK2 step at the paper's
    settings (dt 0.005, dtau 5e-4 .. 5e-3, PTC to 1e-4, GMRES(30) to 1e-1);
    on the 128x128x8 workload one full ESDIRK2 step (dt 0.002, dtau 2e-4 ..
    4e-3, GMRES(30) to 1e-6).  The step builds the preconditioner once at its
    start (sigma = 1/(omega dt) + 1/dtau_max) and uses it in both implicit
    stages; its build time is also measured alone."""
    import torch

    from paper_1910_03693_amd import frx
    from paper_1910_03693_amd import inputs as I

    out = {"study": "precond"}
    for name, k, dt, common, g in (
            ("32x32x4", 2, 0.005, dict(dtau_init=5e-4, dtau_max=5e-3, tol_pseudo=1e-4, max_ptc_iter=50),
             dict(restart=30, max_iter=100, tol=1e-1)),
            ("128x128x8_step", 5, 0.002, dict(dtau_init=2e-4, dtau_max=4e-3, tol_pseudo=1e-4, max_ptc_iter=50),
             dict(restart=30, max_iter=300, tol=1e-6))):
        case = I.config(k)
        res = {"dt": dt, "settings": {**common, **g}}
        for prec, pname, form in ((frx.FR_F32, "mixed_f32", 1), (frx.FR_F32, "mixed_f32_inverse_f16", 2),
                                  (frx.FR_F64, "f64", 1)):
            if k == 5 and prec == frx.FR_F64:
                continue  # float64 blocks of this workload take 94 GB; the float32 ones are timed
            resv = (frx.FR_RESERVE_PRECOND_F32 if prec == frx.FR_F32 else frx.FR_RESERVE_PRECOND_F64) | \
                (frx.FR_GRAPHS_F32_EXACT if prec == frx.FR_F32 else frx.FR_GRAPHS_F64_EXACT)
            ctx = frx.Context.from_case(case, max_restart=30, graphs=resv, fused=True)
            U = torch.tensor(case.U, device="cuda")
            sigma = 1.0 / ((1.0 - 2 ** -0.5) * dt) + 1.0 / common["dtau_max"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.precond_build(U, sigma, frx.FR_PC_F16 if form == 2 else prec)
            torch.cuda.synchronize()
            t_build = (time.perf_counter() - t0) * 1e3
            x = torch.tensor(I.random_direction(case.U.size, 4090).reshape(case.U.shape), device="cuda")
            y = torch.empty_like(x)
            t_apply, _ = median_ms(lambda: ctx.precond_apply(x, out=y), 5, 1, torch.cuda.current_stream(), torch)
            for pc in ((0, form) if form == 1 else (form,)):
                gg = dict(g, precision=prec, use_graph=True, precond=pc, orthog=frx.FR_ORTHO_CGS)
                Uw, ms, st = _timed_step(ctx, U, dt, torch, gmres=gg, **common)
                key = f"{pname}_{'element_jacobi' if pc else 'none'}"
                res[key] = {"ms": round(ms, 1), **st}
                print(f"[bench] precond {name} {key}: {ms:.1f} ms {st}", file=sys.stderr, flush=True)
            res[f"{pname}_build_ms"] = round(t_build, 1)
            res[f"{pname}_apply_ms"] = round(t_apply, 3)
            print(f"[bench] precond {name} {pname}: build {t_build:.1f} ms, apply {t_apply:.3f} ms", file=sys.stderr,
                  flush=True)
            ctx.close()
            del U, x, y
            torch.cuda.empty_cache()
        out[name] = res
    return out


def _vortex_l2_error(case, U, t, uinf, period):
    """L2 errors (over the domain, Gauss weights times |J| of the cube
    elements) of the solution against the exact translated vortex sampled at
    the same solution points: all conserved variables, and density alone."""
    from paper_1910_03693_amd import inputs as I

    X = I.solution_points(case.mesh, case.elem_p)
    Ue = I.vortex_field(X[0], X[1], X[2], 0.0, 0.0, t=t, ma=0.5, uinf=uinf, period=period)
    h = np.asarray(case.mesh["lengths"]) / np.asarray(case.mesh["shape"])
    jac = float(np.prod(h / 2.0))
    w = np.empty(X.shape[1])
    off = I.sp_offsets(case.elem_p)
    for n in range(2, 7):
        els = np.nonzero(case.elem_p.astype(np.int64) + 1 == n)[0]
        if not len(els):
            continue
        g = np.polynomial.legendre.leggauss(n)[1]
        wk = (g[None, None, :] * g[None, :, None] * g[:, None, None]).ravel()  # xi fastest
        for e in els:
            w[off[e]:off[e + 1]] = wk * jac
    d = U - Ue
    return float(np.sqrt(np.sum(d * d * w[None, :]))), float(np.sqrt(np.sum(d[0] * d[0] * w)))


def g2_study(p_values=(1, 2, 3, 4, 5), steps=60):
    """The p / p_max refinement study of the isentropic vortex (section 3.3):
    2-D vortex (alpha 5, phi 1/2) in the free stream (rho, u, v, w) =
    (1, 1, 1, 0), Mach 0.5, on a periodic [-10, 10]^2 x [0, 0.8] box of
    50 x 50 x 2 cubes, 60 steps of dt = 0.05 (PTC from dtau 0.05 up to 10, to
    1e-4; GMRES(30) to 1e-1), in the mixed form on one GPU, with ESDIRK2 and
    with ESDIRK4.  For each k: uniform p = k against the adaptive solver with
    p_min = 1, p_max = k (started from uniform p_max, adapted after every step
    on the device: indicator of rho u, nu_max 0.1, nu_min 0.001, one-degree
    face limiter, new context, projected state), with the criteria's maximum
    indicator read over all elements and over the elements of the same
    degree.  Reports the L2 error against the exact translated vortex at
    t = 3, the run time (every step and adaptation) and the run-time
    reduction of the adaptive solver."""
    import torch

    from paper_1910_03693_amd import adapt, frx
    from paper_1910_03693_amd import inputs as I

    L, Lz, uinf, dt = 20.0, 0.8, (1.0, 1.0, 0.0), 0.05
    mesh = I.box_mesh(50, 50, 2, (L, L, Lz), origin=(-L / 2, -L / 2, 0.0))
    period = (L, L)
    common = dict(dtau_init=0.05, dtau_max=10.0, tol_pseudo=1e-4, max_ptc_iter=100)
    g = dict(restart=30, max_iter=100, tol=1e-1, precision=frx.FR_F32, use_graph=True)
    reserve = dict(max_restart=30, graphs=frx.FR_GRAPHS_F32_EXACT)

    def make(ep):
        U = I.sample(mesh, ep, lambda x, y, z: I.vortex_field(x, y, z, 0.0, 0.0, ma=0.5, uinf=uinf, period=period))
        return I.Case("vortex", mesh, np.asarray(ep, np.int8), U, 0, 0, I.GAMMA, 0.0, 0.72, np.zeros(5), {})

    def run(k, scheme, scope):
        case = make(np.full(mesh["n_elem"], k, np.int8))
        ctx = frx.Context.from_case(case, fused=True, **reserve)
        U = torch.tensor(case.U, device="cuda")
        gm = ptc = 0
        dof_steps = []
        t_adapt = 0.0
        n_new = 0  # adaptations that changed the degree field (a new context)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st = ctx.esdirk_step(U, dt, gmres=g, scheme=scheme, **common)
            if st["status"] != frx.FR_OK:
                raise RuntimeError(f"step failed: {st}")
            gm += st["gmres_iterations"]
            ptc += st["ptc_iterations"]
            dof_steps.append(ctx.n_dof)
            if scope is not None:
                ta = time.perf_counter()
                case, ctx2, U = adapt.adapt_step(case, ctx, U, p_min=1, p_max=k, reserve=reserve, fused=True,
                                                 eta_max_scope=scope)
                if ctx2 is not ctx:
                    ctx.close()
                    n_new += 1
                ctx = ctx2
                t_adapt += time.perf_counter() - ta
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        err, err_rho = _vortex_l2_error(case, U.cpu().numpy(), steps * dt, uinf, period)
        ctx.close()
        rec = {"run_ms": round(ms, 1), "adapt_ms": round(t_adapt * 1e3, 1), "new_contexts": n_new,
               "l2_error": err, "l2_error_rho": err_rho,
               "gmres_iterations": gm, "ptc_iterations": ptc, "mean_dof": int(np.mean(dof_steps)),
               "final_degree_histogram_p1_to_p5": np.bincount(case.elem_p, minlength=6)[1:].tolist()}
        print(f"[bench] g2 scheme {scheme} {'uniform p' if scope is None else 'adaptive (scope %d) p_max' % scope}"
              f" = {k}: {rec}", file=sys.stderr, flush=True)
        return rec

    out = {"study": "g2", "mesh": "50x50x2 periodic cubes on [-10,10]^2 x [0,0.8]", "dt": dt, "steps": steps,
           "settings": {**common, **g}, "free_stream": "(rho, u, v, w) = (1, 1, 1, 0), Mach 0.5", "runs": {}}
    run(2, frx.FR_ESDIRK2, None)  # warm-up: kernels and graph paths loaded once
    for scheme, sname in ((frx.FR_ESDIRK2, "esdirk2"), (frx.FR_ESDIRK4, "esdirk4")):
        res = {"uniform": {}, "adaptive_eta_max_all": {}, "adaptive_eta_max_same_degree": {}}
        for k in p_values:
            res["uniform"][k] = run(k, scheme, None)
            for key, scope in (("adaptive_eta_max_all", frx.FR_ETA_MAX_ALL),
                               ("adaptive_eta_max_same_degree", frx.FR_ETA_MAX_SAME_DEGREE)):
                r = run(k, scheme, scope) if k > 1 else dict(res["uniform"][k])
                r["run_time_reduction"] = round(1.0 - r["run_ms"] / res["uniform"][k]["run_ms"], 4)
                # without the adaptations themselves (new context, graphs, projection)
                r["solver_time_reduction"] = round(1.0 - (r["run_ms"] - r["adapt_ms"]) / res["uniform"][k]["run_ms"], 4)
                res[key][k] = r
        out["runs"][sname] = res
    return out


if __name__ == "__main__":
    main()
