"""Benchmark of the FR hot path on one MI355X.

Workload: Navier-Stokes, mixed degree, 32x32x4 periodic hexahedra with
perturbed vertices, Re 3900, Pr 0.72, Mach 0.2 base flow plus seeded
divergence-free Fourier modes, p in {1,2,3,4} with weights .4/.3/.2/.1
(synthetic, seeded).  A step computes the FR residual R(U) and the exact
tangent J(U) v in float64, both from one forward-mode (dual-number) pass;
`value` is GDOF/s for that pair (n_dof / step time); the same pair from two
separate calls is reported beside it.  The same run also reports each operator alone, the
float32 and finite-difference tangents, the implicit ESDIRK2 step in its
plain (float64, finite-difference Jv, per-bucket launches, no graph) and
mixed (float32 exact Jv and Krylov basis, graph-captured Arnoldi) forms, the
roofline of the dominant kernel and the CPU oracle on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
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

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6
FP32_VECTOR_TFLOPS = 157.3
SK_NAME = {0: "float64", 1: "dual float64", 2: "dual float32"}


def fused_counts(stage, elem_p, faces_by_pair, op, ns=True):
    """Bytes and nominal flops of one fused launch: the sum over its buckets."""
    by = fl = 0.0
    if stage in ("k_trace_fused", "k_div_fused"):
        base = stage.replace("_fused", "")
        for n, cnt in elem_p.items():
            b, f = nominal_counts(base, n, n, cnt, op, ns)
            by += b
            fl += f
    else:
        for (nl, nh), cnt in faces_by_pair.items():
            b, f = nominal_counts("k_face" if nl > 0 else "k_bface", abs(nl), nh, cnt, op, ns)
            by += b
            fl += f
    return by, fl


def nominal_counts(stage, nl, nh, units, op, ns=True):
    """Algorithmic bytes and nominal flops of one launch.

    Bytes: the launch's compulsory inputs and outputs (state, tangent
    direction, face data, result; the element stages read 24 map
    coefficients per element, the face stages the precomputed face-point
    geometry: the area vector and, for Navier-Stokes, the lifting
    coefficients).
    Flops: the arithmetic of the stage's formulation counted per solution or
    face point (multiply-add = 2), a dual number doubling the products."""
    sb_in = 8 if op < 2 else 4             # state / result precision
    n_in = 1 if op == 0 else 2             # U (and v for a tangent)
    sb_T = {0: 8, 1: 16, 2: 8}[op]         # face-buffer scalar
    sb_g = 8 if op < 2 else 4              # geometry scalar
    dual = 1.0 if op == 0 else 2.5
    n = nh
    if stage == "k_trace":
        n3, n2 = n ** 3, n * n
        by = units * (5 * n3 * sb_in * n_in + (24 * 8 if ns else 0) + (30 + (90 if ns else 0)) * n2 * sb_T)
        fl = units * (60 * n3 + (n3 * (30 * n + 185) + 180 * n3 if ns else 0)) * dual
    elif stage == "k_div":
        n3, n2 = n ** 3, n * n
        by = units * (5 * n3 * sb_in * n_in + 24 * 8 + (60 if ns else 30) * n2 * sb_T + 5 * n3 * sb_in)
        fl = units * n3 * ((60 * n + 570) if ns else (30 * n + 160)) * dual + units * 60 * n3 * dual
    elif stage == "k_face":
        by = units * ((20 if ns else 5) * (nl * nl + nh * nh) * sb_T + (5 if ns else 3) * nh * nh * sb_g
                      + 10 * (nl * nl + nh * nh) * sb_T)
        fl = units * nh * nh * (500 if ns else 200) * dual
    else:  # boundary faces
        by = units * ((20 if ns else 5) * n * n * sb_T + (4 if ns else 3) * n * n * sb_g + 10 * n * n * sb_T)
        fl = units * n * n * (400 if ns else 150) * dual
    return float(by), float(fl)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-implicit", action="store_true", help="skip the ESDIRK2 step comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB five times (reference for the HBM byte counters)")
    ap.add_argument("--study", choices=("c3", "c5", "c3adapt"), default=None,
                    help="instead of the headline: the implicit-step comparison on the 64x64x8 vortex street "
                         "(c3, degrees from the indicator) or the 128x128x8 Re 60000 box (c5)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the hot path is built and "
              "measured on a single MI355X, with no collectives).", file=sys.stderr)
        sys.exit(2)
    if args.study:
        res = adaptive_study() if args.study == "c3adapt" else step_study(args.study)
        print(json.dumps(res), flush=True)
        return

    import torch

    from paper_1910_03693_amd import frx
    from paper_1910_03693_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    case = I.config(2)
    ctx = frx.Context.from_case(case)
    U = torch.tensor(case.U, device=dev)
    v = torch.tensor(I.random_direction(case.U.size, 4002).reshape(case.U.shape), device=dev)
    v32 = v.float()
    R = torch.empty_like(U)
    Jv = torch.empty_like(U)
    J32 = torch.empty_like(v32)
    n_dof = ctx.n_dof
    print(f"[bench] workload ns_mixed 32x32x4, {case.mesh['n_elem']} elements, {n_dof} DOF", file=sys.stderr,
          flush=True)
    ctx.autotune(U)
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps  # ms

    def step():
        # R(U) and J(U) v in float64 from one forward-mode pass: the dual-number
        # kernels carry the residual in their value part
        ctx.residual_jvp(U, v, R, Jv)

    def step_separate():
        ctx.residual(U, out=R)
        ctx.jvp(U, v, out=Jv)

    # the batched design: one degree-bucketed launch per stage
    ctx.set_launch(True)

    # headline: K timed steps of (residual + exact float64 tangent)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    value = n_dof / (ms_step * 1e-3) / 1e9
    print(f"[bench] residual + exact Jv (one pass): {ms_step:.4f} ms/step, {value:.2f} GDOF/s", file=sys.stderr,
          flush=True)

    reps = max(20, args.steps // 2)
    ms_sep = timed(step_separate, args.steps)
    print(f"[bench] separate residual and exact Jv calls: {ms_sep:.4f} ms, {n_dof / (ms_sep * 1e-3) / 1e9:.2f} GDOF/s",
          file=sys.stderr, flush=True)
    per_op = {}
    for mode in ("fused", "per_bucket"):
        ctx.set_launch(mode == "fused")
        ops = {
            "residual_f64": timed(lambda: ctx.residual(U, out=R), reps),
            "jvp_exact_f64": timed(lambda: ctx.jvp(U, v, out=Jv), reps),
            "jvp_exact_f32": timed(lambda: ctx.jvp(U, v32, precision=frx.FR_F32, out=J32), reps),
            "jvp_fd_f64": timed(lambda: ctx.jvp(U, v, jv_mode=frx.FR_JV_FD, out=Jv), reps),
            "residual_and_jvp_one_pass": timed(lambda: ctx.residual_jvp(U, v, R, Jv), reps),
            "vjp_f64": timed(lambda: ctx.vjp(U, v, out=Jv), reps),
        }
        per_op[mode] = {k: {"ms": round(t, 5), "gdof_s": round(n_dof / (t * 1e-3) / 1e9, 3)} for k, t in ops.items()}
    ctx.set_launch(True)
    # the nodal filter (p > 2, alpha = 0.2; one launch per filtered degree in either mode), in place
    Uf = U.clone()
    t_f = timed(lambda: ctx.nodal_filter(Uf, 0.2, 3, out=Uf), reps)
    n_filt = int(5 * ((case.elem_p.astype(np.int64) + 1) ** 3)[case.elem_p >= 3].sum())
    per_op["nodal_filter_p_gt_2"] = {"ms": round(t_f, 5), "filtered_dof": n_filt,
                                     "gb_s": round(16 * n_filt / (t_f * 1e-3) / 1e9, 1)}

    # per-kernel timing of the float64 tangent in the batched launch (HIP events on this stream)
    kt = ctx.profile(U, op=1, reps=20)
    for k in kt:
        k["total_ms"] = k["ms"]
    dom = max(kt, key=lambda k: k["ms"])
    counts_n = {int(p) + 1: int(c) for p, c in zip(*np.unique(case.elem_p, return_counts=True))}
    pairs = {}
    nbr = case.mesh["elem_nbr"]
    for e in range(case.mesh["n_elem"]):
        ne = int(case.elem_p[e]) + 1
        for f in range(6):
            nb = int(nbr[e, f])
            if nb >= 0 and f % 2 == 1:
                nn = int(case.elem_p[nb]) + 1
                key = (min(ne, nn), max(ne, nn))
                pairs[key] = pairs.get(key, 0) + 1
            elif nb < 0:
                pairs[(-ne, ne)] = pairs.get((-ne, ne), 0) + 1
    if dom["stage"].endswith("_fused"):
        by, fl = fused_counts(dom["stage"], counts_n, pairs, 1)
    else:
        by, fl = nominal_counts(dom["stage"], dom["n_lo"], dom["n_hi"], dom["units"], 1)
    intensity = fl / by
    ridge = FP64_VECTOR_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    t_s = dom["ms"] * 1e-3
    if intensity >= ridge:
        roof = {"bound": "alu", "achieved": round(fl / t_s / 1e12, 3), "peak": FP64_VECTOR_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": round(by / t_s / 1e9, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["traffic"] = measured_traffic(dom["stage"])
    flux = "rusanov" if case.flux == 1 else "roe"
    roof["kernel"] = f"{dom['stage']}<{SK_NAME[1]},navier-stokes,{flux}>" if dom["stage"].endswith("_fused") else \
        f"{dom['stage']}<n={dom['n_hi']}{'' if dom['n_lo'] == dom['n_hi'] else ',' + str(dom['n_lo'])}," \
        f"{SK_NAME[1]},navier-stokes,{flux}>"
    roof["launch_ms"] = round(dom["ms"], 5)
    roof["algorithmic_bytes"] = by
    roof["nominal_flops"] = fl
    print(f"[bench] dominant kernel {roof['kernel']}: {dom['ms']:.4f} ms, {roof}", file=sys.stderr, flush=True)

    out = {
        "metric": "GDOF/s for FR residual + exact Jv; implicit step time, mixed vs plain FP64",
        "value": round(value, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded mesh, degrees and Fourier-mode flow field)",
        "config": {"workload": "navier-stokes mixed-degree 32x32x4 periodic hex, Re 3900, Mach 0.2, "
                               "p in {1,2,3,4} w .4/.3/.2/.1, perturbed vertices",
                   "n_elem": int(case.mesh["n_elem"]), "n_dof": int(n_dof),
                   "step": "R(U) and exact J(U)v, float64, from one forward-mode pass (fr_residual_jvp)",
                   "parallelism": "single GPU"},
        "separate_calls": {"ms": round(ms_sep, 5), "gdof_s": round(n_dof / (ms_sep * 1e-3) / 1e9, 3),
                           "calls": "fr_residual + fr_jvp(exact, float64)"},
        "operators": per_op,
        "kernels_jvp_f64": [{k2: (round(v2, 5) if isinstance(v2, float) else v2) for k2, v2 in k.items()
                             if k2 != "total_ms"} for k in kt],
        "roofline": roof,
    }

    if args.copy_calibration > 0:
        out["copy_calibration"] = copy_calibration(torch, args.copy_calibration)
    if not args.no_implicit:
        out["implicit_step"] = implicit_steps(ctx, case, U, frx, torch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds)
    print(json.dumps(out), flush=True)


# Sources that define the dominant kernel (the fused face stage of the float64
# tangent).  Its HBM traffic is taken from the rocprofv3 FETCH_SIZE / WRITE_SIZE
# summary under profiles/ only while these files hash to the value recorded
# there; after any change to them `traffic` is null until the counters are
# taken again.
TRAFFIC_SOURCES = ("frx_device.hpp", "frx_residual.hpp", "frx_launch.hpp", "frx_host.hpp", "frx_k_dual64.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "face_fused_dual64_ns_32x32x4_hbm_traffic.md")


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1910_03693_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(stage):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (lines 'kernel: ...', 'source_sha256: ...', 'traffic_bytes: ...'),
    or None if there is none or the kernel's sources have changed since."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            kv = dict(line.split(":", 1) for line in f if line.count(":") >= 1 and not line.startswith(("#", "|")))
    except OSError:
        return None
    kv = {k.strip().strip("-* `"): v.strip().strip("`") for k, v in kv.items()}
    if kv.get("kernel") != stage or kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes"])
    except (KeyError, ValueError):
        return None


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


def implicit_steps(ctx, case, U, frx, torch):
    """One ESDIRK2 step, plain float64 / finite-difference Jv / uniform launches
    versus mixed float32 exact Jv + float32 basis + graph, same tolerances;
    and one six-stage ESDIRK4 step in the mixed form."""
    dt = 0.005
    common = dict(dtau_init=dt / 10, dtau_max=dt, tol_pseudo=1e-4, max_ptc_iter=50)
    plain_g = dict(restart=30, max_iter=100, tol=1e-1, jv_mode=frx.FR_JV_FD, precision=frx.FR_F64,
                   use_graph=False)
    mixed_g = dict(restart=30, max_iter=100, tol=1e-1, jv_mode=frx.FR_JV_EXACT, precision=frx.FR_F32,
                   use_graph=True)
    exact64_g = dict(mixed_g, precision=frx.FR_F64)
    res = {"dt": dt, "settings": {**common, "restart": 30, "tol_gmres": 1e-1}}
    outs = {}
    for name, g, fused, scheme in (("plain_f64_fd", plain_g, False, frx.FR_ESDIRK2),
                                   ("mixed_f32_exact_graph", mixed_g, True, frx.FR_ESDIRK2),
                                   ("f64_exact_graph", exact64_g, True, frx.FR_ESDIRK2),
                                   ("esdirk4_mixed_f32_exact_graph", mixed_g, True, frx.FR_ESDIRK4)):
        ctx.set_launch(fused)
        Uw = U.clone()
        ctx.esdirk_step(Uw, dt, gmres=g, scheme=scheme, **common)  # warm-up (allocation, capture)
        Uw = U.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.esdirk_step(Uw, dt, gmres=g, scheme=scheme, **common)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        outs[name] = Uw
        res[name] = {"ms": round(ms, 3), **st}
        res[name]["launch"] = "fused" if fused else "per-bucket"
        print(f"[bench] implicit step {name}: {ms:.2f} ms {st}", file=sys.stderr, flush=True)
    ctx.set_launch(True)
    d = (outs["plain_f64_fd"] - outs["mixed_f32_exact_graph"]).norm().item()
    res["rel_diff_mixed_vs_plain"] = d / outs["plain_f64_fd"].norm().item()
    res["rel_change_of_step"] = (outs["plain_f64_fd"] - U).norm().item() / U.norm().item()
    res["speedup_mixed_vs_plain"] = round(res["plain_f64_fd"]["ms"] / res["mixed_f32_exact_graph"]["ms"], 3)
    return res


def adaptive_study(steps=4):
    """The paper's loop on the 64x64x8 vortex street: starting from the
    indicator's degree field, each time step is one implicit ESDIRK2 step
    (mixed form) followed by one p-adaptation on the device (indicator,
    criteria, face limiter, new degree buckets, projected state)."""
    import torch

    from paper_1910_03693_amd import adapt, frx
    from paper_1910_03693_amd import inputs as I

    p, _ = adapt.indicator_degree_field(lambda ep: I.case_street(elem_p=ep))
    case = I.case_street(elem_p=p)
    ctx = frx.Context.from_case(case)
    ctx.set_launch(True)
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
        case, ctx2, U = adapt.adapt_step(case, ctx, U)
        ctx2.set_launch(True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ctx.close()
        ctx = ctx2
        rec = {"step_ms": round((t1 - t0) * 1e3, 1), "adapt_ms": round((t2 - t1) * 1e3, 1), **st,
               "n_dof_after": int(ctx.n_dof),
               "degree_histogram_p1_to_p5_after": np.bincount(case.elem_p, minlength=6)[1:].tolist()}
        out["steps"].append(rec)
        print(f"[bench] c3adapt step {k}: {rec}", file=sys.stderr, flush=True)
    return out


def step_study(which):
    """One ESDIRK2 step in the plain, FP64-exact and mixed forms on a larger
    workload (not the headline): c3 = 64x64x8 vortex street with the degree
    field chosen by the spectral-decay indicator; c5 = 128x128x8 box at
    Re 60000, Mach 0.1 with the settings of the paper's SD7003 runs."""
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
    ctx = frx.Context.from_case(case)
    U = torch.tensor(case.U, device="cuda")
    out["n_dof"] = int(ctx.n_dof)
    out["dt"] = dt
    # the operators alone on this workload (fused launches, HIP events)
    ctx.set_launch(True)
    vv = torch.tensor(I.random_direction(case.U.size, 4005).reshape(case.U.shape), device="cuda")
    R, J = torch.empty_like(U), torch.empty_like(U)
    J32 = torch.empty_like(vv, dtype=torch.float32)
    v32 = vv.float()

    def t_op(fn, reps=10, batches=3):
        # median over batches of reps calls: a single batch can catch a stall
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(batches):
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b) / reps)
        return float(np.median(times))

    ops = {"residual_f64": t_op(lambda: ctx.residual(U, out=R)),
           "jvp_exact_f64": t_op(lambda: ctx.jvp(U, vv, out=J)),
           "jvp_exact_f32": t_op(lambda: ctx.jvp(U, v32, precision=frx.FR_F32, out=J32)),
           "residual_and_jvp_one_pass": t_op(lambda: ctx.residual_jvp(U, vv, R, J)),
           "vjp_f64": t_op(lambda: ctx.vjp(U, vv, out=J))}
    out["operators_fused"] = {k: {"ms": round(t, 4), "gdof_s": round(ctx.n_dof / (t * 1e-3) / 1e9, 3)}
                              for k, t in ops.items()}
    print(f"[bench] {which} operators: {out['operators_fused']}", file=sys.stderr, flush=True)
    # per-stage times of the float64 tangent and their algorithmic bandwidth
    # (this working set does not fit the Infinity Cache)
    kt = ctx.profile(U, op=1, reps=5)
    counts_n = {int(p) + 1: int(c) for p, c in zip(*np.unique(case.elem_p, return_counts=True))}
    pairs = {}
    nbr = case.mesh["elem_nbr"]
    for e in range(case.mesh["n_elem"]):
        ne = int(case.elem_p[e]) + 1
        for f in range(6):
            nb = int(nbr[e, f])
            if nb >= 0 and f % 2 == 1:
                nn = int(case.elem_p[nb]) + 1
                key = (min(ne, nn), max(ne, nn))
                pairs[key] = pairs.get(key, 0) + 1
            elif nb < 0:
                pairs[(-ne, ne)] = pairs.get((-ne, ne), 0) + 1
    stages = []
    for k in kt:
        by, fl = fused_counts(k["stage"], counts_n, pairs, 1)
        stages.append({"stage": k["stage"], "ms": round(k["ms"], 4), "algorithmic_bytes": by,
                       "gb_s": round(by / (k["ms"] * 1e-3) / 1e9, 1), "hbm_frac": round(by / (k["ms"] * 1e-3) / 1e9 /
                                                                                      HBM_PEAK_GBS, 4)})
    out["tangent_f64_stages"] = stages
    print(f"[bench] {which} tangent stages: {stages}", file=sys.stderr, flush=True)
    del R, J, J32, v32, vv
    out["settings"] = {**common, **g}
    variants = (("f64_exact_graph", dict(g, precision=frx.FR_F64, use_graph=True), True),
                ("mixed_f32_exact_graph", dict(g, precision=frx.FR_F32, use_graph=True), True),
                ("plain_f64_fd", dict(g, jv_mode=frx.FR_JV_FD, precision=frx.FR_F64, use_graph=False), False))
    outs = {}
    for name, gv, fused in variants:
        ctx.set_launch(fused)
        Uw = U.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.esdirk_step(Uw, dt, gmres=gv, **common)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        outs[name] = Uw
        out[name] = {"ms": round(ms, 1), **st, "launch": "fused" if fused else "per-bucket"}
        print(f"[bench] {which} {name}: {ms:.1f} ms {st}", file=sys.stderr, flush=True)
    ref = outs["f64_exact_graph"]
    for name in ("mixed_f32_exact_graph", "plain_f64_fd"):
        out[f"rel_diff_{name}_vs_f64_exact"] = (outs[name] - ref).norm().item() / ref.norm().item()
    out["speedup_mixed_vs_plain"] = round(out["plain_f64_fd"]["ms"] / out["mixed_f32_exact_graph"]["ms"], 3)
    return out


def cpu_baseline(case, seconds):
    """The CPU oracle as it stands (single thread) on a bounded sample: repeated
    residual + complex-step exact tangent on the same workload."""
    import oracle

    orc = oracle.Oracle.from_case(case)
    v = np.random.default_rng(4002).normal(size=case.U.shape)
    t0 = time.perf_counter()
    n = 0
    while True:
        orc.residual(case.U)
        orc.jvp(case.U, v)
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = (time.perf_counter() - t0) / n
    return {"value": round(case.U.size / dt / 1e9, 6), "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} x (residual + complex-step exact Jv) on the full 32x32x4 workload, "
                      f"{dt:.3f} s each, single-threaded"}


if __name__ == "__main__":
    main()
