#!/usr/bin/env python3
"""Power-ψ benchmark on one MI355X.

Default workload (cl_40m), the largest single-GPU configuration: directed
Chung–Lu follower graph, N = 40,000,000 users, mean degree 35 (≈1.4·10⁹
edges after clean-up), exponent 2.1, followers per user capped at 3·10⁶ (hub
rows), λ, μ ~ LogNormal(0, 2), tolerance 1e-8 on ‖s_t − s_{t−1}‖₁, int32
CSR.  A step is one complete time-to-ψ solve (all Power-ψ passes, the fused
axpy and gap reductions, and the final ψ pass; with a warm start also the
network's inference) on the operator already resident in HBM; the one-time
operator build is timed separately.

value = edges traversed per second over the whole solve (Σ passes × M / t),
in GTEPS; ms_per_step = time-to-ψ.  The headline mode is the fastest of FP64
(factored operator), MIXED (FP32 corrections + FP64 residual) and the
learned warm start ahead of each of those two, each in the schedule the
autotuner picked; all are reported with the plain FP64 per-edge-weight
iteration as the comparator.  The Anderson-accelerated solve and the
asynchronous block Gauss–Seidel sweeps (same fixed point and stopping test,
fewer passes) are reported beside them.  On big
workloads the comparison modes are timed over fewer solves
(--compare-steps); the headline mode is timed over --steps after --warmup.

cpu_baseline: the C/OpenMP oracle (oracle/psi_oracle_c.c, FP64 Algorithm 2)
on every host thread, on the same workload: whole solves after its own
operator build (excluded, like the GPU's), repeated to about 10 s of CPU
work; its ψ is also the parity reference of every GPU mode in the line.

Other workloads (--workload): cl_1m (N=1e6, 2e7 edges), cl_10m (N=1e7, 2e8
edges), cl_4m_k64 (64 activity scenarios on one N=4e6, 8e7-edge graph,
batched), graphs256 (256 graphs with N in [1e3, 1e5] in one batched solve).

Prints one JSON line.  ``--gpus N`` with N > 1 exits: the benchmark runs on one
GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS per iteration + time-to-ψ at tol 1e-8 (1 MI355X), vs plain FP64"
DEFAULT_WORKLOAD = "cl_40m"
SINGLE = ("cl_1m", "cl_10m", "cl_40m")
PEAK_HBM_GBS = 8000.0
WEIGHTS = os.path.join(ROOT, "paper_2206_09960_amd", "weights", "warmstart_cl.npy")
DESCRIPTIONS = {
    "cl_1m": "directed Chung-Lu, N=1,000,000, mean degree 20, exponent 2.2, "
             "lambda,mu ~ LogNormal(0,1.5), tol 1e-8 (L1 step), int32 CSR",
    "cl_10m": "directed Chung-Lu, N=10,000,000, mean degree 20, exponent 2.2, "
              "lambda,mu ~ LogNormal(0,1.5), tol 1e-8 (L1 step), int32 CSR",
    "cl_40m": "directed Chung-Lu, N=40,000,000, mean degree 35, exponent 2.1, max followers "
              "3,000,000, lambda,mu ~ LogNormal(0,2), tol 1e-8 (L1 step), int32 CSR",
    "cl_4m_k64": "64 activity scenarios (LogNormal(0,1.5), independent streams) on one directed "
                 "Chung-Lu graph, N=4,000,000, mean degree 20, exponent 2.2, tol 1e-8 per scenario",
    "graphs256": "256 directed Chung-Lu graphs, N_g uniform in [1,000, 100,000], mean degree 15, "
                 "exponent 2.2, LogNormal(0,1.5), tol 1e-8 per graph, one block-diagonal operator",
}


def algorithmic_bytes(kind: str, n: int, m: int, segs: int = 1) -> int:
    """Compulsory HBM bytes of one pass (each array touched once): the
    per-edge and per-user figures of the scope table's roofline."""
    if kind in ("step64", "part64", "band64", "bins64"):  # col 4M; row_ptr 4, z 8, c 8,
        return 4 * m + 44 * n                   # mu 8, invden 8, s_new 8 (factored FP64 pass)
    if kind == "step64_w":   # col 4M + val 8M; row_ptr 4, s 8, c 8, s_new 8
        return 12 * m + 28 * n
    if kind in ("step32", "part32", "band32", "bins32"):  # col 4M; row_ptr 4, ze 4, r 4,
        return 4 * m + 32 * n                   # mu 4, invden 4, e_old 4, e_new 4, ze_new 4 (FP32)
    if kind == "final64":    # col 4M; row_ptr 4, z 8, lam 8, d 8, psi 8
        return 4 * m + 36 * n
    raise ValueError(kind)


def batched_bytes(kind: str, n: int, m: int, k: int) -> int:
    """Compulsory bytes of one pass over a K-scenario batch (the pattern read
    once): the FP64 step (per user and scenario z, c, mu, invden, s_new: 8 B
    each) or the factored FP32 SpMM (ze, r, mu, invden, e_new: 4 B each)."""
    if kind == "scen64":
        return 4 * m + 4 * n + 40 * k * n
    if kind == "scen32":
        return 4 * m + 4 * n + 20 * k * n
    raise ValueError(kind)


def source_hash() -> str:
    """Hash of the code (comments and blank lines left out) of the source that
    defines the pass kernels whose HBM traffic the committed counter summaries
    record."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2206_09960_amd", "csrc")
    for f in ("psi_pass.hip",):
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            code = [ln.split("//", 1)[0].rstrip() for ln in fh]
        h.update(f.encode() + "\n".join(ln for ln in code if ln).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_kind: str, workload: str, kernel: str, alg: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing, was taken on other kernel sources, or on another
    launch configuration (kernel instance or column segments)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_kind}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if (rec.get("source_hash") != source_hash() or rec.get("kernel") != kernel
            or rec.get("algorithmic_bytes") != alg):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(n, follower, leader, lam, mu, tol, min_seconds=10.0, max_solves=10):
    """The C/OpenMP oracle (FP64 Algorithm 2, every host thread) on the same
    workload: its own operator build from the raw edges (excluded), then
    whole solves until about min_seconds of CPU work; the median counts."""
    import statistics

    import oracle.psi_oracle_c as oc
    t0 = time.perf_counter()
    G = oc.Graph(n, follower, leader, lam, mu)
    t_build = time.perf_counter() - t0
    times = []
    r = None
    while not times or (sum(times) < min_seconds and len(times) < max_solves):
        r = G.power_psi(tol)
        times.append(r["seconds"] + r["final_seconds"])
    t_solve = statistics.median(times)
    passes = r["iterations"] + 1
    threads = oc.max_threads()
    return dict(value=passes * G.m / t_solve / 1e9, unit="GTEPS", cores=threads, kind="oracle",
                sample=f"{'median of ' + str(len(times)) + ' whole solves' if len(times) > 1 else 'one whole solve'} "
                       f"of the same workload (N={n}, M={G.m}, {passes} passes, FP64 Algorithm 2 "
                       f"in C with OpenMP on {threads} threads; {sum(times):.1f}s in all); its "
                       f"operator build from the raw edges ({t_build:.1f}s) excluded",
                seconds=t_solve, iterations=r["iterations"]), r["psi"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed(fn, k, w):
    import torch
    for _ in range(w):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(k):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / k, out


def generate(name):
    import synth
    t0 = time.perf_counter()
    big = name in ("cl_10m", "cl_40m", "cl_4m_k64", "graphs256")
    g = synth.workload(name, device="cuda" if big else None)
    log(f"generated {name}: N={g.n} M_raw={g.m_raw} in {time.perf_counter() - t0:.1f}s")
    return g


def run_single(args, name):
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_2206_09960_amd import api

    tol = synth.WORKLOADS[name]["tol"]
    g = generate(name)
    f_dev = torch.as_tensor(g.follower).cuda()
    l_dev = torch.as_tensor(g.leader).cuda()
    lam_dev = torch.from_numpy(g.lam).cuda()
    mu_dev = torch.from_numpy(g.mu).cuda()
    torch.cuda.synchronize()
    builds = []
    for _ in range(2 if name == "cl_1m" else 1):
        t0 = time.perf_counter()
        op = api.Operator(g.n, f_dev, l_dev, lam_dev, mu_dev, flags=api.PSI_WEIGHTED_FP64)
        torch.cuda.synchronize()
        builds.append((time.perf_counter() - t0) * 1e3)
    # host copies of the raw edges for the CPU oracle (drawn on the GPU for big workloads)
    f_host = f_dev.cpu().numpy() if not isinstance(g.follower, np.ndarray) else g.follower
    l_host = l_dev.cpu().numpy() if not isinstance(g.leader, np.ndarray) else g.leader
    del f_dev, l_dev
    g.follower = g.leader = None
    torch.cuda.empty_cache()
    st = op.stats()
    m = st["n_edges"]
    log(f"operator built: M={m} max_row={st['max_followers']} in {builds[-1]:.1f} ms")

    t0 = time.perf_counter()
    tuned = {p: op.autotune(p) for p in ("fp64_weighted", "fp64", "mixed")}
    tune_ms = (time.perf_counter() - t0) * 1e3
    log(f"autotuned in {tune_ms:.0f} ms: {tuned}")
    bands = op.band_info()

    big = m > 200_000_000
    cmp_k = max(1, min(args.steps, args.compare_steps)) if big else args.steps
    cmp_w = 1 if big else args.warmup
    modes = {}
    for prec in ("fp64_weighted", "fp64", "mixed"):
        ms, (psi, info) = timed(lambda: op.solve(tol=tol, precision=prec), cmp_k, cmp_w)
        assert info["status"] == 0, (prec, info)
        modes[prec] = dict(ms=ms, info=info, psi=psi.cpu().numpy())
        log(f"{prec}: {ms:.3f} ms/solve, {info['spmv_passes']} passes "
            f"({info['iterations']} FP64, {info['fp32_passes']} FP32), layout "
            f"{api.SEG_FORM_NAMES[info['seg_form']]}")

    warm = None
    if not args.no_warm and os.path.exists(WEIGHTS):
        model = api.Model(np.load(WEIGHTS))
        s0 = model.warmstart(op)
        ms_inf, _ = timed(lambda: model.warmstart(op, s0_out=s0), cmp_k, cmp_w)
        with open(os.path.splitext(WEIGHTS)[0] + ".json") as fh:
            rec = json.load(fh)
        lo = rec.get("n_users_min", min(rec.get("n_users", [0])))
        hi = rec.get("n_users_max", max(rec.get("n_users", [0])))
        warm = dict(ms_inference=round(ms_inf, 4),
                    model=f"3-layer message passing, hidden 64, trained on {rec['n_graphs']} "
                          f"Chung-Lu graphs of N in [{lo}, {hi}] ({rec['steps']} Adam steps)")
        # the warm start ahead of each cold mode: the solve from s0 plus inference
        for prec in ("fp64", "mixed"):
            wname = f"{prec}_warm"
            ms, (psi, info) = timed(lambda: op.solve(tol=tol, precision=prec,
                                                     s0=model.warmstart(op, s0_out=s0)),
                                    cmp_k, cmp_w)
            assert info["status"] == 0, (wname, info)
            modes[wname] = dict(ms=ms, info=info, psi=psi.cpu().numpy())
            warm[wname] = dict(ms_total=round(ms, 4), passes_warm=info["spmv_passes"],
                               passes_cold=modes[prec]["info"]["spmv_passes"],
                               ms_cold=round(modes[prec]["ms"], 4), used_s0=info["used_s0"])
            log(f"{wname}: {ms:.3f} ms/solve incl. {ms_inf:.3f} ms inference, "
                f"{info['spmv_passes']} passes (cold {modes[prec]['info']['spmv_passes']})")

    # Anderson-accelerated passes (same fixed point and stopping test; reported,
    # not a headline candidate: the headline is Power-ψ itself)
    ms_aa, (psi_aa, info_aa) = timed(lambda: op.solve_anderson(tol=tol, depth=4), cmp_k, cmp_w)
    assert info_aa["status"] == 0, info_aa
    modes["fp64_anderson"] = dict(ms=ms_aa, info=info_aa, psi=psi_aa.cpu().numpy())
    log(f"fp64_anderson: {ms_aa:.3f} ms/solve, {info_aa['spmv_passes']} passes")
    # the same mixing in each FP32 correction solve of the mixed refinement
    ms_am, (psi_am, info_am) = timed(lambda: op.solve_anderson(tol=tol, depth=4,
                                                               precision="mixed"), cmp_k, cmp_w)
    assert info_am["status"] == 0, info_am
    modes["mixed_anderson"] = dict(ms=ms_am, info=info_am, psi=psi_am.cpu().numpy())
    log(f"mixed_anderson: {ms_am:.3f} ms/solve, {info_am['spmv_passes']} passes "
        f"({info_am['iterations']} FP64, {info_am['fp32_passes']} FP32)")
    # asynchronous local updates: block Gauss–Seidel sweeps over the band layout
    # (same fixed point and stopping test; reported beside, like Anderson)
    ms_gs, (psi_gs, info_gs) = timed(lambda: op.solve_async(tol=tol), cmp_k, cmp_w)
    assert info_gs["status"] == 0, info_gs
    modes["fp64_async"] = dict(ms=ms_gs, info=info_gs, psi=psi_gs.cpu().numpy())
    log(f"fp64_async: {ms_gs:.3f} ms/solve, {info_gs['spmv_passes']} passes (sweeps + final)")

    # per-origin newsfeed shares (Algorithm 1 for 64 origins at once), for the
    # 64 most influential users; their ψ_i must agree with Power-ψ's
    origins = None
    if g.n <= 4_000_000:
        psi64 = modes["fp64"]["psi"]
        top = np.argsort(-psi64, kind="stable")[:64]
        ms_o, (psi_o, _, infos_o) = timed(
            lambda: op.solve_origins(top, tol=tol, want_p=False), max(1, args.steps // 2), 1)
        assert all(i["status"] == 0 for i in infos_o), [i["status_name"] for i in infos_o][:5]
        po = [i["spmv_passes"] for i in infos_o]
        origins = dict(ms=round(ms_o, 3), origins=64, passes_max=int(max(po)),
                       origin_gteps=round(sum(po) * m / (ms_o * 1e-3) / 1e9, 1),
                       psi_rel_err_max=float(np.max(np.abs(psi_o.cpu().numpy() - psi64[top])
                                                    / psi64[top])))
        log(f"origins: 64 origins in {ms_o:.3f} ms, up to {max(po)} passes")

    head = min((p for p in modes
                if p not in ("fp64_weighted", "fp64_anderson", "mixed_anderson", "fp64_async")),
               key=lambda p: modes[p]["ms"])
    head_prec = head.replace("_warm", "")
    # the timed region of the reported value: K solves of the headline mode
    if head.endswith("_warm"):
        ms, (psi, info) = timed(lambda: op.solve(tol=tol, precision=head_prec,
                                                 s0=model.warmstart(op, s0_out=s0)),
                                args.steps, args.warmup)
    else:
        ms, (psi, info) = timed(lambda: op.solve(tol=tol, precision=head_prec), args.steps,
                                args.warmup)
    passes = info["spmv_passes"]
    value = passes * m / (ms * 1e-3) / 1e9
    log(f"headline {head}: {ms:.3f} ms/solve over {args.steps} solves, {value:.1f} GTEPS")

    # per-pass and dominant-kernel times, with HIP events on the stream the
    # kernels run on, in the tuned schedule of each precision
    mixed = head_prec == "mixed"
    form = api.SEG_FORM_NAMES[info["seg_form"]]
    segs = info["col_segments"]
    launch = {"step64": tuned["fp64"], "step64_w": tuned["fp64_weighted"], "step32": tuned["mixed"],
              "final64": tuned["fp64"]}
    pass_ms = {k: op.pass_time(k, reps=max(3, min(50, int(200 / max(modes["fp64"]["ms"] / 50, 0.01)))),
                               tile_items=v["tile_items"], col_segments=v["col_segments"],
                               seg_form=v["seg_form"])
               for k, v in launch.items()}
    kind = "step32" if mixed else "step64"
    reps = max(3, min(50, int(2000 / max(pass_ms[kind], 0.01))))
    if form == "bins":
        # the binned pass is two streaming launches and the small closing
        # kernel: its roofline is that of the whole pass (HIP events around
        # the three launches on their stream)
        dom = "bins32" if mixed else "bins64"
        kernel = (f"k_bins_expand<{'float' if mixed else 'double'}> + "
                  f"k_bins<{3 if mixed else 0}, 1280, 4> + k_band_fix<{3 if mixed else 0}>")
        dom_ms = pass_ms[kind]
        launches = 1
    elif form == "bands":
        dom = "band32" if mixed else "band64"
        kernel = f"k_band<{3 if mixed else 0}, {bands['rows']}, 4>"
        dom_ms = op.pass_time("part32" if mixed else "part64", reps=reps, seg_form="bands")
        launches = bands["bands"]
    elif segs > 1:
        dom = "part32" if mixed else "part64"
        kernel = (f"k_slices<{5 if mixed else 4}>" if form == "slices" else
                  f"k_pass_seg<{info['tile_items'] // 256}, {5 if mixed else 4}>")
        dom_ms = op.pass_time(dom, reps=reps, tile_items=info["tile_items"], col_segments=segs,
                              seg_form=info["seg_form"])
        launches = 1
    else:
        dom = kind
        kernel = f"k_pass<{info['tile_items'] // 256}, {3 if mixed else 0}>"
        dom_ms = pass_ms[kind]
        launches = 1
    pass_ms[dom if dom != kind else kind] = dom_ms
    alg_pass = algorithmic_bytes(kind, g.n, m)
    alg = alg_pass // launches  # the launch's share: its edges' indices, its users' vectors
    achieved = alg / (dom_ms * 1e-3) / 1e9
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(achieved / PEAK_HBM_GBS, 4),
                    traffic=traffic_from_profile(dom, name, kernel, alg),
                    kernel=kernel, algorithmic_bytes=alg, launches_per_pass=launches,
                    mean_launch_us=round(dom_ms * 1e3, 2),
                    pass_algorithmic_bytes=alg_pass, pass_us=round(pass_ms[kind] * 1e3, 2),
                    pass_achieved=round(alg_pass / (pass_ms[kind] * 1e-3) / 1e9, 1),
                    pass_frac=round(alg_pass / (pass_ms[kind] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                    gathers_per_s=round(m / (pass_ms[kind] * 1e-3) / 1e9, 1),
                    gather_unit="G random lines/s (per pass)")
    log(f"dominant kernel {kernel}: {dom_ms * 1e3:.1f} us per launch, {launches} per pass; "
        f"pass {pass_ms[kind] * 1e3:.1f} us")

    # the random-gather ceiling a pass is held to: the same gathers without arithmetic
    probe = api.gather_probe(g.n, m, col_segments=8 if g.n > 1_000_000 else max(1, segs), reps=5)
    roofline["gather_ceiling"] = dict(
        gathers_per_s=round(probe["gathers_per_s"] / 1e9, 1), unit="G random lines/s",
        frac=round(m / (pass_ms[kind] * 1e-3) / probe["gathers_per_s"], 4),
        probe=f"psi_gather_probe: {m} random 8-byte gathers, 4-byte indices streamed, into a "
              f"vector of {g.n} FP64 split in column segments by XCD group")

    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": DESCRIPTIONS[name], "name": name,
                   "n_users": g.n, "n_edges": m, "max_followers": st["max_followers"],
                   "tol": tol, "headline_mode": head, "layout": form,
                   "col_segments": info["col_segments"], "tile_items": info["tile_items"],
                   "band_layout": bands if form == "bands" else None,
                   "bins_layout": op.bins_info() if form == "bins" else None,
                   "parallelism": "single GPU"},
        "time_to_psi_ms": {p: round(v["ms"], 4) for p, v in modes.items()},
        "solves_timed": {p: (args.steps if p == head else cmp_k) for p in modes},
        "passes": {p: v["info"]["spmv_passes"] for p, v in modes.items()},
        "speedup_vs_plain_fp64": round(modes["fp64_weighted"]["ms"] / ms, 3),
        "speedup_vs_plain_fp64_by_mode": {p: round(modes["fp64_weighted"]["ms"] / v["ms"], 3)
                                          for p, v in modes.items()},
        "gteps_per_pass": {k: round(m / (v * 1e-3) / 1e9, 1) for k, v in pass_ms.items()
                           if not k.startswith(("band", "part", "bins"))},
        "pass_us": {k: round(v * 1e3, 2) for k, v in pass_ms.items()},
        "roofline": roofline,
        "warm_start": warm,
        "per_origin_shares": origins,
        "build_ms": round(builds[-1], 2),
        "autotune_ms": round(tune_ms, 1),
        "autotuned": {p: {k: v[k] for k in ("tile_items", "col_segments", "seg_form")}
                      for p, v in tuned.items()},
        "mixed_vs_fp64_rel_l1": float(np.abs(modes["mixed"]["psi"] - modes["fp64"]["psi"]).sum()
                                      / np.abs(modes["fp64"]["psi"]).sum()),
    }
    if not args.no_cpu_baseline:
        log("CPU oracle: building its operator from the raw edges")
        cb, psi_ref = cpu_baseline(g.n, f_host, l_host, g.lam, g.mu, tol)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline"]["value"] = round(cb["value"], 4)
        out["parity_vs_oracle"] = {
            p: dict(rel_l1=oracle.rel_l1(psi_ref, v["psi"]),
                    max_rel=oracle.max_rel(psi_ref, v["psi"]))
            for p, v in modes.items()}
        out["oracle_seconds"] = round(cb["seconds"], 2)
        log(f"CPU oracle: {cb['value']:.3f} GTEPS on {cb['cores']} threads")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


def run_batched(args, name):
    """cl_4m_k64 (scenario mode) or graphs256 (graph mode)."""
    import numpy as np
    import torch

    import synth
    from paper_2206_09960_amd import api

    tol = synth.WORKLOADS[name]["tol"]
    g = generate(name)
    f_dev = torch.as_tensor(g.follower).cuda()
    l_dev = torch.as_tensor(g.leader).cuda()
    t0 = time.perf_counter()
    op = api.Operator(g.n, f_dev, l_dev, torch.from_numpy(g.lam).cuda(),
                      torch.from_numpy(g.mu).cuda(), node_offsets=g.node_offsets)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    del f_dev, l_dev
    st = op.stats()
    m = st["n_edges"]
    log(f"operator built: M={m} in {build_ms:.1f} ms")
    if name == "cl_4m_k64":
        k = synth.WORKLOADS[name]["scenarios"]
        seed, sigma = synth.WORKLOADS[name]["seed"], synth.WORKLOADS[name]["sigma"]
        lam = np.empty((g.n, k))
        mu = np.empty((g.n, k))
        for s in range(k):
            lam[:, s], mu[:, s] = synth.activity(g.n, seed, "lognormal", sigma, scenario=s)
        lam_t, mu_t = torch.from_numpy(lam).cuda(), torch.from_numpy(mu).cuda()
        del lam, mu
        # the schedule of each precision, tuned first (scenarios per tile, items
        # per wave tile, hub chunk); its timing runs give one pass over all K
        t0 = time.perf_counter()
        tuned = {p: op.autotune_batched(k, p) for p in ("fp64", "mixed")}
        autotune_ms = (time.perf_counter() - t0) * 1e3
        log(f"autotuned: {tuned}")
        ms, (psi, infos) = timed(lambda: op.solve_batched(lam_t, mu_t, tol=tol), args.steps,
                                 args.warmup)
        units = k
        unit_name = "scenarios"
        # one scenario alone, for the speedup of batching: the faster of its
        # FP64 and mixed solves, each in the schedule the autotuner picks
        single = api.Operator(g.n, g.follower, g.leader, lam_t[:, 0].contiguous(),
                              mu_t[:, 0].contiguous())
        best1 = None
        for p in ("fp64", "mixed"):
            single.autotune(p)
            ms_p, (_, info_p) = timed(lambda: single.solve(tol=tol, precision=p),
                                      max(1, args.steps // 2), 1)
            if best1 is None or ms_p < best1[0]:
                best1 = (ms_p, info_p, p)
        ms1, info1, prec1 = best1
        ref = dict(single_solve_ms=round(ms1, 3), single_passes=info1["spmv_passes"],
                   single_precision=prec1,
                   single_layout=api.SEG_FORM_NAMES[info1["seg_form"]],
                   sequential_estimate_ms=round(ms1 * k, 2))
        del single
        # the same batch with FP32 corrections refined in FP64 (reported beside)
        solve_mixed = lambda: op.solve_batched(lam_t, mu_t, tol=tol, precision="mixed")  # noqa: E731
        ms_m, (psi_m, infos_m) = timed(solve_mixed, max(1, args.steps // 2), 1)
        assert all(i["status"] == 0 for i in infos_m), [i["status_name"] for i in infos_m][:5]
        ref["mixed"] = dict(ms=round(ms_m, 3),
                            fp64_passes_max=int(max(i["iterations"] for i in infos_m)),
                            fp32_passes_max=int(max(i["fp32_passes"] for i in infos_m)),
                            rel_l1_vs_fp64=float((psi_m - psi).abs().sum() / psi.abs().sum()))
        del psi_m
        # roofline of the pass that dominates each precision, over all K
        # scenarios (its rows, hub and gap kernels), from the tuner's HIP events
        roof = {}
        for p, kind in (("fp64", "scen64"), ("mixed", "scen32")):
            alg = batched_bytes(kind, g.n, m, k)
            pms = tuned[p]["pass_ms"]
            roof[p] = {"bound": "hbm", "achieved": round(alg / (pms * 1e-3) / 1e9, 1),
                       "peak": 8000.0, "unit": "GB/s",
                       "frac": round(alg / (pms * 1e-3) / 8e12, 4), "traffic": None,
                       "kernel": "scenario pass (k_spmm_rows + hub kernels + gap kernels)"
                       if p == "fp64" else "FP32 correction pass (same kernels, kScen32)",
                       "algorithmic_bytes": alg, "pass_ms": round(pms, 4),
                       "schedule": {x: tuned[p][x] for x in ("batch_tile", "batch_items",
                                                              "hub_chunk")}}
    else:
        t0 = time.perf_counter()
        tuned = {p: op.autotune_graphs(p, tol=tol) for p in ("fp64", "mixed")}
        autotune_ms = (time.perf_counter() - t0) * 1e3
        log(f"autotuned: {tuned}")
        ms, (psi, infos) = timed(lambda: op.solve_graphs(tol=tol), args.steps, args.warmup)
        units = len(infos)
        unit_name = "graphs"
        solve_mixed = lambda: op.solve_graphs(tol=tol, precision="mixed")  # noqa: E731
        ms_m, (psi_m, infos_m) = timed(solve_mixed, max(1, args.steps // 2), 1)
        assert all(i["status"] == 0 for i in infos_m), [i["status_name"] for i in infos_m][:5]
        ref = {"mixed": dict(ms=round(ms_m, 3),
                             fp64_passes_max=int(max(i["iterations"] for i in infos_m)),
                             fp32_passes_max=int(max(i["fp32_passes"] for i in infos_m)),
                             rel_l1_vs_fp64=float((psi_m - psi).abs().sum() / psi.abs().sum()))}
        del psi_m
        # roofline over the whole solve: each graph's passes move its own
        # compulsory bytes (4M_g + 44N_g per FP64 pass, 4M_g + 32N_g per FP32
        # pass, 4M_g + 36N_g for the final ψ), a frozen graph none; their sum
        # over the solve's time
        rp = op.views()["row_ptr"].cpu().numpy().astype(np.int64)
        m_g = rp[g.node_offsets[1:]] - rp[g.node_offsets[:-1]]
        n_g = np.diff(np.asarray(g.node_offsets, dtype=np.int64))
        roof = {}
        for p, t_ms, inf in (("fp64", ms, infos), ("mixed", ms_m, infos_m)):
            it = np.array([i["iterations"] for i in inf], dtype=np.int64)
            f32 = np.array([i["fp32_passes"] for i in inf], dtype=np.int64)
            alg = int(np.dot(it, 4 * m_g + 44 * n_g) + np.dot(f32, 4 * m_g + 32 * n_g)
                      + np.sum(4 * m_g + 36 * n_g))  # the final ψ pass
            roof[p] = {"bound": "hbm", "achieved": round(alg / (t_ms * 1e-3) / 1e9, 1),
                       "peak": 8000.0, "unit": "GB/s",
                       "frac": round(alg / (t_ms * 1e-3) / 8e12, 4), "traffic": None,
                       "kernel": "the whole batch solve (each live graph's passes)",
                       "algorithmic_bytes": alg, "solve_ms": round(t_ms, 3),
                       "schedule": {x: tuned[p][x] for x in ("tile_items", "col_segments",
                                                              "seg_form")}}
    assert all(i["status"] == 0 for i in infos), [i["status_name"] for i in infos][:5]
    # the headline is the faster precision, timed over --steps (the other one
    # stays in the reference block)
    headline = "fp64"
    if ms_m < ms:
        headline = "mixed"
        ref["fp64"] = dict(ms=round(ms, 3), passes_max=int(max(i["spmv_passes"] for i in infos)))
        ms, (_, infos) = timed(solve_mixed, args.steps, args.warmup)
        assert all(i["status"] == 0 for i in infos), [i["status_name"] for i in infos][:5]
        log(f"headline mixed: {ms:.3f} ms")
    other = "fp64" if headline == "mixed" else "mixed"
    roofline = dict(roof[headline], **{other: roof[other]})
    passes = [i["spmv_passes"] for i in infos]
    if name == "cl_4m_k64":
        edge_visits = sum(p * m for p in passes)
    else:
        # a graph stops at its own tolerance and is frozen: its edges count for its own passes
        rp = op.views()["row_ptr"].cpu().numpy().astype(np.int64)
        m_g = rp[g.node_offsets[1:]] - rp[g.node_offsets[:-1]]
        edge_visits = int(np.dot(m_g, np.asarray(passes, dtype=np.int64)))
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    out = {
        "metric": f"batched time-to-psi at tol 1e-8 over {units} {unit_name} (1 MI355X)",
        "value": round(edge_visits / (ms * 1e-3) / 1e9, 2),
        "unit": "GTEPS (edges x passes summed over the batch)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if headline == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": DESCRIPTIONS[name], "name": name, "n_users": g.n, "n_edges": m,
                   "units": units, "tol": tol, "headline_mode": headline,
                   "parallelism": "single GPU"},
        "passes": {"min": int(min(passes)), "max": int(max(passes)),
                   "mean": round(float(np.mean(passes)), 2)},
        "single_scenario_reference" if name == "cl_4m_k64" else "reference": ref,
        "roofline": roofline, "cpu_baseline": None, "build_ms": round(build_ms, 2),
        "autotune_ms": round(autotune_ms, 1), "autotuned": tuned,
    }
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD,
                    choices=list(SINGLE) + ["cl_4m_k64", "graphs256"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compare-steps", type=int, default=3,
                    help="solves timed per comparison mode on workloads above 2e8 edges")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm start mode")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design, not a build", file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    if args.workload in SINGLE:
        return run_single(args, args.workload)
    return run_batched(args, args.workload)


if __name__ == "__main__":
    sys.exit(main())
