#!/usr/bin/env python3
"""Throughput of the coupled phi / c lattice-Boltzmann step on one MI355X.

One "step" advances both distributions (phi-LBE and c-LBE) of every node by
one time step through the C ABI (gplbm_step).  The headline workload is the
3-D porous-medium dissolution on a 512^3 D3Q19 periodic grid (Gaussian random
field, correlation length 8, porosity 0.40, W = 2.5, counter term and
anti-trapping on) in FP64; inputs are generated on the host, copied to HBM and
initialised before the timed region.

Printed: one JSON line with MLUPS (million node updates per second), the
HBM roofline of the step kernel (algorithmic bytes per launch over the mean
launch time, measured with HIP events on the stream the library launches on),
the other forms of the same step beside it (FP32, FP16 and BF16 deviation
storage; h, or g and h, on the light lattice D3Q7 / D2Q5 in FP64, FP32 and FP16
deviations; the alternative
equilibrium h^eq,alt and general quadratic free energies in FP64), the
differentiation workload (adjoint / forward time), and the CPU oracle timed on
a bounded crop of the same workload.

    python bench.py [--steps K] [--warmup W] [--precision fp64|fp32|fp16dev|bf16dev]
                    [--h-lattice full|light|light-gh] [--h-scheme source|alt]
                    [--free-energy equal|quadratic] [--schedule auto|split|fused]
                    [--workload NAME] [--no-cpu-baseline] [--no-forms]
                    [--adjoint-steps K] [--variants]
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import statistics
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
LLC_BYTES = 256 << 20  # MI355X last-level (Infinity) cache
PROFILE_CMD = ""


def bytes_per_node_step(lattice_q: int, precision: str, lattice_qh: int | None = None) -> int:
    """Algorithmic bytes each node-step must move: read and write both
    distributions once (Q populations of g, Qh of h), and read and write the
    carried phi field (and, for the 16-bit deviation formats, the Lambda field
    their h references need)."""
    qh = lattice_q if lattice_qh is None else lattice_qh
    if precision in ("fp16dev", "bf16dev"):
        dist_g = (lattice_q - 1) * 2 + 4        # 16-bit moving + FP32 rest
        dist_h = (qh - 1) * 2 + 4
        return 2 * (dist_g + dist_h + 4 + 4)
    elem = 8 if precision == "fp64" else 4
    return (2 * lattice_q + 2 * qh + 2) * elem


def form_name(precision: str, h_lattice: str = "full", h_scheme: str = "source",
              free_energy: str = "equal") -> str:
    """Label of a form of the step: the precision, with '_light_h' when h
    runs on D3Q7 / D2Q5, '_light_gh' when g and h do, '_alt_h' with h^eq,alt,
    '_quadratic' with general quadratic free energies."""
    return (precision + {"full": "", "light": "_light_h", "light-gh": "_light_gh"}[h_lattice]
            + ("_alt_h" if h_scheme == "alt" else "")
            + ("_quadratic" if free_energy == "quadratic" else ""))


# general quadratic free energies for the workloads: eps_l / eps_s = 1.5,
# minima at the coexistence compositions of the equal-curvature parameters and
# df_min = 0, so that mu_eq = 0 and the coexistence compositions are unchanged
QUADRATIC = dict(free_energy=1, eps_s=1.0, eps_l=1.5)


def form_params(p, h_lattice="full", h_scheme="source", free_energy="equal"):
    q = dict(p, h_lattice=1 if h_lattice == "light" else 0,
             h_scheme=1 if h_scheme == "alt" else 0)
    if h_lattice == "light-gh":  # D2Q9 -> D2Q5, D3Q19 -> D3Q7
        q["lattice"] = p["lattice"] + 2
    if free_energy == "quadratic":
        q.update(QUADRATIC, m_s=p["c_s_co"], m_l=p["c_l_co"], df_min=0.0)
    return q


WORKLOADS = {
    "porous3d_512_d3q19": dict(kind="porous3d", n=512, steps=5000),
    "porous3d_256_d3q19": dict(kind="porous3d", n=256, steps=10000),
    "grain2d_1024_d2q9": dict(kind="grain2d", n=1024, steps=20000),
    "porous2d_512_d2q9": dict(kind="porous2d", n=512, steps=4000),
}


def make_workload(name):
    import workloads as wl
    w = WORKLOADS[name]
    if w["kind"] == "porous3d":
        p, phi0, c0 = wl.config_porous3d(w["n"])
    elif w["kind"] == "grain2d":
        p, phi0, c0, _ = wl.config1(n=w["n"])
    else:
        p, phi0, c0, _ = wl.config_porous2d(n=w["n"])
    return p, phi0, c0


def time_gpu(p, phi0, c0, precision, schedule, steps, warmup, log, h_lattice="full",
             h_scheme="source", free_energy="equal", ref_phi=None, keep_phi=False,
             repeats=1):
    """Times `steps` steps after `warmup` untimed ones.  ref_phi: phi of an
    FP64 run of the same form and step count (device), against which the
    final phi is compared; keep_phi: return this run's final phi as well;
    repeats > 1: time that many runs of `steps` steps in all (the extra ones
    after the comparison) and report each run's ms per step and the median."""
    import torch
    from paper_2111_05960_amd import Simulation

    p = form_params(p, h_lattice, h_scheme, free_energy)
    sim = Simulation(p, precision, schedule)
    sim.init(phi0, c0)
    torch.cuda.synchronize()
    d0 = sim.diagnostics(allow_nonfinite=True)
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    d1 = sim.diagnostics(allow_nonfinite=True)
    N = sim.N
    launches = 1 if sim.schedule == "fused" else 2
    balg = bytes_per_node_step(sim.Q, precision, sim.Qh)
    ms_step = ms / steps
    res = dict(
        mlups=N * steps / (ms * 1e-3) / 1e6, ms_per_step=ms_step, wall_s=wall,
        schedule=sim.schedule, launches_per_step=launches, nodes=N, Q=sim.Q, Qh=sim.Qh,
        bytes_per_node_step=balg,
        achieved_gbs=balg * N / (ms_step * 1e-3) / 1e9,
        mass_drift_rel=abs(d1["total_mass"] - d0["total_mass"]) / abs(d0["total_mass"]),
        nonfinite=d1["nonfinite"], solid_fraction=[d0["solid_fraction"], d1["solid_fraction"]],
    )
    log(f"gpu {form_name(precision, h_lattice, h_scheme, free_energy)} {sim.schedule}: "
        f"{res['mlups']:.1f} MLUPS, {ms_step:.3f} ms/step, "
        f"{res['achieved_gbs']:.0f} GB/s algorithmic, mass drift {res['mass_drift_rel']:.2e}")
    phi_end = None
    if ref_phi is not None or keep_phi:
        phi_end = sim.fields_device()[0]
    if ref_phi is not None:
        res["vs_fp64"] = {"phi_linf": float((phi_end - ref_phi).abs().max().item()),
                          "solid_fraction_diff": abs(d1["solid_fraction"] - float(
                              1.0 - ref_phi.mean().item())),
                          "steps": warmup + steps}
        log(f"  vs FP64 after {warmup + steps} steps: max|phi - phi_fp64| = "
            f"{res['vs_fp64']['phi_linf']:.2e}")
    if repeats > 1:
        runs = [ms_step]
        for _ in range(repeats - 1):
            e0.record(stream)
            sim.step(steps)
            e1.record(stream)
            torch.cuda.synchronize()
            runs.append(e0.elapsed_time(e1) / steps)
        res["runs_ms_per_step"] = runs
        res["median_ms_per_step"] = statistics.median(runs)
        log(f"  {repeats} runs of {steps} steps: " + ", ".join(f"{v:.3f}" for v in runs)
            + f" ms/step, median {res['median_ms_per_step']:.3f}")
    del sim
    if not keep_phi:
        phi_end = None
    torch.cuda.empty_cache()
    return (res, phi_end) if keep_phi else res


def adjoint_bytes_per_node(Q: int, D: int, precision: str) -> int:
    """Algorithmic HBM bytes of one reverse step (the two reverse kernels) per
    node: every array the step reads or writes, once.  Adjoint arrays are
    FP64; the forward states (H pulls and phi at n and n+1) are in the
    context's precision.
      first kernel:  reads  H^{n+1} (Q), phi^{n+1}, A1 and B2, B3 (D), B4 of the
                     previous step, the lambda accumulator;
                     writes A1 (Q), A2 (D), A3, A4, the lambda accumulator
      second kernel: reads  B1 of the previous step (Q), A3, A4, A2 (D),
                     H^n (Q), phi^n, phi^{n+1}, both accumulators;
                     writes B1 (Q), B2, B3 (D), B4, both accumulators
    A deviation-format state is read as Q - 1 16-bit codes, the FP32 rest
    population and the FP32 Lambda the decode needs per H read, FP32 phi."""
    adj_values = (Q + 1 + D + 1 + 1) + (Q + D + 1 + 1 + 1) \
        + (Q + 1 + 1 + D + 2) + (Q + 1 + D + 1 + 2)
    if precision in ("fp16dev", "bf16dev"):
        return 8 * adj_values + 2 * ((Q - 1) * 2 + 4 + 4) + 3 * 4
    fwd = 8 if precision == "fp64" else 4
    fwd_values = (Q + 1) + (Q + 1 + 1)
    return 8 * adj_values + fwd * fwd_values


def time_reverse_steps(n, precision, log, reps=200, dim=2):
    """Mean time of one reverse step (both reverse kernels) on the n^2 D2Q9
    porous workload (dim 2) or the n^3 D3Q19 one (dim 3), timed with HIP
    events on the stream the library launches on, between two saved states.
    The working set of a reverse step (adjoint state read and written, two
    forward states) is compared with the 256 MB last-level cache: where it
    fits, the rate is partly a cache rate."""
    import torch
    import workloads as wl
    from paper_2111_05960_amd import Simulation
    from paper_2111_05960_amd import binding as B

    if dim == 2:
        p, phi0, c0, _ = wl.config_porous2d(n=n)
    else:
        p, phi0, c0 = wl.config_porous3d(n)
    sim = Simulation(p, precision).init(phi0, c0)
    del phi0, c0
    s0, _ = sim.checkpoint()
    sim.step(1)
    s1, _ = sim.checkpoint()
    nb = B.gplbm_adjoint_bytes(sim.params)
    work = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    base = (work.data_ptr() + 255) // 256 * 256
    pb = torch.zeros(sim.N, dtype=torch.float64, device="cuda")
    B.gplbm_adjoint_begin(sim.ctx, base, nb, pb.data_ptr(), 0)
    for _ in range(10):
        B.gplbm_adjoint_step(sim.ctx, s0.data_ptr(), s1.data_ptr())
    stream = sim.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        B.gplbm_adjoint_step(sim.ctx, s0.data_ptr(), s1.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    balg = adjoint_bytes_per_node(sim.Q, dim, precision)
    working_set = balg * sim.N
    res = {"workload": f"porous{dim}d_{n}_{'d2q9' if dim == 2 else 'd3q19'}",
           "ms_per_reverse_step": round(ms, 5), "mlups": round(sim.N / (ms * 1e-3) / 1e6, 1),
           "bytes_per_node_step": balg,
           "achieved_gbs": round(balg * sim.N / (ms * 1e-3) / 1e9, 1),
           "hbm_frac": round(balg * sim.N / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "working_set_gb": round(working_set / 1e9, 3),
           "cache_resident": working_set <= LLC_BYTES}
    log(f"reverse step {res['workload']} {precision}: {ms:.4f} ms, {res['mlups']} MLUPS, "
        f"{res['achieved_gbs']} GB/s algorithmic ({balg} B/node), working set "
        f"{res['working_set_gb']} GB{' (cache-resident)' if res['cache_resident'] else ''}")
    del sim, work
    torch.cuda.empty_cache()
    return res


def time_adjoint(K, log, n=512, precision="fp64"):
    """Differentiation workload: 2-D porous medium n^2 (D2Q9, periodic), K
    steps (FP64, or FP32 / FP16-deviation forward states with the FP64
    reverse sweep);
    gradients of the final solid fraction with respect to lambda, D_l and
    phi0 through the hand-written adjoint with sqrt(K) checkpointing.
    Returns forward and backward wall times (the backward phase rebuilds each
    checkpoint segment and runs the reverse steps)."""
    import torch
    import workloads as wl
    from paper_2111_05960_amd import adjoint

    p, phi0, c0, _ = wl.config_porous2d(n=n)
    dev = torch.device("cuda")
    g_phi0 = torch.tensor(phi0, device=dev, requires_grad=True)
    c0_t = torch.tensor(c0, device=dev)
    g_lam = torch.tensor(p["lam"], dtype=torch.float64, requires_grad=True)
    g_dl = torch.tensor(p["D_l"], dtype=torch.float64, requires_grad=True)
    def warm_up():
        phiK, _ = adjoint.gplbm_run(g_phi0, c0_t, g_lam, g_dl, p, K, precision=precision)
        adjoint.objectives(g_phi0, phiK, p["W"])[0].backward()

    # untimed warm-up of both directions at the same length, so that the
    # allocator's pool holds the checkpoints and the segment's states (the
    # timed run then measures the steps, not first-touch allocations); its
    # graph and checkpoints are released before the peak memory is reset
    warm_up()
    gc.collect()
    g_phi0.grad = None
    g_lam.grad = None
    g_dl.grad = None
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base_mem = torch.cuda.memory_allocated()
    t0 = time.perf_counter()
    phiK, _ = adjoint.gplbm_run(g_phi0, c0_t, g_lam, g_dl, p, K, precision=precision)
    J1, J2 = adjoint.objectives(g_phi0, phiK, p["W"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J1.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    peak = torch.cuda.max_memory_allocated() - base_mem
    fwd, bwd = t1 - t0, t2 - t1
    res = {"workload": f"porous2d_{n}_d2q9", "K": K, "precision": precision,
           "checkpoint_every": int(math.ceil(math.sqrt(K))),
           "forward_s": round(fwd, 4), "backward_s": round(bwd, 4),
           "adjoint_forward_ratio": round(bwd / fwd, 3),
           "peak_memory_gb": round(peak / 1e9, 3),
           "forward_mlups": round(n * n * K / fwd / 1e6, 1),
           "backward_mlups": round(n * n * K / bwd / 1e6, 1),
           "J1": J1.item(), "dJ1_dlambda": g_lam.grad.item(), "dJ1_dDl": g_dl.grad.item(),
           "dJ1_dphi0_norm": float(g_phi0.grad.norm().item())}
    res["reverse_step"] = time_reverse_steps(n, precision, log)
    if precision == "fp64":
        # the same reverse kernels on a working set far beyond the last-level
        # cache (256^3 D3Q19, about 19 GB per reverse step): the HBM rate,
        # with the counted traffic of the committed rocprofv3 summary
        r = time_reverse_steps(256, precision, log, reps=20, dim=3)
        t = stored_traffic("porous3d_256_d3q19", precision, "reverse")
        r["traffic_gb_per_step"] = None if t is None else round(t["bytes_per_step"] / 1e9, 3)
        res["reverse_step_hbm"] = r
    log(f"adjoint {res['workload']} {precision} K={K}: forward {fwd:.3f} s, backward {bwd:.3f} s "
        f"(ratio {bwd / fwd:.2f}), peak {peak / 1e9:.2f} GB")
    return res


def kernel_source_hash() -> str:
    """Hash of the HIP sources with comments and layout removed: a stored
    traffic measurement is only used while the code it was taken on is
    unchanged."""
    import hashlib
    import re
    d = os.path.join(ROOT, "paper_2111_05960_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".h", ".hip")):
            with open(os.path.join(d, f)) as fh:
                src = fh.read()
            src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
            src = re.sub(r"//[^\n]*", " ", src)
            h.update(f.encode() + b"\0" + " ".join(src.split()).encode())
    return h.hexdigest()[:16]


def traffic_file(workload, precision, schedule):
    return os.path.join(ROOT, "profiles", f"step_{schedule}_{workload}_{precision}_traffic.json")


def stored_traffic(workload, precision, schedule):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, or None when there is none for the current kernel sources."""
    path = traffic_file(workload, precision, schedule)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t


def calibration_copy(log, gib=4):
    """A plain streaming kernel of known size (gib GiB read + gib GiB written,
    one elementwise negation) whose counter readings scale FETCH_SIZE and
    WRITE_SIZE to bytes."""
    import torch
    n = gib * (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    log(f"calibration stream: {gib} GiB read + {gib} GiB written")
    del a, b
    torch.cuda.empty_cache()


def stream_ceiling(log, gib=4, reps=10):
    """Rate of a plain read + write stream on this GPU, gib GiB in and gib GiB
    out, timed with HIP events over reps launches: the library's own copy
    kernel (gplbm_stream_copy: one 16-byte vector per thread, non-temporal
    stores) and, for reference, torch's FP64 negation.  The practical ceiling
    for a kernel that reads and writes in similar amounts, beside the 8 TB/s
    peak.  Returns (in-tree copy GB/s, torch negation GB/s)."""
    import torch
    from paper_2111_05960_amd import binding as B
    nbytes = gib << 30
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rates = []
    for kind in ("copy", "neg"):
        def once():
            if kind == "copy":
                B.gplbm_stream_copy(a.data_ptr(), b.data_ptr(), nbytes, stream.cuda_stream)
            else:
                torch.neg(a, out=b)
        once()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            once()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rates.append(round(2 * nbytes / (ms * 1e-3) / 1e9, 1))
        log(f"stream ceiling ({kind}): {rates[-1]:.0f} GB/s ({gib} GiB read + {gib} GiB "
            f"written, {ms:.3f} ms)")
    assert torch.equal(b, -a)  # the last launches negated a into b
    B.gplbm_stream_copy(a.data_ptr(), b.data_ptr(), nbytes, stream.cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(a, b), "gplbm_stream_copy did not copy"
    del a, b
    torch.cuda.empty_cache()
    return rates[0], rates[1]


def summarize_profile(kind, dbs, out, workload, precision, schedule):
    """Turn rocprofv3 database(s) into the text/JSON summaries kept under
    profiles/.  kind: 'trace' (kernel trace statistics) or 'traffic'
    (FETCH_SIZE and WRITE_SIZE runs, scaled by the calibration copy)."""
    import sqlite3

    def rows(db, sql):
        con = sqlite3.connect(db)
        try:
            return con.execute(sql).fetchall()
        finally:
            con.close()

    cmdline = " ".join(sys.argv)
    if kind == "trace":
        lines = [f"# rocprofv3 --kernel-trace --stats summary",
                 f"# profiled command: {PROFILE_CMD}", f"# summarised by: {cmdline}"]
        lines.append(f"{'calls':>6} {'avg_ms':>10} {'total_ms':>10} {'pct':>6}  kernel")
        # durations in the rocpd views are in microseconds
        for name, calls, total, avg, pct in rows(dbs[0], "select name, total_calls, total_duration, average, percentage from top_kernels"):
            lines.append(f"{calls:>6} {avg / 1e3:>10.3f} {total / 1e3:>10.3f} {pct:>6.2f}  {name}")
        with open(out, "w") as f:
            f.write("\n".join(lines) + "\n")
        return
    vals, sums = {}, {}
    for db in dbs:
        for kname, counter, n, avg, tot in rows(db, "select kernel_name, counter_name, count(*), avg(value), sum(value) from counters_collection group by kernel_name, counter_name"):
            vals[(kname, counter)] = (n, avg)
            sums[(kname, counter)] = tot
    # the step kernels, or in a reverse-step run the two reverse kernels (the
    # run also takes one forward step between its two saved states)
    step = [k for k in vals if any(t in k[0] for t in ("k_adj_ra", "k_adj_rb"))]
    if not step:
        step = [k for k in vals if any(t in k[0] for t in ("k_fused", "k_split", "k_dev_fused",
                                                            "k_dev_split"))]
    # the calibration is one 4 GiB negation (the only one in a profiled run:
    # --calibration-copy skips the stream-ceiling launches), which torch may
    # split into several dispatches: their counters are summed
    copy = [k for k in sums if "neg" in k[0].lower()]
    fetch_copy = sum(v for k, v in sums.items() if k in copy and k[1] == "FETCH_SIZE")
    write_copy = sum(v for k, v in sums.items() if k in copy and k[1] == "WRITE_SIZE")
    gib4_kib = 4 * (1 << 20)
    f_scale, w_scale = gib4_kib / fetch_copy, gib4_kib / write_copy
    res = {"source_hash": kernel_source_hash(), "workload": workload, "precision": precision,
           "schedule": schedule, "profiled_commands": PROFILE_CMD, "summarised_by": cmdline,
           "calibration": {"copy_bytes_each_way": 4 << 30, "FETCH_SIZE_kib": fetch_copy,
                           "WRITE_SIZE_kib": write_copy, "fetch_scale": f_scale,
                           "write_scale": w_scale},
           "kernels": {}}
    total = 0.0
    for kname in sorted({k[0] for k in step}):
        fk = vals.get((kname, "FETCH_SIZE"), (0, 0.0))[1]
        wk = vals.get((kname, "WRITE_SIZE"), (0, 0.0))[1]
        rd, wr = fk * 1024 * f_scale, wk * 1024 * w_scale
        res["kernels"][kname] = {"FETCH_SIZE_kib": fk, "WRITE_SIZE_kib": wk,
                                 "read_bytes": rd, "write_bytes": wr}
        total += rd + wr
    res["bytes_per_step"] = total
    with open(out, "w") as f:
        json.dump(res, f, indent=1)


def cpu_baseline(p, phi0, c0, log, budget_s=12.0):
    """The CPU oracle on a 128^3 (3-D) or 512^2 (2-D) crop of the same
    workload with zero-flux faces, stepped until about budget_s seconds."""
    import numpy as np
    import oracle
    import workloads as wl
    oracle.build(force=False)
    size = 128 if p["lattice"] in (wl.D3Q19, wl.D3Q7) else 512
    q, a, b = wl.crop_zero_flux(p, phi0, c0, min(size, p["shape"][-1]))
    o = oracle.Oracle(q).init(a, b)
    n_nodes = int(np.prod(q["shape"]))
    o.step(1)
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(2)
        steps += 2
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            break
    mlups = n_nodes * steps / dt / 1e6
    log(f"cpu oracle: {mlups:.2f} MLUPS on {oracle.threads()} threads ({steps} steps of {q['shape']})")
    single = cpu_single_thread(p, log)
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{steps} FP64 steps of the {'x'.join(map(str, q['shape'][::-1]))} crop "
                      f"[0,{q['shape'][-1]}) of the same workload, zero-flux faces, "
                      f"{dt:.1f} s wall",
            "cpu_model": cpu_model(), "single_thread": single}


_ORACLE_SAMPLE = """import sys, time
sys.path.insert(0, sys.argv[1])
import numpy as np
import bench, oracle, workloads as wl
name, budget = sys.argv[2], float(sys.argv[3])
p, phi0, c0 = bench.make_workload(name)
if p["lattice"] in (wl.D3Q19, wl.D3Q7):
    p, phi0, c0 = wl.crop_zero_flux(p, phi0, c0, 64)
oracle.build(force=False)
o = oracle.Oracle(p).init(phi0, c0)
o.step(1)
t0, k = time.perf_counter(), 0
while time.perf_counter() - t0 < budget:
    o.step(1)
    k += 1
print(np.prod(p["shape"]) * k / (time.perf_counter() - t0) / 1e6, oracle.threads(), k,
      "x".join(map(str, p["shape"][::-1])))
"""


def cpu_table(log, budget_s=5.0):
    """The FP64 oracle beside the FP64 GPU step on every workload: the GPU on
    the full grid, the oracle (child processes, all host threads and one) on
    the full 2-D grid or the 64^3 zero-flux crop of a 3-D one, each stepped
    for about budget_s seconds."""
    import subprocess
    rows = []
    for name in WORKLOADS:
        p, phi0, c0 = make_workload(name)
        g = time_gpu(p, phi0, c0, "fp64", "auto", 20, 5, log)
        del phi0, c0
        row = {"workload": name, "gpu_fp64_mlups": round(g["mlups"], 1),
               "gpu_schedule": g["schedule"]}
        for label, env in (("oracle", dict(os.environ)),
                           ("oracle_1thread", dict(os.environ, OMP_NUM_THREADS="1"))):
            out = subprocess.run([sys.executable, "-c", _ORACLE_SAMPLE, ROOT, name, str(budget_s)],
                                 env=env, capture_output=True, text=True, timeout=600, check=True)
            v, th, k, shape = out.stdout.split()[-4:]
            row[label] = {"mlups": round(float(v), 3), "threads": int(th), "steps": int(k),
                          "grid": shape}
        row["gpu_over_oracle"] = round(row["gpu_fp64_mlups"] / row["oracle"]["mlups"], 1)
        log(f"cpu table {name}: GPU {row['gpu_fp64_mlups']} MLUPS; oracle "
            f"{row['oracle']['mlups']} MLUPS on {row['oracle']['threads']} threads, "
            f"{row['oracle_1thread']['mlups']} on 1 ({row['oracle']['grid']})")
        rows.append(row)
    return rows


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"



def cpu_single_thread(p, log):
    """The oracle on one thread (OMP_NUM_THREADS=1, a child process), on a
    small random instance of the same lattice, about 3 s of stepping."""
    script = """import sys, time
sys.path.insert(0, sys.argv[1])
import numpy as np
import oracle, workloads as wl
lat, n = int(sys.argv[2]), int(sys.argv[3])
three = lat in (wl.D3Q19, wl.D3Q7)
shape = (n, n, n) if three else (1, n, n)
p = wl.base_params(lattice=lat, shape=shape, bc=(1, 1, 1 if three else 0))
phi0, c0 = wl.random_state_fields(shape, seed=1)
o = oracle.Oracle(p).init(phi0, c0)
o.step(1)
t0, k = time.perf_counter(), 0
while time.perf_counter() - t0 < 3.0:
    o.step(1)
    k += 1
print(np.prod(shape) * k / (time.perf_counter() - t0) / 1e6, oracle.threads())
"""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    three = p["lattice"] in (1, 3)
    n = 48 if three else 256
    try:
        out = subprocess.run([sys.executable, "-c", script, ROOT, str(p["lattice"]), str(n)],
                             env=env, capture_output=True, text=True, timeout=120, check=True)
        v, th = out.stdout.split()
    except (subprocess.SubprocessError, ValueError) as e:
        log(f"single-thread oracle timing failed: {e}")
        return None
    log(f"cpu oracle, 1 thread: {float(v):.2f} MLUPS")
    return {"value": round(float(v), 3), "unit": "MLUPS", "threads": int(th),
            "sample": f"{'x'.join([str(n)] * (3 if three else 2))} random fields, zero flux, ~3 s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="porous3d_512_d3q19", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "fp16dev", "bf16dev"])
    ap.add_argument("--h-lattice", default="full", choices=["full", "light", "light-gh"],
                    help="h on the lattice of g, h on D3Q7 / D2Q5, or g and h on D3Q7 / D2Q5")
    ap.add_argument("--h-scheme", default="source", choices=["source", "alt"],
                    help="source H_k, or h^eq,alt")
    ap.add_argument("--free-energy", default="equal", choices=["equal", "quadratic"],
                    help="equal curvatures, or general quadratic")
    ap.add_argument("--schedule", default="auto", choices=["auto", "split", "fused"])
    ap.add_argument("--bc", default="periodic", choices=["periodic", "walls"],
                    help="periodic grid, or zero flux on every face")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-table", action="store_true",
                    help="also time the FP64 oracle (all threads and one) beside the "
                         "FP64 GPU step on every workload")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip timing the other precision forms of the step")
    ap.add_argument("--variants", action="store_true",
                    help="also time the other precision and schedule")
    ap.add_argument("--adjoint-steps", type=int, default=4000,
                    help="K of the differentiation workload (0 skips it)")
    ap.add_argument("--reverse-only", action="store_true",
                    help="time only the reverse step on the 256^3 D3Q19 instance (--steps of "
                         "them) and exit: the command profiled for the reverse kernels")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="run a 4 GiB device copy after the timed region (counter calibration)")
    ap.add_argument("--summarize-profile", nargs="+", metavar="DB",
                    help="write a profiles/ summary from rocprofv3 database(s) and exit")
    ap.add_argument("--profile-kind", choices=["trace", "traffic"], default="trace")
    ap.add_argument("--out", default=None)
    ap.add_argument("--profile-cmd", default="", help="rocprofv3 command(s) recorded in a summary")
    args = ap.parse_args()

    if args.summarize_profile:
        global PROFILE_CMD
        PROFILE_CMD = args.profile_cmd
        summarize_profile(args.profile_kind, args.summarize_profile, args.out, args.workload,
                          form_name(args.precision, args.h_lattice, args.h_scheme,
                                    args.free_energy) + ("_walls" if args.bc == "walls" else ""),
                          args.schedule)
        return

    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the step runs on a single MI355X; there is no "
              "multi-GPU path (--gpus 1 only).", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.reverse_only:
        r = time_reverse_steps(256, args.precision, log, reps=args.steps, dim=3)
        if args.calibration_copy:
            calibration_copy(log)
        print(json.dumps(r), flush=True)
        return

    t0 = time.perf_counter()
    p, phi0, c0 = make_workload(args.workload)
    log(f"workload {args.workload} generated in {time.perf_counter() - t0:.1f} s")

    variant = (args.h_lattice, args.h_scheme, args.free_energy)
    main_form = form_name(args.precision, *variant) + ("_walls" if args.bc == "walls" else "")
    if args.bc == "walls":
        p = dict(p, bc=(1, 1, 1))
    keep = args.precision == "fp64" and not args.no_forms
    main_res = time_gpu(p, phi0, c0, args.precision, args.schedule, args.steps, args.warmup, log,
                        *variant, keep_phi=keep, repeats=3)
    ref_phi = None
    if keep:
        main_res, ref_phi = main_res
    # the other forms of the same step, side by side (auto schedule)
    forms = {}
    if not args.no_forms:
        precs = ("fp64", "fp32", "fp16dev", "bf16dev")
        todo = ([(prec, "full", "source", "equal") for prec in precs]
                + [("fp64", "light", "source", "equal"), ("fp32", "light", "source", "equal"),
                   ("fp16dev", "light", "source", "equal"),
                   ("fp64", "light-gh", "source", "equal"), ("fp32", "light-gh", "source", "equal"),
                   ("fp16dev", "light-gh", "source", "equal"),
                   ("fp64", "full", "alt", "equal"), ("fp64", "full", "source", "quadratic")])
        for prec, *var in todo:
            name = form_name(prec, *var)
            if name == main_form:
                continue
            # the precision forms of the main variant are compared with its FP64 phi
            same = tuple(var) == variant and prec in ("fp32", "fp16dev", "bf16dev")
            r = time_gpu(p, phi0, c0, prec, "auto", args.steps, args.warmup, log, *var,
                         ref_phi=ref_phi if same else None)
            t = stored_traffic(args.workload, name, r["schedule"])
            forms[name] = {
                "mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                "schedule": r["schedule"], "bytes_per_node_step": r["bytes_per_node_step"],
                "achieved_gbs": round(r["achieved_gbs"], 1),
                "hbm_frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                "traffic_gb_per_step": None if t is None else round(t["bytes_per_step"] / 1e9, 3),
                "mass_drift_rel": r["mass_drift_rel"]}
            if "vs_fp64" in r:
                forms[name]["vs_fp64"] = r["vs_fp64"]
        # the same grid with zero-flux faces (the porous case's boundary in
        # the paper): the walled instantiation of the z-march
        for prec in ("fp64", "fp32", "fp16dev"):
            name = form_name(prec) + "_walls"
            pw = dict(p, bc=(1, 1, 1))
            r = time_gpu(pw, phi0, c0, prec, "auto", args.steps, args.warmup, log)
            t = stored_traffic(args.workload, name, r["schedule"])
            forms[name] = {
                "mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                "schedule": r["schedule"], "bc": "zero flux on every face",
                "bytes_per_node_step": r["bytes_per_node_step"],
                "achieved_gbs": round(r["achieved_gbs"], 1),
                "hbm_frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                "traffic_gb_per_step": None if t is None else round(t["bytes_per_step"] / 1e9, 3),
                "mass_drift_rel": r["mass_drift_rel"]}
    ref_phi = None
    torch.cuda.empty_cache()
    variants = []
    if args.variants:
        precs = ("fp64", "fp32", "fp16dev", "bf16dev")
        for prec in precs:
            for sch in ("split", "auto"):
                if prec == args.precision and sch == args.schedule:
                    continue
                r = time_gpu(p, phi0, c0, prec, sch, args.steps, args.warmup, log)
                r["hbm_frac"] = round(r["achieved_gbs"] / HBM_PEAK_GBS, 4)
                variants.append(dict(precision=prec, **r))

    adj = None
    if args.adjoint_steps > 0:
        adj = time_adjoint(args.adjoint_steps, log)
        adj["fp32_forward"] = time_adjoint(args.adjoint_steps, log, precision="fp32")
        adj["fp16dev_forward"] = time_adjoint(args.adjoint_steps, log, precision="fp16dev")

    if args.calibration_copy:
        calibration_copy(log)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(form_params(p, *variant), phi0, c0, log)
    traffic = stored_traffic(args.workload, main_form, main_res["schedule"])
    # a profiled counter run (--calibration-copy) keeps its single calibration
    # negation: the stream-ceiling launches would be counted with it
    ceiling, ceiling_neg = (None, None) if args.calibration_copy else stream_ceiling(log)
    # rate of the bytes the step actually moves (the profiled counters), over
    # the stream ceiling measured here
    traffic_rate = None if traffic is None else \
        traffic["bytes_per_step"] / (main_res["ms_per_step"] * 1e-3) / 1e9

    nz, ny, nx = p["shape"]
    achieved = main_res["achieved_gbs"]
    # a step reads the state at n and writes the state at n+1: where both fit
    # in the 256 MB last-level cache the rate is partly a cache rate
    from paper_2111_05960_amd import binding as B
    working_set = 2 * B.gplbm_checkpoint_bytes(
        B.make_params(form_params(p, *variant), args.precision, args.schedule))
    line = {
        "metric": "MLUPS of coupled phi-mu LBM step + % HBM roofline; adjoint/forward cost ratio",
        "value": round(main_res["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        # the timed region above, then two more runs of as many steps
        "runs_ms_per_step": [round(v, 4) for v in main_res["runs_ms_per_step"]],
        "median_ms_per_step": round(main_res["median_ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16dev": "f16 storage / f32 math",
                  "bf16dev": "bf16 storage / f32 math"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "lattice": {(1, "light-gh"): "D3Q7", (0, "light-gh"): "D2Q5"}.get(
                (p["lattice"], args.h_lattice), "D3Q19" if p["lattice"] == 1 else "D2Q9"),
            "h_lattice": {(1, "full"): "D3Q19", (1, "light"): "D3Q7", (0, "full"): "D2Q9",
                          (0, "light"): "D2Q5", (1, "light-gh"): "D3Q7",
                          (0, "light-gh"): "D2Q5"}[(p["lattice"], args.h_lattice)],
            "h_scheme": args.h_scheme, "free_energy": args.free_energy,
            "grid": [nx, ny, nz],
            "bc": "periodic" if args.bc == "periodic" else "zero flux on every face",
            "precision": args.precision,
            "schedule": main_res["schedule"],
            "counter_term": p["counter_term"], "anti_trapping": p["anti_trapping"],
            "W": p["W"], "M_phi": p["M_phi"], "lambda": round(p["lam"], 6), "D_l": p["D_l"],
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic["bytes_per_step"] / 1e9, 3),
            "traffic_unit": "GB per step (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_gb_per_step": round(main_res["bytes_per_node_step"] * main_res["nodes"] / 1e9, 3),
            "kernel": "step (all launches of one time step)",
            "bytes_per_node_step": main_res["bytes_per_node_step"],
            "working_set_gb": round(working_set / 1e9, 3),
            "cache_resident": working_set <= LLC_BYTES,
            "launches_per_step": main_res["launches_per_step"],
            "stream_ceiling_gbs": ceiling,
            "stream_ceiling_kernel": "gplbm_stream_copy: 4 GiB read + 4 GiB written, one "
                                     "16-byte vector per thread, non-temporal stores",
            "stream_torch_neg_gbs": ceiling_neg,
            "traffic_rate_gbs": None if traffic_rate is None else round(traffic_rate, 1),
            "traffic_rate_frac_of_ceiling": None if traffic_rate is None or ceiling is None
            else round(traffic_rate / ceiling, 4),
        },
        "cpu_baseline": cpu,
        "checks": {"mass_drift_rel": main_res["mass_drift_rel"], "nonfinite": main_res["nonfinite"]},
        "context": {"paper_v100_mlups_2d_1024sq_d2q9": 149.8},
    }
    if forms:
        line["precision_forms"] = forms
    if adj is not None:
        line["adjoint"] = adj
    if variants:
        line["variants"] = variants
    if args.cpu_table:
        line["cpu_table"] = cpu_table(log)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
