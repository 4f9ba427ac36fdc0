"""Throughput of the fused collide-and-stream step on one MI355X.

Headline workload: D2Q9 modified MRT on the 4096^2 periodic cellular-flow
grid (rotated anisotropic D, 64 Gaussian hills), populations in FP32 shifted
storage.  One step = one collide-and-stream pass over all nodes; `value` is
million lattice updates per second with the populations resident in HBM.
The same line carries the other forms measured the same way: the plain FP64
and the FP16 split step on that grid, the D3Q15 256^3 step in FP64 and FP32,
the 64-channel Taylor-Aris ensemble advanced by the batched persistent
kernel, one adjoint gradient of the 512^2 inverse problem, the roofline of
the dominant kernel and the FP64 CPU oracle timed on the host cores.

Timing: after W warm-up steps each variant is timed in 5 blocks of at
least K steps (a multiple of the library's 32-step captured graph, and at
least 0.1 s), with HIP events on the stream the library launches on; the
median per-step time is reported with the minimum and maximum.  The tuned
variant of a run may take several steps per launch (LDS-blocked D2Q9); its
launch is timed on its own (5 blocks of 40 back-to-back launches, median)
for the roofline, whose bound is HBM (algorithmic bytes of a launch: the
state read and written once) or VALU (the algorithmic lane operations of the
launch's lattice updates against the VALU issue rate), whichever is nearer
its peak; the rate of all VALU instructions the launch issues (from the
committed instruction-count profile) is given beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only NAME]
                       [--quick] [--no-cpu] [--no-tune] [--copy-probe]
NAME: d2q9_4096_fp32 | d2q9_4096_fp64 | d2q9_4096_fp16 | d3q15_256_fp32 |
      d3q15_256_fp64 | taylor_aris_batch | unsteady | adjoint | adjoint_segment
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
# VALU issue rate without packed FP32 math (the library is built without it):
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane instructions per second
VALU_PEAK_TINSTR = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU lane operations of the method's own arithmetic per D2Q9 lattice update
# (an FMA counts once): the modified MRT collision with an equilibrium linear
# in phi and phi u (Eq. 31 and 37) in the add/sub-tree form of the step --
# phi and the population sums 9, the moments 22, their non-equilibrium parts
# 8, the relaxation increments S n / |M_k|^2 14, the back-transform f - M^T a
# 36 -- and the separable velocity's two products per component, 4
ALG_VALU_PER_LU_D2Q9 = 93
# algorithmic bytes per lattice update: Q populations read + Q written
BYTES_PER_LU = {("d2q9", "fp64"): 144, ("d2q9", "fp32"): 72, ("d2q9", "fp16"): 44,
                ("d3q15", "fp64"): 240, ("d3q15", "fp32"): 120}
COPY_PROBE_BYTES = 1 << 30     # bytes read (and written) by one calibration copy


def kernel_tag(launch):
    """Key of a launch variant in the committed counter profile: tile shape,
    rows per thread, streaming stores, block order (and the persistent grid
    of a batched launch, the steps per launch of a multi-step one)."""
    bx, by = launch["block"]
    tag = f"{bx}x{by}x{launch['rows_per_thread']}x{int(bool(launch['nt_stores']))}|order{launch['block_order']}"
    tag += f"|grid{launch['grid']}" if launch.get("grid") else ""
    return tag + (f"|steps{launch['steps_per_launch']}" if launch.get("steps_per_launch", 1) > 1 else "")


def kernel_name(launch, real):
    """The step kernel a launch variant of a D2Q9 run stepped alone runs."""
    T = launch.get("steps_per_launch", 1)
    if T == 1:
        return f"k_step_d2q9<{real}>"
    bx, by = launch["block"]
    return f"k_fused_d2q9<{real}, {bx}, {by}, {launch['rows_per_thread']}, {T}>"


def _profile(name, path="traffic.json"):
    """The committed PMC record of a workload, or None when its kernel
    sources differ from what the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", path)
    try:
        rec = json.load(open(path))[name]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec["source_files"]:
        h.update(open(os.path.join(ROOT, "paper_1404_2363_amd", "csrc", f), "rb").read())
    return rec if h.hexdigest()[:16] == rec["source_sha"] else None


def profiled_traffic(name, launch):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated on a 1 GiB
    copy) from the committed PMC profile of this kernel and launch variant,
    or None when the kernel source or the variant differs from what the
    counters were taken on."""
    rec = _profile(name)
    k = None if rec is None else rec["kernels"].get(kernel_tag(launch))
    return None if k is None else k["traffic_bytes_per_launch"]


def profiled_valu(name, launch):
    """VALU wave instructions per launch (SQ_INSTS_VALU) from the committed
    instruction-count profile of this kernel and launch variant, or None when
    the kernel source or the variant differs from what was counted."""
    rec = _profile(name, "valu.json")
    k = None if rec is None else rec["kernels"].get(kernel_tag(launch))
    return None if k is None else k["valu_wave_instr_per_launch"]


def roofline(v, name, real):
    """The roofline of a run's step kernel: the HBM one (algorithmic bytes of
    a launch over its measured duration) and the VALU one (the algorithmic
    lane operations of a launch, ALG_VALU_PER_LU_D2Q9 per lattice update, over
    the same duration, against the VALU issue rate); the bound is the one
    nearer its peak.  Where the kernel's VALU instruction count is profiled,
    "issued" gives the rate of all lane instructions the launch issues
    (recomputed halo rings and addressing included)."""
    launch = v["launch"]
    secs = v["ms_per_launch"] * 1e-3
    hbm = {"bound": "hbm", "achieved": v["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": v["hbm_frac"]}
    ops = ALG_VALU_PER_LU_D2Q9 * v["nodes"] * v["steps_per_launch"]
    t = ops / secs / 1e12
    alu = {"bound": "alu", "achieved": t, "peak": VALU_PEAK_TINSTR, "unit": "T VALU lane operations/s",
           "frac": t / VALU_PEAK_TINSTR, "algorithmic_lane_ops_per_launch": ops}
    valu = profiled_valu(name, launch)
    if valu is not None:
        ti = valu * 64 / secs / 1e12
        alu["issued"] = {"achieved": ti, "frac": ti / VALU_PEAK_TINSTR, "unit": "T VALU lane instructions/s",
                         "valu_wave_instructions_per_launch": valu}
    if alu["frac"] > hbm["frac"]:
        out = dict(alu)
        out["hbm"] = hbm
    else:
        out = dict(hbm)
        out["alu"] = alu
    out.update({"traffic": v.get("traffic"), "kernel": kernel_name(launch, real), "launch": launch,
                "bytes_per_launch": v["bytes_per_launch"], "ms_per_launch": v["ms_per_launch"],
                "steps_per_launch": v["steps_per_launch"]})
    return out


def profiled_segment_traffic(K, T=4):
    """HBM bytes of one FP32 adjoint checkpoint segment of K steps launched as
    segment_plan_bytes describes, from the per-kernel counters: multi-step
    forward and reverse launches (each averaged over its dispatches), the
    first reverse step, and the one-step launches of the left-over steps."""
    rec = _profile("adjoint_segment_2048_fp32")
    if rec is None:
        return None
    t = {k: v["traffic_bytes_per_launch"] for k, v in rec["kernels"].items()}
    out, k = 0.0, 0
    try:
        while k < K:
            if k + T <= K:
                out += t["forward_multi"]
                k += T
            else:
                out += t["forward_v"] if k + 1 < K else t["forward_v_last"]
                k += 1
        out += t["reverse_first"]
        k = K - 2
        while k >= 0:
            if k - T + 1 >= 0:
                out += t["reverse_multi_fold"] if k - T + 1 == 0 else t["reverse_multi"]
                k -= T
            else:
                out += t["reverse_last"] if k == 0 else t["reverse"]
                k -= 1
    except KeyError:
        return None
    return out


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


GRAPH_STEPS = 32               # steps per captured graph in the library
REPS = 5                       # timed blocks per variant (the median is reported)
MIN_BLOCK_S = 0.1              # each timed block lasts at least this long


def time_blocks(advance, steps, warmup):
    """Seconds per step of ``advance(n)`` (enqueues n steps on torch's
    current stream, the stream the library launches on): after ``warmup``
    steps, REPS blocks are timed with HIP events, each a multiple of the
    library's graph length (so long advances run as graph replays), at least
    ``steps`` steps and at least MIN_BLOCK_S long.  Returns the median, the
    minimum and maximum per-step time, the block length and the wall time."""
    import torch
    advance(max(warmup, 1))
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    advance(GRAPH_STEPS)           # a probe block sizes the timed ones
    ev[1].record()
    torch.cuda.synchronize()
    per = max(ev[0].elapsed_time(ev[1]) / 1e3 / GRAPH_STEPS, 1e-7)
    n = max(steps, int(MIN_BLOCK_S / per) + 1)
    n = -(-n // GRAPH_STEPS) * GRAPH_STEPS
    out = []
    t0 = time.perf_counter()
    for _ in range(REPS):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        advance(n)
        stop.record()
        torch.cuda.synchronize()
        out.append(start.elapsed_time(stop) / 1e3 / n)
    wall = time.perf_counter() - t0
    out.sort()
    return {"median": out[len(out) // 2], "min": out[0], "max": out[-1], "steps_per_block": n, "blocks": REPS,
            "wall_s": wall}


def time_launch(advance, steps_per_launch, per_block=40):
    """Average duration of one launch of a run's kernel: ``advance(T)`` with T
    the variant's steps per launch (below the graph length) enqueues exactly
    one launch; REPS blocks of ``per_block`` back-to-back launches are timed
    with HIP events on the library's stream and the median is returned."""
    import torch
    advance(steps_per_launch)
    torch.cuda.synchronize()
    out = []
    for _ in range(REPS):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(per_block):
            advance(steps_per_launch)
        stop.record()
        torch.cuda.synchronize()
        out.append(start.elapsed_time(stop) / 1e3 / per_block)
    return sorted(out)[len(out) // 2]


def check_against_default(s, default, steps=GRAPH_STEPS):
    """The tuned variant of a run stepped alone against its default variant
    (which the parity tests compare with the oracle at this grid size): from
    the same state, ``steps`` steps in each must give bitwise the same phi."""
    import torch
    tuned = s.variant()
    t0 = s.steps_done()
    ck = s.get_state()
    s.step(steps)
    a = s.phi()
    s.set_state(ck, t0)
    s.set_variant(default)
    s.step(steps)
    b = s.phi()
    same = bool(torch.equal(a, b))
    s.set_state(ck, t0)
    s.set_variant(tuned)
    return same


def gpu_variant(wl, precision, steps, warmup, tune=True):
    from paper_1404_2363_amd.solver import Solver
    s = Solver(wl, precision)
    default = s.variant()
    if tune:
        s.tune(10)
    tm = time_blocks(s.step, steps, warmup)
    var = s.variant()
    T = var.get("steps_per_launch", 1)
    t_launch = time_launch(s.step, T)
    nonfinite = s.nonfinite()
    same = check_against_default(s, default) if var != default else True
    s.close()
    t_step = tm["median"]
    # a launch reads and writes the state once, whatever its number of steps
    bpl = BYTES_PER_LU[(wl.lattice, precision)]
    gbs = wl.nodes * bpl / t_launch / 1e9
    return {"precision": precision, "nodes": wl.nodes, "ms_per_step": t_step * 1e3,
            "ms_per_step_min_max": [tm["min"] * 1e3, tm["max"] * 1e3], "timed_blocks": tm["blocks"],
            "steps_per_block": tm["steps_per_block"], "mlups": wl.nodes / t_step / 1e6,
            "steps_per_launch": T, "ms_per_launch": t_launch * 1e3, "bytes_per_launch": wl.nodes * bpl,
            "achieved_gbs": gbs, "bytes_per_lu": bpl / T, "hbm_frac": gbs / HBM_PEAK_GBS, "wall_s": tm["wall_s"],
            "nonfinite": nonfinite, "launch": var, "bitwise_equal_to_default_variant": same}


def batch_variant(runs, precision, steps, warmup, tune=True):
    """The Taylor-Aris ensemble: all channels in one batched launch (of one or
    several steps) per launch."""
    from paper_1404_2363_amd.solver import Solver
    per_run = [{"heat": [1 / r.meta["tau"]] * 2, "xref0": r.meta["x0"], "xref_drift": r.meta["U_node_mean"]}
               for r in runs]
    s = Solver(runs, precision, per_run=per_run)
    if tune:
        s.tune(10)
    tm = time_blocks(s.step, steps, warmup)
    nonfinite = sum(s.nonfinite(i) for i in range(len(runs)))
    var = s.variant()
    s.close()
    nodes = sum(r.nodes for r in runs)
    t_step = tm["median"]
    # the runs have no budget, so a timed 32-step block is 32 / T launches of
    # the (multi-step) batched kernel, each reading and writing every state once
    T = var.get("steps_per_launch", 1)
    bpl = BYTES_PER_LU[("d2q9", precision)]
    gbs = nodes * bpl / (T * t_step) / 1e9
    return {"precision": precision, "runs": len(runs), "nodes": nodes, "ms_per_step": t_step * 1e3,
            "ms_per_step_min_max": [tm["min"] * 1e3, tm["max"] * 1e3], "timed_blocks": tm["blocks"],
            "steps_per_block": tm["steps_per_block"], "mlups": nodes / t_step / 1e6,
            "steps_per_launch": T, "ms_per_launch": T * t_step * 1e3, "bytes_per_launch": nodes * bpl,
            "achieved_gbs": gbs, "bytes_per_lu": bpl / T, "hbm_frac": gbs / HBM_PEAK_GBS, "wall_s": tm["wall_s"],
            "nonfinite": nonfinite, "launch": var}


def unsteady_variant(precision, steps, warmup):
    """Time-dependent u on the 4096^2 grid: before every step a new velocity
    field (device FP64, already resident) replaces the run's field and the
    step reads it."""
    import torch
    from paper_1404_2363_amd import workloads as W
    from paper_1404_2363_amd.solver import Solver
    wl = W.drifting_cellular(nx=4096, ny=4096, steps=steps, n_hills=64, sigma=32.0, drift=0.5)
    fields = [torch.as_tensor(wl.u_schedule(n), dtype=torch.float64, device="cuda") for n in range(4)]
    s = Solver(wl, precision)
    count = [0]

    def advance(n):
        for _ in range(n):
            s.set_velocity(fields[count[0] % 4])
            s.step(1)
            count[0] += 1

    tm = time_blocks(advance, steps, warmup)
    nonfinite = s.nonfinite()
    s.close()
    t_step = tm["median"]
    bpl = BYTES_PER_LU[("d2q9", precision)] + 16               # populations + the FP64 field read by the step
    return {"precision": precision, "nodes": wl.nodes, "ms_per_step": t_step * 1e3,
            "ms_per_step_min_max": [tm["min"] * 1e3, tm["max"] * 1e3], "steps_per_block": tm["steps_per_block"],
            "mlups": wl.nodes / t_step / 1e6, "bytes_per_lu": bpl,
            "achieved_gbs": wl.nodes * bpl / t_step / 1e9, "hbm_frac": wl.nodes * bpl / t_step / 1e9 / HBM_PEAK_GBS,
            "nonfinite": nonfinite}


def adjoint_variant(precision="fp32"):
    """One gradient of the snapshot misfit for one initial condition of the
    512^2 inverse problem (2000 steps, snapshots every 200, checkpoints every
    100): forward, segment recomputation and reverse sweep."""
    import torch
    from paper_1404_2363_amd import workloads as W
    from paper_1404_2363_amd.adjoint import RolloutSpec, misfit
    inv = W.inverse_dfield()
    ic = inv["ics"][0]
    spec = RolloutSpec(ic, inv["steps"], inv["snap_every"], inv["ckpt_every"], precision, (1.0, 1.0))
    dev = "cuda:0"
    D = torch.tensor(inv["D_trial"], dtype=torch.float64, device=dev, requires_grad=True)
    p0 = torch.tensor(ic.phi0(), dtype=torch.float64, device=dev)
    obs = torch.zeros((inv["steps"] // inv["snap_every"],) + ic.grid, dtype=torch.float64, device=dev)
    misfit(D, p0, obs, spec).backward()          # warm-up (compiles graphs, allocator)
    D.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = misfit(D, p0, obs, spec)
    J.backward()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lu = ic.nodes * inv["steps"]
    return {"precision": precision, "nodes": ic.nodes, "steps": inv["steps"], "seconds_per_gradient": dt,
            "forward_lu_per_s_equiv": lu / dt / 1e6, "note": "MLUPS of forward steps per second of "
            "forward + recompute + reverse (3 passes)"}


def adjoint_all_ics_variant(precision="fp32"):
    """The gradient of the total misfit over all 10 initial conditions of the
    512^2 inverse problem, the rollouts run one after another (one autograd
    graph over ten rollouts) and side by side (misfit_many: a stream per
    condition).  One warm-up each, then one timed gradient each."""
    import torch
    from paper_1404_2363_amd import workloads as W
    from paper_1404_2363_amd.adjoint import RolloutSpec, misfit, misfit_many
    inv = W.inverse_dfield()
    dev = "cuda:0"
    specs = [RolloutSpec(ic, inv["steps"], inv["snap_every"], inv["ckpt_every"], precision, (1.0, 1.0))
             for ic in inv["ics"]]
    phi0s = [torch.tensor(ic.phi0(), dtype=torch.float64, device=dev) for ic in inv["ics"]]
    obs = [torch.zeros((inv["steps"] // inv["snap_every"],) + ic.grid, dtype=torch.float64, device=dev)
           for ic in inv["ics"]]
    D = torch.tensor(inv["D_trial"], dtype=torch.float64, device=dev, requires_grad=True)

    def sequential():
        return sum(misfit(D, p, o, sp) for p, o, sp in zip(phi0s, obs, specs))

    def side_by_side():
        return misfit_many(D, phi0s, obs, specs)

    out = {"precision": precision, "initial_conditions": len(specs), "nodes": specs[0].workload.nodes,
           "steps": inv["steps"]}
    for name, fn in (("sequential", sequential), ("side_by_side", side_by_side)):
        fn().backward()
        D.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn().backward()
        torch.cuda.synchronize()
        out[f"seconds_{name}"] = time.perf_counter() - t0
        D.grad = None
    out["speedup_side_by_side"] = out["seconds_sequential"] / out["seconds_side_by_side"]
    return out


def adjoint_segment_variant(n=2048, K=16, precision="fp32"):
    """One checkpoint segment of the adjoint on an n^2 grid with a per-node D
    field (FP32): K forward steps recomputed from the checkpoint, then K
    reverse steps, several per launch (segment_plan_bytes).  Algorithmic
    bytes per node of one step per launch: a recomputed step reads 36
    (populations) + 12 (per-node flux block A) and writes 36 (populations,
    not for the last step) + 8 (v); a reverse step gathers 36 (mu), reads 8
    (v) + 12 (A), writes 36 (mu) and moves the gradient: 12 (FP32 partial
    written, first reverse step), 24 (partial read and written), or 12 + 48
    (partial read, FP64 output read and written, last reverse step); the
    last segment step adds the 8-byte injection dL/dphi."""
    import torch
    from paper_1404_2363_amd import _lib as L
    from paper_1404_2363_amd import workloads as W
    from paper_1404_2363_amd.solver import Solver
    inv = W.inverse_dfield(n=n, n_ic=1, steps=K)
    ic = inv["ics"][0]
    D = torch.tensor(inv["D_trial"], dtype=torch.float64, device="cuda")
    import dataclasses
    wl = dataclasses.replace(ic, D_field=D)
    s = Solver(wl, precision, heat=[1.0, 1.0])
    nb = s.state_bytes()
    ck = s.get_state()
    mu = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    mu_tmp = torch.empty_like(mu)
    seg = torch.empty(L.lbm_cde_adjoint_scratch_bytes(s.h, 0, K), dtype=torch.uint8, device="cuda")
    grad = torch.zeros((3, n, n), dtype=torch.float64, device="cuda")
    g = torch.ones((n, n), dtype=torch.float64, device="cuda") * 1e-3
    inj = [None] * (K - 1) + [g.data_ptr()]
    L.lbm_cde_adjoint_segment(s.h, 0, ck.data_ptr(), K, seg.data_ptr(), inj, mu.data_ptr(), mu_tmp.data_ptr(),
                              grad.data_ptr())                      # warm-up
    torch.cuda.synchronize()
    per_block, times = 10, []
    for _ in range(REPS):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(per_block):
            L.lbm_cde_adjoint_segment(s.h, 0, ck.data_ptr(), K, seg.data_ptr(), inj, mu.data_ptr(),
                                      mu_tmp.data_ptr(), grad.data_ptr())
        stop.record()
        torch.cuda.synchronize()
        times.append(start.elapsed_time(stop) / 1e3 / per_block)
    t = sorted(times)[REPS // 2]
    finite = bool(torch.isfinite(grad).all())
    s.close()
    nodes = n * n
    one_step = (K - 1) * 92 + 56 + K * 92 + 12 + (K - 2) * 24 + 60 + 8
    plan = segment_plan_bytes(K, 4)
    byts = nodes * plan
    return {"precision": precision, "nodes": nodes, "segment_steps": K, "seconds_per_segment": t,
            "forward_plus_reverse_mlups": nodes * K / t / 1e6,
            "bytes_per_node": {"forward_step": 92, "reverse_step_first": 104, "reverse_step": 116,
                               "reverse_step_last": 152, "segment_one_step_per_launch": one_step,
                               "segment": plan},
            "steps_per_launch": 4, "achieved_gbs": byts / t / 1e9, "hbm_frac": byts / t / 1e9 / HBM_PEAK_GBS,
            "finite": finite}


def segment_plan_bytes(K, T):
    """Algorithmic bytes per node of one FP32 checkpoint segment as the
    library launches it on a periodic grid that spans its tiles: forward
    chunks of T steps from the checkpoint (state read 36 and, except at the
    segment's end, written 36, flux block 12, v 8 per step), the rest one step
    per launch (92, the last 56); the first reverse step one per launch (104 +
    the 8-byte injection), reverse chunks of T steps down to the start (mu 36
    + 36, v 8 per step, flux block 12, FP32 partial read and written 24, or
    partial read 12 and FP64 gradient read and written 48 for the chunk that
    ends at the segment's start), the left-over steps one per launch (116,
    the segment's first step 152)."""
    out, k = 0, 0
    while k < K:                                        # forward
        if k + T <= K:
            out += 36 + 12 + 8 * T + (36 if k + T < K else 0)
            k += T
        else:
            out += 92 if k + 1 < K else 56
            k += 1
    out += 104 + 8                                      # first reverse step, with the injection
    k = K - 2
    while k >= 0:                                       # reverse
        if k - T + 1 >= 0:
            out += 72 + 8 * T + 12 + (12 + 48 if k - T + 1 == 0 else 24)
            k -= T
        else:
            out += 152 if k == 0 else 116
            k -= 1
    return out


def copy_probe():
    """A plain device copy of known size, for calibrating HBM byte counters."""
    import torch
    n = COPY_PROBE_BYTES // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    torch.cuda.empty_cache()


def host_description():
    """Logical CPUs this process may use and the CPU model."""
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return ncpu, model


def cpu_baseline(wl, steps_all=40, steps_one=6):
    """The oracle's FP64 step on the same 4096^2 grid on the host: the C
    reference of the oracle (oracle/lbm_ref.c, plain C with OpenMP over rows,
    pinned to the numpy oracle), timed with one thread and with every
    available one (the box's share: OMP_NUM_THREADS when set), after one
    untimed step that touches both buffers."""
    from oracle import lbm as O
    from oracle import ref as R
    ncpu, model = host_description()
    nall = max(1, min(ncpu, int(os.environ.get("OMP_NUM_THREADS", ncpu))))
    t0 = time.perf_counter()
    prob = O.problem_for(wl)
    run = R.Run(prob, prob.equilibrium(wl.phi0()))
    run.advance(1, nall)
    log(f"cpu baseline: set-up {time.perf_counter() - t0:.1f} s")
    res = {}
    for threads, steps in ((1, steps_one), (nall, steps_all)):
        t0 = time.perf_counter()
        run.advance(steps, threads)
        res[threads] = (steps, time.perf_counter() - t0)
        log(f"cpu baseline: {steps} reference steps with {threads} thread(s): {res[threads][1]:.1f} s")
    best = max(res, key=lambda k: res[k][0] / res[k][1])
    steps, secs = res[best]
    return {"value": wl.nodes * steps / secs / 1e6, "unit": "MLUPS", "cores": best, "kind": "oracle",
            "sample": f"{steps} FP64 steps of the full {wl.shape[0]}x{wl.shape[1]} D2Q9 grid with the oracle's C "
                      f"reference (OpenMP over rows), {secs:.1f} s on {best} thread(s)",
            "host": {"cpus_available": ncpu, "threads_all": nall, "cpu_model": model},
            "by_threads": {str(k): {"mlups": wl.nodes * v[0] / v[1] / 1e6, "steps": v[0], "seconds": v[1]}
                           for k, v in res.items()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--only", default="")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline variant only")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1404_2363_amd import _lib
    from paper_1404_2363_amd import workloads as W
    _lib.load()
    torch.cuda.init()
    if args.copy_probe:
        copy_probe()
    tune = not args.no_tune
    wl2 = W.cellular()
    out = {}
    plan = [("d2q9_4096_fp32", wl2, "fp32", args.steps, args.warmup)]
    wl3 = None
    if (not args.only and not args.quick) or args.only.startswith("d3q15"):
        wl3 = W.sine3d()
    plan += [("d2q9_4096_fp64", wl2, "fp64", args.steps, args.warmup),
             ("d2q9_4096_fp16", wl2, "fp16", args.steps, args.warmup),
             ("d3q15_256_fp32", wl3, "fp32", args.steps, args.warmup),
             ("d3q15_256_fp64", wl3, "fp64", args.steps, args.warmup)]
    for name, wl, prec, k, w in plan:
        if args.only and name != args.only:
            continue
        if name != "d2q9_4096_fp32" and not args.only and args.quick:
            continue
        log(f"{name}: {k} steps")
        out[name] = gpu_variant(wl, prec, k, w, tune)
        out[name]["traffic"] = profiled_traffic(name, out[name]["launch"]) if prec != "fp64" else None
        log(f"{name}: {out[name]['mlups']:.0f} MLUPS, {out[name]['achieved_gbs']:.0f} GB/s")
    if (not args.only and not args.quick) or args.only == "taylor_aris_batch":
        runs = W.taylor_aris_batch()
        k = args.steps
        log(f"taylor_aris_batch: {len(runs)} channels, {k} steps")
        out["taylor_aris_batch_fp32"] = batch_variant(runs, "fp32", k, args.warmup, tune)
        out["taylor_aris_batch_fp32"]["traffic"] = profiled_traffic("taylor_aris_batch_fp32",
                                                                    out["taylor_aris_batch_fp32"]["launch"])
        log(f"taylor_aris_batch: {out['taylor_aris_batch_fp32']['mlups']:.0f} MLUPS")
    if (not args.only and not args.quick) or args.only == "unsteady":
        k = args.steps
        log(f"unsteady: 4096^2 FP32 with a new velocity field every step, {k} steps")
        out["d2q9_4096_fp32_unsteady_u"] = unsteady_variant("fp32", k, args.warmup)
        log(f"unsteady: {out['d2q9_4096_fp32_unsteady_u']['mlups']:.0f} MLUPS")
    if (not args.only and not args.quick) or args.only in ("adjoint", "adjoint_segment"):
        log("adjoint: one 2048^2 checkpoint segment of 16 steps (forward recompute + reverse)")
        out["adjoint_segment_2048_fp32"] = adjoint_segment_variant()
        seg = out["adjoint_segment_2048_fp32"]
        seg["traffic"] = profiled_segment_traffic(seg["segment_steps"])
        log(f"adjoint segment: {out['adjoint_segment_2048_fp32']['achieved_gbs']:.0f} GB/s")
    if (not args.only and not args.quick) or args.only == "adjoint":
        log("adjoint: one 512^2 x 2000-step gradient")
        out["inverse_adjoint_fp32"] = adjoint_variant("fp32")
        log(f"adjoint: {out['inverse_adjoint_fp32']['seconds_per_gradient']:.3f} s per gradient")
        log("adjoint: the gradient over all 10 initial conditions, sequential and side by side")
        out["inverse_adjoint_10ics_fp32"] = adjoint_all_ics_variant("fp32")
        a = out["inverse_adjoint_10ics_fp32"]
        log(f"adjoint 10 ICs: {a['seconds_sequential']:.3f} s sequential, {a['seconds_side_by_side']:.3f} s "
            f"side by side")
    if "d2q9_4096_fp32" not in out:
        out["d2q9_4096_fp32"] = gpu_variant(wl2, "fp32", args.steps, args.warmup, tune)
    main_v = out["d2q9_4096_fp32"]
    if "d2q9_4096_fp64" in out:
        out["speedup_fp32_over_fp64_d2q9"] = main_v["mlups"] / out["d2q9_4096_fp64"]["mlups"]
    if "d2q9_4096_fp16" in out and "d2q9_4096_fp64" in out:
        out["speedup_fp16_over_fp64_d2q9"] = out["d2q9_4096_fp16"]["mlups"] / out["d2q9_4096_fp64"]["mlups"]
    if "d3q15_256_fp64" in out:
        out["speedup_fp32_over_fp64_d3q15"] = out["d3q15_256_fp32"]["mlups"] / out["d3q15_256_fp64"]["mlups"]
    cpu = None if args.no_cpu else cpu_baseline(wl2)
    line = {
        "metric": "MLUPS, D2Q9 4096^2 modified MRT step, FP32 shifted storage",
        "value": main_v["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_v["ms_per_step"],
        "timing": {"statistic": "median", "blocks": main_v["timed_blocks"],
                   "steps_per_block": main_v["steps_per_block"],
                   "ms_per_step_min_max": main_v["ms_per_step_min_max"],
                   "note": "blocks are multiples of the 32-step captured graph, at least --steps steps and "
                           "at least 0.1 s long, timed with HIP events on the library's stream"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D2Q9 modified MRT, 4096x4096 periodic, cellular u (U0=0.05), D eigenvalues "
                               "0.01/0.1 rotated 30 deg, 64 Gaussian hills sigma=32, FP32 shifted storage",
                   "nodes": wl2.nodes},
        "roofline": roofline(main_v, "d2q9_4096_fp32", "float"),
        "variants": out,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
