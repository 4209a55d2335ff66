"""Benchmark: right-hand-side evaluations per second at 128^3 on one MI355X.

Workload: the closed-end hollow cylinder shield (R 10/8 mm, H 40 mm, cap
2 mm, 64^3 voxels in a 128^3 FFT box, n = 100, jc = 1e8 A/m^2, 0.05 T at
50 Hz, 45 degrees to the axis).  One step = one fixed-size Bogacki-Shampine
step of the device integrator (3 right-hand-side evaluations with 3 exterior
iterations each, stage combinations, FP64 error norm, accept) plus the
magnetic-moment readout of the accepted state; value = RHS evaluations per
second over the timed steps.  Inputs are seeded synthetic fields resident in
HBM before timing starts.

Beside the headline line: the right-hand side alone (FP64 and FP32), the
paper's stopping rule (delta_it = 2e-5) with its mean iteration count, and
the 256^3 lens box in FP32, whose working set exceeds the last-level cache.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time


ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FIXED_ITER = 3
T_STAR = 0.005            # s: quarter period of the 50 Hz drive (peak field)
DT_STEP = 1e-8            # s: fixed step of the timed integration


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rhs_passes_cup128_f64_hbm_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1803_01346_amd", "csrc", f)
                  for f in ("fft_core.h", "internal.h", "tuning.h", "passes.hip")]


def measured_traffic(kind):
    """HBM bytes per launch of `kind` from the committed counter summary, or
    None if the kernels changed since those counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    h = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)).hexdigest()[:16]
    if ("source_hash %s" % h) not in text:
        return None
    for line in text.splitlines():
        parts = line.split()
        if len(parts) == 3 and parts[0] == "traffic" and parts[1] == kind:
            return int(parts[2])
    return None


def make_sim(cfg, precision, fixed_iter):
    from paper_1803_01346_amd import scfft
    return scfft.Simulation(cfg, precision=precision,
                            rhs_opts=scfft.default_rhs_opts(fixed_iter=fixed_iter))


def initial_state(sim, cfg):
    import torch
    from paper_1803_01346_amd import scfft, workloads
    he, _ = scfft.scfft_drive_eval(sim.drive, sim.material, T_STAR)
    h = workloads.synthetic_state(cfg, seed=0, background=tuple(he))
    return torch.from_numpy(h).to(device="cuda", dtype=sim.dtype).contiguous(), h


def run_steps(sim, h, t0, k, with_moment=True):
    from paper_1803_01346_amd import scfft
    moments = []

    def obs(_u, t, _p):
        if with_moment:  # from the current density the step already formed
            moments.append(scfft.scfft_step_moment(sim.ctx))
        return 0

    st = scfft.OdeStats()
    o = scfft.default_ode_opts(fixed_steps=k)
    rc = scfft.scfft_integrate(sim.ctx, t0, t0 + k * DT_STEP, h, o, observer=obs, stats=st)
    return rc, st, moments


def time_rhs_only(sim, h, calls, warm=5):
    import torch
    hd = sim.empty_field()
    for _ in range(warm):
        sim.rhs_eval(T_STAR, h, hd)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(calls):
        sim.rhs_eval(T_STAR, h, hd)
    torch.cuda.synchronize()
    return calls / (time.perf_counter() - t), hd


def kernel_profile(sim, fn):
    """Per-kernel-kind launches, average duration and achieved GB/s of the
    algorithmic bytes, from HIP events the library attaches to each
    dispatch on its stream while fn() runs."""
    from paper_1803_01346_amd import scfft
    scfft.scfft_profile(sim.ctx, 1)
    fn()
    prof = scfft.scfft_profile_read(sim.ctx)
    scfft.scfft_profile(sim.ctx, 0)
    per_kind = {}
    for kind, (la, ms, by) in prof.items():
        if la:
            per_kind[kind] = dict(launches=la, avg_us=round(ms / la * 1e3, 2),
                                  bytes_per_launch=int(by / la),
                                  GBs=round(by / (ms * 1e-3) / 1e9, 1), total_ms=round(ms, 3))
    return per_kind


def roofline_of(per_kind, traffic=None, rhs=None):
    """The kernel with the largest total time against the HBM peak, the
    runner-up beside it (two kinds can be within a percent of each other, so
    either may lead from run to run), and the whole right-hand side."""
    order = sorted(per_kind, key=lambda k: -per_kind[k]["total_ms"])
    total = sum(v["total_ms"] for v in per_kind.values())

    def one(k):
        d = per_kind[k]
        return {"kernel": k, "achieved": d["GBs"], "frac": round(d["GBs"] / HBM_PEAK_GBS, 4),
                "bytes_per_launch": d["bytes_per_launch"], "avg_launch_us": d["avg_us"],
                "launches": d["launches"], "time_share": round(d["total_ms"] / total, 4),
                "traffic": traffic(k) if traffic else None}

    top = one(order[0])
    out = {"bound": "hbm", "kernel": top["kernel"], "achieved": top["achieved"], "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": top["frac"], "traffic": top["traffic"],
           "bytes_per_launch": top["bytes_per_launch"], "avg_launch_us": top["avg_launch_us"],
           "launches": top["launches"], "time_share": top["time_share"]}
    if len(order) > 1:
        out["runner_up"] = one(order[1])
    if rhs is not None:
        out["whole_rhs"] = rhs
    return out


def rhs_event_median(sim, h, hd, calls=100, warm=10):
    """Median duration (ms) of single rhs_eval calls, each bracketed by HIP
    events on the context's stream (torch's current stream here)."""
    import torch
    for _ in range(warm):
        sim.rhs_eval(T_STAR, h, hd)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
    for a, b in ev:
        a.record()
        sim.rhs_eval(T_STAR, h, hd)
        b.record()
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in ev)
    return ts[len(ts) // 2]


def rhs_bandwidth(sim, h, hd, rhs_ps, n, calls=10):
    """The whole right-hand side against the HBM peak: its bytes per call
    (the library's count for the launches of this schedule, and the counter
    bytes of the committed traffic summary per launch of each kernel kind
    when it matches the sources) times the calls per second of the timed
    run; beside it the byte model of a plain R2C pencil schedule,
    (3 + 2k) F + (17 + 16k) S + (2 + 2k) N^3 with F = 3 N^3 w and
    S = 3 N^2 (N/2 + 1) 2w, at the same rate."""
    pk = kernel_profile(sim, lambda: [sim.rhs_eval(T_STAR, h, hd) for _ in range(calls)])
    b = sum(v["bytes_per_launch"] * v["launches"] for v in pk.values()) / calls
    tr = {k: measured_traffic(k) for k in pk} if sim.dtype == __import__("torch").float64 else {}
    cb = (sum(tr[k] * pk[k]["launches"] for k in pk) / calls) if tr and all(v is not None for v in tr.values()) else None
    w, k = float(sim.dtype.itemsize), FIXED_ITER
    nodes = float(n[0] * n[1] * n[2])
    F = 3.0 * nodes * w
    S = 3.0 * n[2] * n[1] * (n[0] // 2 + 1) * 2.0 * w
    model = (3 + 2 * k) * F + (17 + 16 * k) * S + (2 + 2 * k) * nodes
    out = dict(bytes_per_rhs=int(b), rhs_per_s=round(rhs_ps, 2), achieved_GBs=round(b * rhs_ps / 1e9, 1),
               frac=round(b * rhs_ps / (HBM_PEAK_GBS * 1e9), 4),
               counter_bytes_per_rhs=int(cb) if cb is not None else None,
               counter_frac=round(cb * rhs_ps / (HBM_PEAK_GBS * 1e9), 4) if cb is not None else None,
               model_bytes_per_rhs=int(model),
               model_equivalent_frac=round(model * rhs_ps / (HBM_PEAK_GBS * 1e9), 4))
    return out


def converged_leg(cfg, h, calls=20):
    """rhs_eval with the paper's stopping rule (delta_it = 2e-5) instead of a
    fixed count, on consecutive stage times so each call starts from the
    previous call's exterior rate: calls per second and mean iterations."""
    import torch
    from paper_1803_01346_amd import scfft
    sim = scfft.Simulation(cfg, precision=scfft.F64)
    hd = sim.empty_field()
    st = scfft.RhsStats()
    for i in range(3):
        sim.rhs_eval(T_STAR - (3 - i) * DT_STEP, h, hd)
    torch.cuda.synchronize()
    iters = 0
    t = time.perf_counter()
    for i in range(calls):
        sim.rhs_eval(T_STAR + i * DT_STEP, h, hd, st)
        iters += st.iters
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    return dict(value=round(calls / el, 2), unit="RHS evals/s", mean_iters=round(iters / calls, 2),
                delta_it=2e-5, calls=calls)


def batch128_leg(calls=40):
    """Same-size batches of the 128^3 shield (one launch per pass over the
    members, instance = blockIdx.z; members differ in n and in their seeded
    states): 4 members in FP64, 6 in FP32.  Aggregate right-hand sides per
    second over `calls` back-to-back batched calls (3 exterior iterations)
    and the library's bytes of one batched call against the HBM peak."""
    import torch
    from paper_1803_01346_amd import scfft, workloads
    out = {}
    base = workloads.config("cup128")
    for prec, name, k in ((scfft.F64, "f64", 4), (scfft.F32, "f32", 6)):
        dt = torch.float64 if prec == scfft.F64 else torch.float32
        cfgs = [dict(base, n_power=base["n_power"] - 5 * i) for i in range(k)]
        b = scfft.Batch(cfgs, precision=prec, rhs_opts=scfft.default_rhs_opts(fixed_iter=FIXED_ITER))
        h = torch.stack([torch.from_numpy(workloads.synthetic_state(c, seed=i, background=(0.0, 0.0, 0.01)))
                         .to(dtype=dt) for i, c in enumerate(cfgs)]).cuda().contiguous()
        hd = b.empty_field()
        pk = kernel_profile(b.sims[0], lambda: b.rhs_eval(T_STAR, h, hd))
        nbytes = sum(v["bytes_per_launch"] * v["launches"] for v in pk.values())
        for _ in range(5):
            b.rhs_eval(T_STAR, h, hd)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(calls):
            b.rhs_eval(T_STAR, h, hd)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t) / calls
        out[name] = dict(instances=k, rhs_per_s=round(k / el, 1), bytes_per_batched_call=int(nbytes),
                         achieved_GBs=round(nbytes / el / 1e9, 1), frac=round(nbytes / el / (HBM_PEAK_GBS * 1e9), 4))
        b.close()
        del h, hd
        torch.cuda.empty_cache()
    return out


def lens256_leg(calls=30):
    """The 256^3 lens box in FP32 (working set beyond the 256 MB last-level
    cache: the HBM regime): RHS/s with 3 exterior iterations and the
    dominant kernel against the HBM peak."""
    import torch
    from paper_1803_01346_amd import scfft, workloads
    cfg = workloads.config("lens256")
    sim = make_sim(cfg, scfft.F32, FIXED_ITER)
    h = torch.from_numpy(workloads.synthetic_state(cfg, seed=0, background=(0.0, 0.0, 0.1))).to(
        device="cuda", dtype=torch.float32).contiguous()
    rate, hd = time_rhs_only(sim, h, calls, warm=3)
    per_kind = kernel_profile(sim, lambda: [sim.rhs_eval(T_STAR, h, hd) for _ in range(3)])
    whole = rhs_bandwidth(sim, h, hd, rate, cfg["n"], calls=3)
    out = dict(value=round(rate, 2), unit="RHS evals/s", dtype="f32", grid=[256, 256, 256],
               exterior_iters=FIXED_ITER, roofline=roofline_of(per_kind, None, whole), kernels=per_kind)
    sim.close()
    return out


def adjoint_leg(cfg, steps=2000, every=50):
    """Reverse-mode cost on the shield with a jc(x) map (kappa = 1 + 0.1 N(0,1),
    seed 5): 2000 fixed steps of 2e-5 s with checkpoints every 50 steps.  Time
    of the checkpointed adjoint giving the gradients in h0, the kappa map, n
    and the drive vector (forward with checkpoints, segment recomputation,
    reverse steps) over the time of the plain forward integration of the
    same steps."""
    import numpy as np
    import torch
    from paper_1803_01346_amd import autograd as sag, scfft
    sim = make_sim(cfg, scfft.F64, FIXED_ITER)
    n = cfg["n"]
    kap = 1.0 + 0.1 * np.random.default_rng(5).normal(size=(n[2], n[1], n[0]))
    dk = torch.from_numpy(kap).to(device="cuda").contiguous()
    scfft.scfft_set_jc_map(sim.ctx, dk)
    h0, _ = initial_state(sim, cfg)
    hT, h0b, ybar = sim.empty_field(), sim.empty_field(), torch.ones_like(h0)

    def fwd(k):
        h = h0.clone()
        scfft.scfft_reset_warm(sim.ctx)
        torch.cuda.synchronize()
        t = time.perf_counter()
        scfft.scfft_integrate(sim.ctx, 0.0, k * 2e-5, h, scfft.default_ode_opts(fixed_steps=k))
        torch.cuda.synchronize()
        return time.perf_counter() - t

    kbar = torch.zeros_like(dk)

    def adj(k, ev):
        ws = sag.adjoint_workspace(sim, k, ev)
        kbar.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        scfft.scfft_integrate_adjoint(sim.ctx, 0.0, k * 2e-5, k, ev, ws, h0, ybar, hT, h0b, kbar)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    fwd(10), adj(10, 5)                            # warm-up
    tf = fwd(steps)
    ta = adj(steps, every)
    out = dict(ratio=round(ta / tf, 3), forward_s=round(tf, 3), adjoint_s=round(ta, 3), steps=steps,
               checkpoint_every=every, dt_s=2e-5, dtype="f64",
               gradients="h0, kappa map, n, drive vector",
               note="ratio = (forward with checkpoints + recomputation + reverse) / forward")
    sim.close()
    return out


def graph_leg(count=64, steps=4):
    """Launch-bound and batched regimes, fixed steps (3 exterior iterations)
    replayed from captured graphs:
      cube32          one 32^3 cube: per-kernel launches vs graph replay;
      batch           the 64 mixed instances of workloads.batch_instances
                      (seed 4; box edges 48 to 192, cube / cylinder / cup,
                      n, jc and field directions drawn): each instance its
                      own context on its own stream (schedule autotuned),
                      against one batch per box edge whose members share
                      every launch (scfft_batch), the batches on their own
                      streams.  Aggregate right-hand sides per second
                      (1 + 3 steps per instance), also per box edge, and the
                      batched right-hand side's bytes against the HBM peak."""
    import gc

    import torch
    from paper_1803_01346_amd import scfft, workloads
    opts = lambda: scfft.default_rhs_opts(fixed_iter=FIXED_ITER)

    def per_instance(cl):
        sts = [torch.cuda.Stream() for _ in cl]
        sims = [scfft.Simulation(c, precision=scfft.F64, stream=st.cuda_stream, rhs_opts=opts())
                for c, st in zip(cl, sts)]
        hs = [workloads.synthetic_state_torch(c, seed=i) for i, c in enumerate(cl)]
        wss = [scfft.device_buffer(scfft.scfft_graph_workspace_size(s_.ctx, steps)) for s_ in sims]
        torch.cuda.synchronize()
        picks = [scfft.scfft_autotune(s_.ctx, h, calls=3)[0] for s_, h in zip(sims, hs)]

        def run():
            hh = [h.clone() for h in hs]
            torch.cuda.synchronize()
            t = time.perf_counter()
            for s_, h, ws in zip(sims, hh, wss):
                scfft.scfft_integrate_graph(s_.ctx, 0.0, 1e-3, steps, ws, h)
            for s_ in sims:
                scfft.scfft_integrate_wait(s_.ctx)
            torch.cuda.synchronize()
            return time.perf_counter() - t

        run()
        el = run()
        for s_ in sims:
            s_.close()
        return len(cl) * (1 + 3 * steps) / el, picks

    def batched(groups):
        bs = []
        for cl in groups:
            st = torch.cuda.Stream()
            b = scfft.Batch(cl, precision=scfft.F64, stream=st.cuda_stream, rhs_opts=opts())
            h = torch.stack([workloads.synthetic_state_torch(c, seed=i) for i, c in enumerate(cl)]).contiguous()
            bs.append((b, h, b.graph_workspace(steps)))
        torch.cuda.synchronize()

        def run():
            hh = [h.clone() for _, h, _ in bs]
            torch.cuda.synchronize()
            t = time.perf_counter()
            for (b, _, ws), h in zip(bs, hh):
                b.integrate_graph(0.0, 1e-3, steps, h, ws)
            for b, _, _ in bs:
                b.wait()
            torch.cuda.synchronize()
            return time.perf_counter() - t

        run()
        el = run()
        # bytes of one batched right-hand side (library count) and its rate, batch by batch
        nbytes, secs = 0.0, 0.0
        for b, h, _ in bs:
            pk = kernel_profile(b.sims[0], lambda: b.rhs_eval(0.2, h))
            nbytes += sum(v["bytes_per_launch"] * v["launches"] for v in pk.values())
            hd = b.empty_field()
            for _ in range(2):
                b.rhs_eval(0.2, h, hd)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(5):
                b.rhs_eval(0.2, h, hd)
            torch.cuda.synchronize()
            secs += (time.perf_counter() - t) / 5
        n = sum(len(cl) for cl in groups)
        for b, _, _ in bs:
            b.close()
        return n * (1 + 3 * steps) / el, dict(bytes_per_batched_rhs_all=int(nbytes),
                                               rhs_per_s=round(n / secs, 1),
                                               achieved_GBs=round(nbytes / secs / 1e9, 1),
                                               frac=round(nbytes / secs / (HBM_PEAK_GBS * 1e9), 4))

    out = dict(steps=steps, exterior_iters=FIXED_ITER, dtype="f64", unit="RHS evals/s")
    sims = [scfft.Simulation(workloads.config("cube32"), precision=scfft.F64, rhs_opts=opts())]
    h = workloads.synthetic_state_torch(workloads.config("cube32"), seed=0)
    ws = scfft.device_buffer(scfft.scfft_graph_workspace_size(sims[0].ctx, steps))
    pick = scfft.scfft_autotune(sims[0].ctx, h, calls=3)[0]

    def cube(graph):
        hh = h.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        if graph:
            scfft.scfft_integrate_graph(sims[0].ctx, 0.0, 1e-3, steps, ws, hh)
            scfft.scfft_integrate_wait(sims[0].ctx)
        else:
            scfft.scfft_integrate(sims[0].ctx, 0.0, 1e-3, hh, scfft.default_ode_opts(fixed_steps=steps))
        torch.cuda.synchronize()
        return (1 + 3 * steps) / (time.perf_counter() - t)

    cube(False), cube(True)
    out["cube32"] = dict(plain=round(cube(False), 1), graph=round(cube(True), 1), fuse_xy=pick)
    sims[0].close()

    cfgs = workloads.batch_instances(count)
    groups = {}
    for c in cfgs:
        groups.setdefault(c["n"][0], []).append(c)
    edges = sorted(groups)
    res = dict(instances=count, edges=edges, per_edge={str(e): len(groups[e]) for e in edges})
    t = time.perf_counter()
    rate, picks = per_instance(cfgs)
    res["per_instance_streams"] = round(rate, 1)
    res["fused_plane_picks"] = int(sum(x == 2 for x in picks))
    gc.collect()
    torch.cuda.empty_cache()
    rate, hbm = batched([groups[e] for e in edges])
    res["batched"] = round(rate, 1)
    res["batched_rhs_hbm"] = hbm
    gc.collect()
    torch.cuda.empty_cache()
    small = {}
    for e in edges:
        if e > 64:
            continue
        r_inst, _ = per_instance(groups[e])
        gc.collect()
        torch.cuda.empty_cache()
        r_b, _ = batched([groups[e]])
        gc.collect()
        torch.cuda.empty_cache()
        small[str(e)] = dict(instances=len(groups[e]), per_instance_streams=round(r_inst, 1),
                             batched=round(r_b, 1), gain=round(r_b / r_inst, 3))
    res["small_boxes"] = small
    res["wall_s"] = round(time.perf_counter() - t, 1)
    out["batch"] = res
    return out


def lens_gain_leg(n_grid=128, f32=False):
    """The lens of Sec. 3 as the paper runs it (n = 30, rho_out = 100, field
    along the axis h_e' = t', virgin start, adaptive steps and the stopping
    rule of the exterior iteration) on the slit-lens stand-in geometry
    (straight bore): the field-concentration factor, mean |B| over the
    central region {r <= 0.2, |z| <= 0.33} over the applied B, at h_e' = 0.05
    and 0.2 (the paper's biconical lens: about 2 and 1.6)."""
    import numpy as np
    import torch
    from paper_1803_01346_amd import scfft, workloads
    mu0 = 4e-7 * np.pi
    l, jc, e0 = 0.015, 5e8, 1e-4
    t0 = mu0 * jc * l * l / e0
    cfg = dict(n=(n_grid,) * 3, l_m=l, half_width=(2.0,) * 3, shapes=workloads.shape_lens(),
               n_power=30.0, jc=jc, e0=e0, rho_out=100.0,
               drive=dict(kind="ramp_hold", direction=(0.0, 0.0, 1.0), amp_T=0.2 * mu0 * jc * l,
                          t_ramp_s=0.2 * t0))
    s = scfft.Simulation(cfg, precision=scfft.F32 if f32 else scfft.F64)
    x = -2.0 + (np.arange(n_grid) + 0.5) * (4.0 / n_grid)
    r = np.sqrt(x[None, None, :] ** 2 + x[None, :, None] ** 2)
    region = torch.from_numpy(((r <= 0.2) & (np.abs(x)[:, None, None] <= 0.33)).astype(np.uint8)).cuda()
    h = s.empty_field()
    scfft.scfft_init_state(s.ctx, 0.0, h)
    out, t, steps, rhs = dict(dtype="f32" if f32 else "f64"), 0.0, 0, 0
    wall = time.perf_counter()
    for he in (0.05, 0.2):
        st = scfft.OdeStats()
        scfft.scfft_integrate(s.ctx, t, he * t0, h, scfft.default_ode_opts(), stats=st)
        out["gain_%.2f" % he] = round(scfft.scfft_region_mean_abs_b(s.ctx, h, region) / (he * mu0 * jc * l), 3)
        steps, rhs, t = steps + st.accepted, rhs + st.rhs_calls, he * t0
    out.update(steps=steps, rhs_calls=rhs, wall_s=round(time.perf_counter() - wall, 2))
    s.close()
    return out


def shield_config_leg(outputs=40):
    """The shield configuration run over its two periods (n = 100, jc = 1e8,
    0.05 T at 50 Hz and 45 degrees, virgin start, adaptive steps with the
    stopping rule) in FP64 and FP32: B on the bore axis (z = -1, 0, 1 cm)
    at evenly spaced output times, its largest magnitude relative to the
    applied amplitude, and the FP32 / FP64 difference of the probe
    histories."""
    import numpy as np
    import torch
    from paper_1803_01346_amd import scfft, workloads
    cfg = workloads.config("cup128")
    l = cfg["l_m"]
    pts = [[0.0, 0.0, -l], [0.0, 0.0, 0.0], [0.0, 0.0, l]]
    t_end = cfg["t_end_s"]
    res = {}
    out = dict(grid=list(cfg["n"]), outputs=outputs, probe_z_m=[p[2] for p in pts])
    for prec, name in ((scfft.F64, "f64"), (scfft.F32, "f32")):
        s = scfft.Simulation(cfg, precision=prec)
        h = s.empty_field()
        scfft.scfft_init_state(s.ctx, 0.0, h)
        hist, t, steps, rhs = [], 0.0, 0, 0
        torch.cuda.synchronize()
        wall = time.perf_counter()
        for k in range(1, outputs + 1):
            tt = t_end * k / outputs
            st = scfft.OdeStats()
            scfft.scfft_integrate(s.ctx, t, tt, h, scfft.default_ode_opts(), stats=st)
            hist.append(scfft.scfft_probe_b(s.ctx, h, pts))
            steps, rhs, t = steps + st.accepted, rhs + st.rhs_calls, tt
        torch.cuda.synchronize()
        res[name] = np.array(hist)
        mags = np.sqrt(np.sum(res[name] ** 2, axis=2))
        out[name] = dict(steps=steps, rhs_calls=rhs, wall_s=round(time.perf_counter() - wall, 2),
                         max_abs_B_over_applied=[round(float(v) / cfg["drive"]["amp_T"], 4)
                                                 for v in mags.max(axis=0)])
        s.close()
    d = res["f32"] - res["f64"]
    out["f32_vs_f64_rel_l2"] = float(np.sqrt(np.sum(d ** 2) / np.sum(res["f64"] ** 2)))
    return out


def lens_config_leg():
    """The slit lens of the 256^3 FP32 configuration run to the end of its
    field ramp (n = 50, jc = 2e8 A/m^2, rho_out = 100, 0 -> 1 T along the
    axis over 150 s, virgin start, adaptive steps with the stopping rule):
    the field-concentration factor at the bore centre, |B(0)| / B_applied,
    at 0.25, 0.5 and 1 T."""
    import torch
    from paper_1803_01346_amd import scfft, workloads
    cfg = workloads.config("lens256")
    s = scfft.Simulation(cfg, precision=scfft.F32)
    h = s.empty_field()
    scfft.scfft_init_state(s.ctx, 0.0, h)
    d = cfg["drive"]
    out, t, steps, rhs = dict(grid=list(cfg["n"]), dtype="f32", n_power=cfg["n_power"],
                              rho_out=cfg["rho_out"]), 0.0, 0, 0
    torch.cuda.synchronize()
    wall = time.perf_counter()
    for frac in (0.25, 0.5, 1.0):
        tt = frac * d["t_ramp_s"]
        st = scfft.OdeStats()
        scfft.scfft_integrate(s.ctx, t, tt, h, scfft.default_ode_opts(), stats=st)
        b = scfft.scfft_probe_b(s.ctx, h, [[0.0, 0.0, 0.0]])[0]
        out["factor_%gT" % (frac * d["amp_T"])] = round(float((b @ b) ** 0.5) / (frac * d["amp_T"]), 4)
        steps, rhs, t = steps + st.accepted, rhs + st.rhs_calls, tt
    torch.cuda.synchronize()
    out.update(steps=steps, rhs_calls=rhs, wall_s=round(time.perf_counter() - wall, 2))
    s.close()
    return out


def shield_leg(n_grid=128):
    """The shield run of Sec. 3 (cases A and B, n = 30, rho_out = 20, virgin
    start, adaptive steps, the stopping rule of the exterior iteration,
    FP64) on the stand-in cup: the mean |B| over the shielded zone over the
    applied |B| at the end of each field segment, steps and wall time (the
    paper's own 128^3 run took about 2 h in Matlab on a Core i5-2400)."""
    import numpy as np
    import torch
    from paper_1803_01346_amd import scfft, workloads
    out = dict(grid=[n_grid] * 3, dtype="f64", n_power=30.0, rho_out=20.0, tau=0.09,
               paper_wall_clock="about 2 h at 128^3 (Matlab R2017a, Intel Core i5-2400)")
    for case in ("A", "B"):
        cfg, t0, zone = workloads.shield_case(case, n_grid)
        s = scfft.Simulation(cfg, precision=scfft.F64)
        sh, ns = scfft.make_shapes([zone], cfg["l_m"])
        region = torch.from_numpy(scfft.scfft_voxelize_host(s.grid, s.material, sh, ns)).cuda()
        h = s.empty_field()
        scfft.scfft_init_state(s.ctx, 0.0, h)
        bs = workloads.MU0 * cfg["jc"] * cfg["l_m"]
        res, t, steps, rhs = {}, 0.0, 0, 0
        torch.cuda.synchronize()
        wall = time.perf_counter()
        for k, (tt, be) in enumerate(((0.09 * t0, 0.09 * bs), (0.18 * t0, 0.09 * bs * np.sqrt(2.0)))):
            st = scfft.OdeStats()
            scfft.scfft_integrate(s.ctx, t, tt, h, scfft.default_ode_opts(), stats=st)
            res["ratio_t%d" % (k + 1)] = round(scfft.scfft_region_mean_abs_b(s.ctx, h, region) / be, 4)
            steps, rhs, t = steps + st.accepted, rhs + st.rhs_calls, tt
        torch.cuda.synchronize()
        res.update(steps=steps, rhs_calls=rhs, wall_s=round(time.perf_counter() - wall, 2))
        out["case_" + case] = res
        s.close()
    return out


# A multi-core CPU right-hand side with scipy.fft, timed as context beside the
# oracle (never used by the GPU path).  It computes what the method computes
# (Sec. 2): j = C_s h (Eq. 4, smoothed spectral curl), e from the power law
# (Eq. 1) in Omega and rho_out j outside, hdot_in = -C_s e on Omega (Eq. 3),
# then a fixed number of exterior iterations (Eq. 5) with Phi of Eq. 7
# (1/|k|^2 := 0 at k = 0), from the Ohm-law start or the previous call's
# exterior rate.  Real-to-complex transforms run on `workers` threads; k_odd
# has 0 on the Nyquist index of each axis, |k|^2 and the smoothing use the
# true k.  Uniform jc (kappa = 1), isotropic law.
import numpy as np  # noqa: E402


class ScipyRhs:
    def __init__(self, n, half_width, chi, n_power, rho_out, fixed_iter, workers=None):
        import os

        import scipy.fft as sf
        self.sf = sf
        self.workers = workers or os.cpu_count() or 1
        nx, ny, nz = (int(v) for v in n)
        L = [float(v) for v in half_width]
        h = [2.0 * L[a] / n[a] for a in range(3)]
        sigma = 0.5 * np.sqrt(h[0] ** 2 + h[1] ** 2 + h[2] ** 2)

        def axis(a, half):
            N = (nx, ny, nz)[a]
            m = np.arange(N // 2 + 1) if half else np.where(np.arange(N) < N // 2, np.arange(N), np.arange(N) - N)
            k = np.pi * m / L[a]
            ko = k.copy()
            ko[np.abs(m) == N // 2] = 0.0
            return k, ko

        kx, kxo = axis(0, True)
        ky, kyo = axis(1, False)
        kz, kzo = axis(2, False)
        sh = (nz, ny, nx // 2 + 1)
        self.kx, self.ky, self.kz = (np.broadcast_to(kxo[None, None, :], sh),
                                     np.broadcast_to(kyo[None, :, None], sh),
                                     np.broadcast_to(kzo[:, None, None], sh))
        k2 = kx[None, None, :] ** 2 + ky[None, :, None] ** 2 + kz[:, None, None] ** 2
        self.smooth = np.exp(-0.5 * sigma ** 2 * k2)
        inv = np.zeros_like(k2)
        inv[k2 > 0] = 1.0 / k2[k2 > 0]
        self.inv_k2 = inv
        self.chi = np.asarray(chi) != 0
        self.out = ~self.chi
        self.n_power = float(n_power)
        self.rho_out = float(rho_out)
        self.fixed_iter = int(fixed_iter)
        self.shape = (nz, ny, nx)
        self.warm = None

    def _apply(self, v, mult):
        """Re F^-1 { mult * i k_odd x F(v) } with real-to-complex transforms."""
        sf = self.sf
        V = sf.rfftn(v, axes=(1, 2, 3), workers=self.workers)
        kx, ky, kz = self.kx, self.ky, self.kz
        c = np.stack([ky * V[2] - kz * V[1], kz * V[0] - kx * V[2], kx * V[1] - ky * V[0]])
        c *= 1j * mult
        return sf.irfftn(c, s=self.shape, axes=(1, 2, 3), workers=self.workers)

    def curl(self, v):
        return self._apply(v, self.smooth)

    def phi(self, v):
        return self._apply(v, self.inv_k2)

    def __call__(self, hedot, h):
        j = self.curl(h)
        s = np.sum(j * j, axis=0)
        with np.errstate(divide="ignore", invalid="ignore"):
            f = np.where(s > 0.0, s ** (0.5 * (self.n_power - 1.0)), 0.0)
        e = np.where(self.chi, f * j, self.rho_out * j)
        g = -self.curl(e)
        hdot_in = g * self.chi
        hdot = hdot_in + (self.warm if self.warm is not None else g) * self.out
        he = np.asarray(hedot, dtype=np.float64).reshape(3, 1, 1, 1)
        for _ in range(self.fixed_iter):
            jd = self.curl(hdot) * self.chi
            hdot = hdot_in + self.out * (he + self.phi(jd))
        self.warm = hdot * self.out
        return hdot


def host_cpu():
    """CPU model and the threads this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(model=model, nproc=usable, logical_cpus=os.cpu_count())


def cpu_baseline(cfg, h_np, calls=3):
    """The oracle's rhs_eval (plain NumPy FP64, its own radix-2 FFT) on the
    same 128^3 state with 3 exterior iterations: median of `calls` full
    calls, BLAS and OpenMP pools held to one thread (NumPy's elementwise work
    is single-threaded); the same protocol on the 32^3 cube and the 64^3 cup
    beside it.  Also, as context, the multi-core scipy.fft right-hand side
    (ScipyRhs) on all usable threads, median of 3."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import geometry, grid, rhs, units
    from paper_1803_01346_amd import workloads

    def problem(c):
        g = grid.Grid(c["n"], c["half_width"])
        chi = geometry.voxelize(g, c["shapes"])
        u = units.Units(c["jc"], c["l_m"])
        d = dict(c["drive"])
        drive = units.Drive(u, d.pop("kind"), **d)
        return rhs.Problem(g, chi, c["n_power"], c["rho_out"], drive, rhs.RhsOptions(fixed_iter=FIXED_ITER)), u, g, chi, drive

    def median_calls(prob, t, h):
        ts = []
        with threadpool_limits(1):
            for _ in range(calls):
                t0 = time.perf_counter()
                rhs.rhs_eval(prob, t, h)
                ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), ts

    # the smaller boxes of the same protocol: the 32^3 cube and the 64^3 cup
    smaller = {}
    for name in ("cube32", "cup64"):
        c = workloads.config(name)
        pr, uu, _, _, _ = problem(c)
        m, _ = median_calls(pr, T_STAR / uu.t0, workloads.synthetic_state(c, seed=0))
        smaller["%d^3" % c["n"][0]] = dict(workload=name, rhs_per_s=round(1.0 / m, 3), median_s=round(m, 3))
    prob, u, g, chi, drive = problem(cfg)
    med, ts = median_calls(prob, T_STAR / u.t0, h_np)
    print("bench: oracle calls %s s" % ", ".join("%.1f" % x for x in ts), file=sys.stderr, flush=True)
    host = host_cpu()
    f = ScipyRhs(cfg["n"], cfg["half_width"], chi, cfg["n_power"], cfg["rho_out"], FIXED_ITER,
                 workers=host["nproc"])
    hedot = drive.hedot(T_STAR / u.t0)
    f(hedot, h_np)                                   # warm-up (plans, warm start)
    tq = []
    for _ in range(3):
        t = time.perf_counter()
        f(hedot, h_np)
        tq.append(time.perf_counter() - t)
    return dict(value=round(1.0 / med, 5), unit="RHS evals/s", cores=1, kind="oracle",
                sample="the oracle's rhs_eval at 128^3 (cup shield, FP64, 3 exterior iterations, own "
                       "radix-2 FFT), median of %d full calls (%s s), one thread"
                       % (calls, ", ".join("%.1f" % x for x in ts)),
                host_cpu=host["model"], host_nproc=host["nproc"], smaller_boxes=smaller,
                context_scipy_fft=dict(value=round(1.0 / float(np.median(tq)), 4), unit="RHS evals/s",
                                       workers=host["nproc"], kind="scipy.fft rfftn/irfftn, FP64",
                                       sample="median of 3 calls at 128^3 after one warm-up call"))


def copy_calibration(nbytes=256 << 20, reps=5):
    """A plain device-to-device copy of known size: reads and writes nbytes per
    launch.  Used to scale the FETCH_SIZE / WRITE_SIZE counters and, at sizes
    beyond the 256 MB last-level cache, as the achievable-bandwidth anchor
    (timed with HIP events on the current stream)."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        b.copy_(a)
        e1.record()
    torch.cuda.synchronize()
    ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev)[reps // 2]
    print(json.dumps({"copy_calibration_bytes_per_launch": nbytes, "launches": 2 * reps, "timed_launches": reps,
                      "median_ms": round(ms, 4), "read_plus_write_GBs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}))


def profile_leg(leg, cfg, calls=20, warm_s=0.5):
    """A few right-hand sides of one leg only, for a kernel trace or counter
    run under rocprofv3 (f64 / f32: the 128^3 shield; lens: the 256^3 lens)."""
    import torch
    from paper_1803_01346_amd import scfft, workloads
    if leg == "lens":
        cfg = workloads.config("lens256")
        sim = make_sim(cfg, scfft.F32, FIXED_ITER)
        h = torch.from_numpy(workloads.synthetic_state(cfg, seed=0, background=(0.0, 0.0, 0.1))).to(
            device="cuda", dtype=torch.float32).contiguous()
        t = 10.0
    else:
        sim = make_sim(cfg, scfft.F64 if leg == "f64" else scfft.F32, FIXED_ITER)
        h, _ = initial_state(sim, cfg)
        t = T_STAR
    hd = sim.empty_field()
    # warm_s seconds of the same calls first (clocks and caches settle; a
    # kernel trace leaves them out), then the `calls` calls a summary keeps
    warm = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < warm_s:
        for _ in range(10):
            sim.rhs_eval(t, h, hd)
        torch.cuda.synchronize()
        warm += 10
    for _ in range(calls):
        sim.rhs_eval(t, h, hd)
    torch.cuda.synchronize()
    # one more call with the library's per-dispatch events: its byte model per
    # launch of each kind, which the counter summaries divide the HBM bytes by
    pk = kernel_profile(sim, lambda: sim.rhs_eval(t, h, hd))
    print(json.dumps({"profile_leg": leg, "warm_calls": warm, "rhs_calls": calls + 1,
                      "bytes_per_launch": {k: v["bytes_per_launch"] for k, v in pk.items()},
                      "launches_per_call": {k: v["launches"] for k, v in pk.items()}}))


def timed_steps(sim, h, steps, warmup):
    import torch
    run_steps(sim, h, T_STAR, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st, moments = run_steps(sim, h, T_STAR + warmup * DT_STEP, steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if rc < 0 or st.accepted != steps:
        raise RuntimeError("timed integration failed: rc=%d accepted=%d" % (rc, st.accepted))
    return st, elapsed


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="cup128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-events", action="store_true", help="skip the per-kernel event timing runs")
    ap.add_argument("--no-converged", action="store_true", help="skip the delta_it stopping-rule leg")
    ap.add_argument("--no-lens", action="store_true", help="skip the 256^3 FP32 lens leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the reverse-mode cost leg")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay / batch leg")
    ap.add_argument("--extras", action="store_true",
                    help="also run the paper's shield and lens runs (lens gain, shield cases, "
                         "two-period shield, 256^3 lens ramp)")
    ap.add_argument("--profile-warm", type=float, default=0.5,
                    help="seconds of right-hand sides before the profiled ones (0 for counter runs)")
    ap.add_argument("--profile-leg", choices=["f64", "f32", "lens"],
                    help="only run a few right-hand sides of one leg (for rocprofv3)")
    ap.add_argument("--copy-calibration", type=int, nargs="?", const=256 << 20, default=None,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the method here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); rerun with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration is not None:
        copy_calibration(args.copy_calibration)
        return

    import torch
    from paper_1803_01346_amd import scfft, workloads
    scfft.load()
    torch.cuda.set_device(0)
    cfg = workloads.config(args.config)
    if args.profile_leg:
        profile_leg(args.profile_leg, cfg, warm_s=args.profile_warm)
        return

    sim = make_sim(cfg, scfft.F64, FIXED_ITER)
    h, h_np = initial_state(sim, cfg)
    print("bench: %s FP64, warmup %d steps" % (args.config, args.warmup), file=sys.stderr, flush=True)
    st, elapsed = timed_steps(sim, h, args.steps, args.warmup)
    value = st.rhs_calls / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    print("bench: %d steps, %d RHS calls in %.3f s" % (args.steps, st.rhs_calls, elapsed),
          file=sys.stderr, flush=True)
    n = tuple(cfg["n"])

    # right-hand side alone (no integrator work)
    rhs_ps, hd64 = time_rhs_only(sim, h, 200)
    rhs_med_ms = rhs_event_median(sim, h, hd64)
    rhs_hbm = None if args.no_events else rhs_bandwidth(sim, h, hd64, rhs_ps, n)

    # per-kernel durations with HIP events on the library's stream, same steps
    per_kind, roof = {}, None
    if not args.no_events:
        per_kind = kernel_profile(sim, lambda: run_steps(sim, h, T_STAR, min(args.steps, 50)))
        whole = dict(rhs_hbm, note="whole right-hand side: library byte count per call x calls/s "
                                   "(rhs_only); at 128^3 its working set (~105 MB FP64) fits in the "
                                   "256 MB last-level cache, so lens256_f32 is the HBM regime")
        roof = roofline_of(per_kind, measured_traffic, whole)

    fp32 = None
    if not args.no_fp32:
        print("bench: FP32 leg", file=sys.stderr, flush=True)
        sim32 = make_sim(cfg, scfft.F32, FIXED_ITER)
        h32 = h.float()
        rhs32, hd32 = time_rhs_only(sim32, h32, 200)
        # FP32 against FP64 on the same state, both from an Ohm-law start
        s32 = make_sim(cfg, scfft.F32, FIXED_ITER)
        s64 = make_sim(cfg, scfft.F64, FIXED_ITER)
        o32, _ = s32.rhs_eval(T_STAR, h32)
        o64, _ = s64.rhs_eval(T_STAR, h)
        torch.cuda.synchronize()
        rel = float(torch.linalg.vector_norm(o32.double() - o64) / torch.linalg.vector_norm(o64))
        s32.close()
        s64.close()
        st32, el32 = timed_steps(sim32, h32, args.steps, args.warmup)
        fp32 = dict(value=round(st32.rhs_calls / el32, 2), rhs_only=round(rhs32, 2),
                    rel_l2_vs_fp64=rel, ms_per_step=round(1e3 * el32 / args.steps, 3))
        if not args.no_events:
            pk32 = kernel_profile(sim32, lambda: run_steps(sim32, h32, T_STAR, min(args.steps, 50)))
            fp32["roofline"] = roofline_of(pk32, None, rhs_bandwidth(sim32, h32, hd32, rhs32, n))
            fp32["kernels"] = pk32
        sim32.close()

    converged = None if args.no_converged else converged_leg(cfg, h)
    print("bench: 256^3 lens leg", file=sys.stderr, flush=True)
    lens = None if args.no_lens else lens256_leg()
    print("bench: adjoint leg", file=sys.stderr, flush=True)
    adj = None if args.no_adjoint else adjoint_leg(cfg)
    print("bench: batch leg", file=sys.stderr, flush=True)
    gleg = None if args.no_graph else graph_leg()
    print("bench: same-size 128^3 batch leg", file=sys.stderr, flush=True)
    b128 = None if args.no_graph else batch128_leg()
    extras = None
    if args.extras:
        extras = {"shield": shield_leg(), "lens_config": lens_config_leg(), "shield_config": shield_config_leg(),
                  "lens_gain": {"n_power": 30.0, "rho_out": 100.0,
                                "paper_biconical": {"gain_0.05": 2.0, "gain_0.20": 1.6},
                                "128": lens_gain_leg(128), "256": lens_gain_leg(256, f32=True)}}

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline (3 oracle calls at 128^3)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg, h_np)

    line = {
        "metric": "RHS evals/sec at 128³ (FP64 vs FP32 @1e-4 rel err), % HBM peak; adjoint cost",
        "value": round(value, 2),
        "unit": "RHS evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s: closed-end hollow cylinder shield, 128^3 FFT box, n=100, "
                               "sine drive 0.05 T 50 Hz at 45 deg; BS23 fixed steps, %d exterior "
                               "iterations per RHS, moment readout per step" % (args.config, FIXED_ITER),
                   "grid": list(n), "exterior_iters": FIXED_ITER, "rhs_per_step": 3},
        "rhs_only": round(rhs_ps, 2),
        "rhs_median_ms": round(rhs_med_ms, 4),
        "rhs_hbm": rhs_hbm,
        "fp32": fp32,
        "converged": converged,
        "lens256_f32": lens,
        "adjoint_cost": adj,
        "graphs": gleg,
        "batch128": b128,
        "extras": extras,
        "roofline": roof,
        "kernels": per_kind,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
