#!/usr/bin/env python3
"""Throughput of the plain complementarity-free contact step on one MI355X.

Workload: the dense pile (4096 worlds x 64 free spheres in a 0.5 m walled box,
radius U(0.02, 0.05) m, density 1000 kg/m^3, condim 3 / 4-facet cone, h = 2 ms,
k_user = 0.1, d_user = 0.001), seeded and synthetic.  A step is one full pass of
the hot path (narrow phase, smooth prediction, facet impulses, per-body
reduction, velocity correction, integration) over all worlds.  The input is
the settled pile: the lattice falls for a fixed number of steps (--settle,
default 500, stated in the output's config), then W untimed warm-up steps run
and exactly K steps are timed with the state resident in HBM.  Further forms
of the step (batched rollouts, learned gains, the hand's MPC rollouts) and the
CPU baseline are measured afterwards; a failure in any of them is recorded in
its own entry and never stops the headline.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "env-steps/s & contact-impulses/s (+% HBM peak) vs plain form, 1 MI355X"
HBM_PEAK = 8.0e12  # B/s, MI355X published HBM3E bandwidth
SETTLE_STEPS = 500       # lattice -> settled pile (about 1 s of simulated time)
SETTLE_STEPS_128 = 800   # the taller 128-sphere pile
LEARNED_MARGIN = 1e-4    # fallback margin of the learned gains (m)
CPU_SHARE = 16           # host threads the GPU machine grants one GPU
PAPER_CONTEXT = ("context only, not a target: the paper reports 2-3x the throughput of MuJoCo Warp in "
                 "dense-contact scenes and ~2.4x faster MPPI steps, on one NVIDIA RTX 4090 with an AMD "
                 "32-core CPU, precision not stated, no absolute env-steps/s printed")


def alg_bytes(nq, nv, nb, ng, contacts, condim=3):
    """Algorithmic HBM bytes per world-step of each kernel (contacts = C_w).

    collide: read q and per-world geom data (size, friction: 16 B/geom), write
             the contact records (32 B each) and the count.
    resolve: read q, v, per-body mass/inertia (16 B/body), per-world geom
             friction (mu_t: 4 B/geom, plus mu_tor and mu_rol for condim >= 4),
             the contact records and count; write q and v.
    Shared tables (candidate slots, static geom poses) are read from L2 by every
    world and are not counted."""
    collide = 4 * nq + 16 * ng + 32 * contacts + 8
    resolve = 8 * nq + 8 * nv + 16 * nb + (4 + (8 if condim >= 4 else 0)) * ng + 32 * contacts + 4
    return collide, resolve


def cpu_baseline(scene, q, v, worlds, steps, threads):
    """Time the FP64 oracle (as it stands) on a bounded sample of the same workload."""
    from oracle.cfo import Oracle
    from paper_2603_12185_amd import scenes
    sub = scenes.select_worlds(scene, worlds)
    o = Oracle(sub)
    qs, vs = q[worlds].astype(np.float64), v[worlds].astype(np.float64)
    t0 = time.perf_counter()
    for _ in range(steps):
        qs, vs = o.step_threads(qs, vs, threads)
    dt = time.perf_counter() - t0
    return len(worlds) * steps / dt, dt


def progress(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def pile_run(nw, nsphere, condim, k_user, d_user, steps, last, seed=0):
    """One plain-form run of the dense pile from its initial lattice: `steps`
    cf_step calls, timed as a whole and over the last `last` steps (HIP events
    on the launch stream at step 0, steps - last and steps), with the contact
    count of every world-step kept on the device.  Returns a dict of rates and
    contact statistics (mean and max contacts per world-step over the whole run
    and over the last steps) and both kernels' durations on the final state."""
    import torch

    from paper_2603_12185_amd import cfsim, scenes
    dev = torch.device("cuda:0")
    scene = scenes.dense_pile(nworld=nw, nsphere=nsphere, seed=seed, condim=condim,
                              k_user=k_user, d_user=d_user)
    model = cfsim.Model(scene)
    lib = cfsim.load()
    stream = torch.cuda.current_stream()
    sp = C.c_void_p(stream.cuda_stream)
    nq, nv = model.nq, model.nv
    q = [torch.from_numpy(scene["q0"]).to(dev), torch.empty((nw, nq), device=dev)]
    v = [torch.from_numpy(scene["v0"]).to(dev), torch.empty((nw, nv), device=dev)]
    ncon = torch.zeros((steps, nw), dtype=torch.int32, device=dev)
    over = torch.zeros((steps, nw), dtype=torch.int32, device=dev)
    ptr = lambda t: C.c_void_p(t.data_ptr())
    cons = [cfsim.Contacts(ptr(ncon[t]), ptr(over[t]), None, None, None, None, None, None)
            for t in range(steps)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for t in range(steps):
        if t == steps - last:
            ev[1].record(stream)
        i = t & 1
        st = lib.cf_step(model._h, sp, ptr(q[i]), ptr(v[i]), None, ptr(q[1 - i]), ptr(v[1 - i]),
                         C.byref(cons[t]))
        if st != 0:
            raise cfsim.CFError(st, cfsim.last_error())
    ev[2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    f = steps & 1
    us_col, us_res = model.time_kernels(q[f], v[f], q[1 - f], v[1 - f], reps=200)
    ms_all, ms_last = ev[0].elapsed_time(ev[2]), ev[1].elapsed_time(ev[2])
    c = ncon.double()
    cl = c[steps - last:]
    bad = int(over.sum())
    finite = bool(torch.isfinite(q[f]).all() and torch.isfinite(v[f]).all())
    return {
        "bodies_per_world": model.nbody, "condim": condim, "k_user": k_user, "d_user": d_user,
        "steps": steps, "wall_s": wall,
        "whole_run": {"env_steps_per_s": nw * steps / (ms_all * 1e-3), "ms_per_step": ms_all / steps,
                      "mean_contacts_per_world": float(c.mean()), "max_contacts_per_world": int(c.max()),
                      "contact_impulses_per_s": float(c.sum()) / (ms_all * 1e-3)},
        f"last_{last}_steps": {"env_steps_per_s": nw * last / (ms_last * 1e-3), "ms_per_step": ms_last / last,
                               "mean_contacts_per_world": float(cl.mean()),
                               "max_contacts_per_world": int(cl.max()),
                               "contact_impulses_per_s": float(cl.sum()) / (ms_last * 1e-3)},
        "kernel_us_final_state": {"collide_kernel": us_col, "resolve_kernel": us_res},
        "step_kernels": model.step_kernels(),
        "capacity_overflows": bad, "state_finite": finite,
    }


def sweep(args):
    """The pile's variants: bodies per world 16/32/64/128 (condim 3), condim 6
    and the stiffer (k, d) = (0.5, 0.005) at 64 bodies; each run from the
    initial lattice for `steps` steps, the whole run and the settled last 100
    steps reported separately.  Prints one JSON line."""
    nw, steps, last = args.nworld, args.sweep_steps, min(100, args.sweep_steps)
    runs = {}
    for nb in (16, 32, 64, 128):
        runs[f"bodies_{nb}"] = pile_run(nw, nb, 3, 0.1, 0.001, steps, last)
        progress(f"sweep bodies {nb}: {runs[f'bodies_{nb}'][f'last_{last}_steps']['env_steps_per_s']:.3e} env-steps/s")
    runs["condim_6"] = pile_run(nw, 64, 6, 0.1, 0.001, steps, last)
    progress("sweep condim 6 done")
    runs["k0.5_d0.005"] = pile_run(nw, 64, 3, 0.5, 0.005, steps, last)
    progress("sweep stiff gains done")
    # linearity in bodies per world: body-steps/s of the settled steps
    lin = {k: r["bodies_per_world"] * r[f"last_{last}_steps"]["env_steps_per_s"]
           for k, r in runs.items() if k.startswith("bodies_")}
    print(json.dumps({
        "metric": METRIC + " (pile variants)", "unit": "env-steps/s", "n_gpus": 1, "nworld": nw,
        "dtype": "f32", "data": "synthetic", "timing": "HIP events on the launch stream",
        "runs": runs, "body_steps_per_s_settled": lin}))


def host_info():
    """The host the CPU baseline runs on: logical CPUs of the machine, CPUs this
    process may run on, and the CPU model name."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": model}


def leg(result, name, fn):
    """Run one auxiliary measurement; a failure is recorded under its name and
    never stops the headline line from printing."""
    try:
        result[name] = fn()
    except Exception as e:  # noqa: BLE001 - recorded, reported, not hidden
        import traceback
        traceback.print_exc()
        progress(f"{name} failed: {type(e).__name__}: {e}")
        result[name] = {"error": f"{type(e).__name__}: {e}"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--settle", type=int, default=SETTLE_STEPS,
                    help="steps that let the pile fall and settle before warm-up and timing "
                         "(input preparation: the timed workload is the settled pile)")
    ap.add_argument("--nworld", type=int, default=4096)
    ap.add_argument("--nsphere", type=int, default=64)
    ap.add_argument("--condim", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-worlds", type=int, default=2048,
                    help="worlds in the CPU-baseline sample on the box's CPU share (0 disables it)")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--cpu1-worlds", type=int, default=96,
                    help="worlds in the 1-core CPU-baseline sample (0 disables it)")
    ap.add_argument("--rollout-steps", type=int, default=1000,
                    help="steps of the batched-rollout form timed after the plain form (0: skip)")
    ap.add_argument("--learned-steps", type=int, default=200,
                    help="steps of the learned-impedance form timed after the plain form (0: skip)")
    ap.add_argument("--learned-big-worlds", type=int, default=8192,
                    help="worlds of 128 spheres for the learned gains' configured evaluation (0: skip)")
    ap.add_argument("--hand-rollouts", type=int, default=2048,
                    help="rollouts per MPPI iteration of the hand-and-cube form (0: skip)")
    ap.add_argument("--hand-horizon", type=int, default=20)
    ap.add_argument("--hand-iters", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain elementwise copy of this many MiB five times (a "
                         "known-traffic kernel that calibrates HBM byte counters under a profiler)")
    ap.add_argument("--sweep", action="store_true",
                    help="run the pile's variants (bodies per world 16/32/64/128, condim 6, "
                         "(k, d) = (0.5, 0.005)) instead of the default measurement")
    ap.add_argument("--sweep-steps", type=int, default=500)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}): "
              "worlds shard across GPUs with no exchange, so this build reports the one-GPU "
              "throughput and runs no multi-GPU configuration.", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0 or args.settle < 0:
        sys.exit("--steps must be >= 1, --warmup and --settle >= 0")

    import torch

    from paper_2603_12185_amd import cfsim, scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.sweep:
        sweep(args)
        return
    scene = scenes.dense_pile(nworld=args.nworld, nsphere=args.nsphere, seed=args.seed,
                              condim=args.condim)
    model = cfsim.Model(scene)
    nw, nq, nv, nb, ng = model.nworld, model.nq, model.nv, model.nbody, model.ngeom
    lib = cfsim.load()
    stream = torch.cuda.current_stream()
    sp = C.c_void_p(stream.cuda_stream)

    q = [torch.from_numpy(scene["q0"]).to(dev), torch.empty((nw, nq), device=dev)]
    v = [torch.from_numpy(scene["v0"]).to(dev), torch.empty((nw, nv), device=dev)]
    K, W, S = args.steps, args.warmup, args.settle
    ncon_log = torch.zeros((K, nw), dtype=torch.int32, device=dev)
    over_log = torch.zeros((K, nw), dtype=torch.int32, device=dev)
    cons = [cfsim.Contacts(C.c_void_p(ncon_log[t].data_ptr()), C.c_void_p(over_log[t].data_ptr()),
                           None, None, None, None, None, None) for t in range(K)]
    ptr = lambda t: C.c_void_p(t.data_ptr())
    args_pp = [(model._h, sp, ptr(q[i]), ptr(v[i]), None, ptr(q[1 - i]), ptr(v[1 - i])) for i in (0, 1)]

    def run(n, logged):
        for t in range(n):
            a = args_pp[t & 1]
            st = lib.cf_step(*a, C.byref(cons[t]) if logged else None)
            if st != 0:
                raise cfsim.CFError(st, cfsim.last_error())
        if n % 2:  # keep the live state in buffer 0
            q[0].copy_(q[1])
            v[0].copy_(v[1])

    # Input preparation: the pile falls from its lattice and settles (S steps);
    # then W untimed warm-up steps; then exactly K timed steps.
    run(S, False)
    torch.cuda.synchronize()
    progress(f"pile settled: {S} steps")
    run(W, False)
    torch.cuda.synchronize()
    state_q, state_v = q[0].clone(), v[0].clone()

    # Timed region: K steps, nothing recorded between the launches.
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for t in range(K):
        st = lib.cf_step(*args_pp[t & 1], C.byref(cons[t]))
        if st != 0:
            raise cfsim.CFError(st, cfsim.last_error())
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)

    # Kernel durations, live, on the launch stream, from the state the timed
    # region started in: each kernel launched K times back to back, one pair of
    # HIP events around each group (events between the two kernels of every
    # step would add their own gaps to both).
    qa, va = state_q.clone(), state_v.clone()
    qb, vb = torch.empty_like(qa), torch.empty_like(va)
    us_col, us_res = model.time_kernels(qa, va, qb, vb, reps=max(K, 20))
    progress(f"plain form: {K} steps in {wall:.3f} s; kernels {us_col:.1f} / {us_res:.1f} us apart")

    ncon = ncon_log.double()
    overflows = int(over_log.sum())
    contacts_per_step = float(ncon.sum(1).mean())
    c_w = contacts_per_step / nw
    ms_step = wall * 1e3 / K
    env_steps = nw * K / wall
    imp = contacts_per_step * K / wall
    b_col, b_res = alg_bytes(nq, nv, nb, ng, c_w, args.condim)
    t_col, t_res = us_col * 1e-6, us_res * 1e-6
    one_kernel = model.step_kernels() == 1
    if one_kernel:
        # cf_step is one kernel (narrow phase and resolution of each world in
        # one workgroup): its launch duration is the timed region's HIP-event
        # time per step (K launches back to back on the launch stream), its
        # algorithmic bytes those of both phases
        dom, t_dom, b_dom = "step_kernel", gpu_ms * 1e-3 / K, b_col + b_res
    elif t_col >= t_res:
        dom, t_dom, b_dom = "collide_kernel", t_col, b_col
    else:
        dom, t_dom, b_dom = "resolve_kernel", t_res, b_res
    achieved = b_dom * nw / t_dom
    step_bytes = (b_col + b_res) * nw
    survey_bytes = (8 * (nq + nv) + 16 * nb + 72 * c_w) * nw

    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        from paper_2603_12185_amd import build as _b
        import hashlib
        src = b"".join(open(os.path.join(_b.CSRC, s), "rb").read() for s in sorted(os.listdir(_b.CSRC)))
        rec = json.load(open(tfile))
        if rec.get("source_sha256") == hashlib.sha256(src).hexdigest() and dom in rec.get("kernels", {}):
            traffic = rec["kernels"][dom]["bytes_per_launch"]

    result = {
        "metric": METRIC, "value": env_steps, "unit": "env-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"dense_pile_{nw}x{args.nsphere}", "nworld": nw,
                   "bodies_per_world": nb, "condim": args.condim, "nfacet": model.nfacet,
                   "h": scene["h"], "k_user": scene["k_user"], "d_user": scene["d_user"],
                   "ncon_max": model.ncon_max, "settle_steps": S,
                   "mean_contacts_per_world": c_w, "form": "plain",
                   "parallelism": "single GPU, one workgroup per world"},
        "contact_impulses_per_s": imp,
        "facet_impulses_per_s": imp * model.nfacet,
        "capacity_overflows": overflows,
        "gpu_event_ms_per_step": gpu_ms / K,
        "kernel_us": {"collide_kernel": t_col * 1e6, "resolve_kernel": t_res * 1e6,
                      "timing": f"HIP events around {max(K, 20)} back-to-back launches of each kernel "
                                "on the launch stream, from the state the timed region started in"
                                + ("; cf_step runs both phases in one kernel (step_kernel: HIP events "
                                   "around the timed region's launches)" if one_kernel else "")},
        "whole_step_alg_GBps": step_bytes / (wall / K) / 1e9,
        "whole_step_hbm_frac": step_bytes / (wall / K) / HBM_PEAK,
        "whole_step_contract_bytes_frac": survey_bytes / (wall / K) / HBM_PEAK,
        "step_kernels": 1 if one_kernel else 2,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK,
                     "traffic": traffic, "alg_bytes_per_launch": b_dom * nw},
        "paper_context": PAPER_CONTEXT,
    }
    if one_kernel:
        result["kernel_us"]["step_kernel"] = t_dom * 1e6
    if args.rollout_steps > 0:
        leg(result, "rollout_form", lambda: rollout_form(model, state_q, state_v, args.rollout_steps,
                                                         env_steps, stream))
    if args.learned_steps > 0:
        leg(result, "learned_form", lambda: learned_form(model, state_q, state_v, args.learned_steps,
                                                         env_steps, sp))
    if args.learned_steps > 0 and args.learned_big_worlds > 0:
        leg(result, "learned_form_128_spheres", lambda: learned_big(args, sp))
    if args.hand_rollouts > 0:
        leg(result, "hand_form", lambda: hand_form(args))
    if args.cpu_worlds > 0 or args.cpu1_worlds > 0:
        leg(result, "cpu_baseline", lambda: cpu_leg(args, scene, state_q, state_v))
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, device=dev)
        dst = torch.empty(n, device=dev)
        for _ in range(5):
            torch.neg(src, out=dst)  # reads and writes copy_mib MiB
        torch.cuda.synchronize()
        result["copy_calibration_mib"] = args.copy_mib
    print(json.dumps(result), flush=True)


def rollout_form(model, state_q, state_v, T, env_steps, stream):
    """Batched-rollout form: the same step, T steps per cf_rollout call (one
    persistent kernel per call when the world fits a workgroup's LDS), from the
    same settled state, trajectory written to HBM every step."""
    import torch
    dev = state_q.device
    nw, nq, nv = model.nworld, model.nq, model.nv
    q0, v0 = state_q.clone(), state_v.clone()
    qt = torch.empty((T + 1, nw, nq), device=dev)
    vt = torch.empty((T + 1, nw, nv), device=dev)
    nct = torch.zeros((T, nw), dtype=torch.int32, device=dev)
    ovt = torch.zeros((T, nw), dtype=torch.int32, device=dev)

    def time_rollout():
        model.rollout(min(T, 20), q0, v0, q_traj=qt, v_traj=vt, ncon_traj=nct, overflow_traj=ovt)
        torch.cuda.synchronize()
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        r0.record(stream)
        model.rollout(T, q0, v0, q_traj=qt, v_traj=vt, ncon_traj=nct, overflow_traj=ovt)
        r1.record(stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r0.elapsed_time(r1) / T

    # the persistent kernel at the default launch shape, then whatever the
    # autotuner picks for this model (persistent kernel or step launches)
    first = model.get_launch()
    rwall_p, _ = time_rollout()
    over_p = int(ovt.sum())
    best_step_us, best_roll_us = model.autotune(q0, v0, steps=50)
    rwall, rgpu = time_rollout()
    rc_w = float(nct.double().sum()) / (T * nw)
    launch = model.get_launch()
    b_roll = 8 * (nq + nv)  # per world-step: the trajectory rows written
    progress(f"rollout form: {T} steps in {rwall:.2f} s")
    return {
        "value": nw * T / rwall, "unit": "env-steps/s", "steps": T,
        "ms_per_step": rwall * 1e3 / T, "gpu_event_ms_per_step": rgpu,
        "mean_contacts_per_world": rc_w, "contact_impulses_per_s": rc_w * nw * T / rwall,
        "capacity_overflows": int(ovt.sum()) + over_p,
        "persistent_kernel": launch[3], "blocks": list(launch[:3]),
        "vs_plain_form": (nw * T / rwall) / env_steps,
        "alg_GBps": b_roll * nw * T / rwall / 1e9,
        "autotune_us_per_step": {"step_launches": best_step_us, "persistent_kernel": best_roll_us},
        "persistent_kernel_default_shape": {"block": first[2], "used": first[3],
                                            "ms_per_step": rwall_p * 1e3 / T,
                                            "vs_plain_form": (nw * T / rwall_p) / env_steps},
    }


def learned_form(model, state_q, state_v, L, env_steps, sp):
    """Learned-impedance form: train the network on the GPU on one step's
    contacts of this workload (exported by the step itself), then time L steps
    with the learned gains and compare mean penetration, normal jitter and the
    fallback rate with the plain form over the same steps from the same state."""
    import torch

    from paper_2603_12185_amd import cfsim, learned
    lib = cfsim.load()
    ptr = lambda t: C.c_void_p(t.data_ptr())
    nw = model.nworld
    qs, vs = state_q.clone(), state_v.clone()
    launch = model.get_launch()
    t0 = time.perf_counter()
    feats, targets, _, _ = learned.collect(model, qs.clone(), vs.clone(), steps=1, margin=LEARNED_MARGIN)
    net, losses = learned.train(feats, targets, model.nfacet, steps=300)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    mp, xp, _, vp, _ = learned.penetration_stats(model, qs.clone(), vs.clone(), 100)
    model.set_learned_impedance(net, margin=LEARNED_MARGIN)
    ml, xl, _, vl, fb = learned.penetration_stats(model, qs.clone(), vs.clone(), 100)
    lq = [qs.clone(), torch.empty_like(qs)]
    lv = [vs.clone(), torch.empty_like(vs)]
    lpp = [(model._h, sp, ptr(lq[i]), ptr(lv[i]), None, ptr(lq[1 - i]), ptr(lv[1 - i])) for i in (0, 1)]
    for t in range(20):
        lib.cf_step(*lpp[t & 1], None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(L):
        st = lib.cf_step(*lpp[t & 1], None)
        if st != 0:
            raise cfsim.CFError(st, cfsim.last_error())
    torch.cuda.synchronize()
    lwall = time.perf_counter() - t0
    us_lc, us_lr = model.time_kernels(qs, vs, lq[1], lv[1], reps=100)
    model.set_learned_impedance(None)
    model.set_launch(*launch[:3])
    ke = lambda vv: float((vv.reshape(nw, -1, 6)[:, :, 0:3] ** 2).sum(-1).mean())
    progress(f"learned form: {L} steps in {lwall:.2f} s")
    return {
        "value": nw * L / lwall, "unit": "env-steps/s", "steps": L, "ms_per_step": lwall * 1e3 / L,
        "vs_plain_form": (nw * L / lwall) / env_steps,
        "kernel_us": {"collide_kernel": us_lc, "resolve_kernel_learned": us_lr},
        "network": "7-64-64-%d SiLU, bf16 MFMA, fp32 accumulation" % model.nfacet,
        "training": f"{feats.shape[0]} contacts of one step of this workload, 300 Adam steps of 65536, "
                    f"loss {losses[0]:.3g} -> {losses[-1]:.3g}, {train_s:.1f} s incl. data export",
        "fallback_margin_m": LEARNED_MARGIN,
        "fallback_fraction": fb,
        "mean_penetration_mm": {"plain": mp * 1e3, "learned": ml * 1e3},
        "max_penetration_mm": {"plain": xp * 1e3, "learned": xl * 1e3},
        "mean_sq_speed_after_100_steps": {"plain": ke(vp), "learned": ke(vl)},
    }


def learned_big(args, sp):
    """The learned gains' configured evaluation: worlds of 128 spheres (about
    twice the contacts per world), a network trained on 1e6 contacts of one
    plain step of this workload, then penetration, jitter, fallback rate and
    throughput of the learned and the plain form from the same settled state."""
    import torch

    from paper_2603_12185_amd import cfsim, learned, scenes
    lib = cfsim.load()
    dev = torch.device("cuda:0")
    ptr = lambda t: C.c_void_p(t.data_ptr())
    NB, L = args.learned_big_worlds, args.learned_steps
    big = scenes.dense_pile(nworld=NB, nsphere=128, seed=args.seed + 1, condim=args.condim, ncon_max=2048)
    bm = cfsim.Model(big)
    bq = [torch.from_numpy(big["q0"]).to(dev), torch.empty((NB, bm.nq), device=dev)]
    bv = [torch.from_numpy(big["v0"]).to(dev), torch.empty((NB, bm.nv), device=dev)]
    bpp = [(bm._h, sp, ptr(bq[i]), ptr(bv[i]), None, ptr(bq[1 - i]), ptr(bv[1 - i])) for i in (0, 1)]

    def big_steps(n):
        for t in range(n):
            st = lib.cf_step(*bpp[t & 1], None)
            if st != 0:
                raise cfsim.CFError(st, cfsim.last_error())

    big_steps(SETTLE_STEPS_128)  # settle (even count: the state ends in buffer 0)
    torch.cuda.synchronize()
    sq0, sv0 = bq[0].clone(), bv[0].clone()
    feats, targets, _, _ = learned.collect(bm, sq0.clone(), sv0.clone(), steps=1, margin=LEARNED_MARGIN)
    g = torch.Generator(device=dev)
    g.manual_seed(args.seed)
    pick = torch.randperm(feats.shape[0], generator=g, device=dev)[:1000000]
    net, losses = learned.train(feats[pick].contiguous(), targets[pick].contiguous(), bm.nfacet, steps=300)
    nrows = int(feats.shape[0])
    del feats, targets
    mp, xp, _, vp, _ = learned.penetration_stats(bm, sq0.clone(), sv0.clone(), 100)
    timings = {}
    for form in ("plain", "learned"):
        bm.set_learned_impedance(net if form == "learned" else None, margin=LEARNED_MARGIN)
        bq[0].copy_(sq0)
        bv[0].copy_(sv0)
        big_steps(20)
        bq[0].copy_(sq0)
        bv[0].copy_(sv0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        big_steps(L)
        torch.cuda.synchronize()
        timings[form] = time.perf_counter() - t0
    bm.set_learned_impedance(net, margin=LEARNED_MARGIN)
    ml, xl, _, vl, fb = learned.penetration_stats(bm, sq0.clone(), sv0.clone(), 100)
    bm.set_learned_impedance(None)
    ncon_big = {"ncon": torch.zeros(NB, dtype=torch.int32, device=dev)}
    bm.step(sq0, sv0, contacts=ncon_big)
    ke = lambda vv: float((vv.reshape(NB, -1, 6)[:, :, 0:3] ** 2).sum(-1).mean())
    progress(f"learned form {NB}x128: {L} steps plain {timings['plain']:.2f} s, learned {timings['learned']:.2f} s")
    out = {
        "workload": f"dense_pile_{NB}x128", "steps": L, "settle_steps": SETTLE_STEPS_128,
        "mean_contacts_per_world": float(ncon_big["ncon"].double().mean()),
        "value": NB * L / timings["learned"], "unit": "env-steps/s",
        "plain_value": NB * L / timings["plain"],
        "vs_plain_form": timings["plain"] / timings["learned"],
        "training": f"{min(nrows, 1000000)} of {nrows} contacts of one plain step, 300 Adam steps of 65536, "
                    f"loss {losses[0]:.3g} -> {losses[-1]:.3g}",
        "fallback_margin_m": LEARNED_MARGIN,
        "fallback_fraction": fb,
        "mean_penetration_mm": {"plain": mp * 1e3, "learned": ml * 1e3},
        "max_penetration_mm": {"plain": xp * 1e3, "learned": xl * 1e3},
        "mean_sq_speed_after_100_steps": {"plain": ke(vp), "learned": ke(vl)},
    }
    del bm, bq, bv, big
    torch.cuda.empty_cache()
    return out


def hand_form(args):
    """Batched-MPC form: the actuated four-finger hand with a free cube (6D
    contacts), N rollouts of H steps per MPPI iteration with Gaussian noise of
    0.1 rad on the 16 finger targets; one cf_rollout call per batch (persistent
    kernel when the autotuner keeps it), eager and replayed from a captured
    graph, the same batch as H cf_step launches, and whole MPPI iterations
    (sampling, rollouts, costs, weights, update, one plant step)."""
    import torch

    from paper_2603_12185_amd import cfsim, mpc
    lib = cfsim.load()
    N, H, R = args.hand_rollouts, args.hand_horizon, args.hand_iters
    ctl = mpc.HandMPPI(nroll=N, H=H, sigma=0.1, seed=args.seed)
    for _ in range(3):
        ctl.iterate()
    u, _ = ctl.sample()
    ctl.tau_seq[:, :, 6:] = u.transpose(0, 1)
    ctl.q0s.copy_(ctl.q.expand(N, -1))
    ctl.v0s.copy_(ctl.v.expand(N, -1))
    dev = ctl.q0s.device
    ncon_h = torch.zeros((H, N), dtype=torch.int32, device=dev)
    over_h = torch.zeros((H, N), dtype=torch.int32, device=dev)
    hs = torch.cuda.current_stream()
    m = ctl.model

    def hand_roll():
        m.rollout(H, ctl.q0s, ctl.v0s, tau_seq=ctl.tau_seq, q_traj=ctl.q_traj,
                  v_traj=ctl.v_traj, ncon_traj=ncon_h, overflow_traj=over_h)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(hs)
        for _ in range(R):
            fn()
        e1.record(hs)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / R, e0.elapsed_time(e1) / R

    hwall, hgpu = timed(hand_roll)
    hc_w = float(ncon_h.double().mean())
    hmax = int(ncon_h.max())
    hover = int(over_h.sum())

    # the same batch as H step launches (what cf_rollout does without the
    # persistent kernel), trajectory rows written by the steps themselves
    sp = C.c_void_p(hs.cuda_stream)
    ptr = lambda t: C.c_void_p(t.data_ptr())
    stride_q, stride_v = N * m.nq * 4, N * m.nv * 4
    qt0, vt0, tt0 = ctl.q_traj.data_ptr(), ctl.v_traj.data_ptr(), ctl.tau_seq.data_ptr()

    def hand_steps():
        ctl.q_traj[0].copy_(ctl.q0s)
        ctl.v_traj[0].copy_(ctl.v0s)
        for t in range(H):
            st = lib.cf_step(m._h, sp, C.c_void_p(qt0 + t * stride_q), C.c_void_p(vt0 + t * stride_v),
                             C.c_void_p(tt0 + t * stride_v), C.c_void_p(qt0 + (t + 1) * stride_q),
                             C.c_void_p(vt0 + (t + 1) * stride_v), None)
            if st != 0:
                raise cfsim.CFError(st, cfsim.last_error())

    swall, sgpu = timed(hand_steps)

    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(hs)
    with torch.cuda.stream(side):
        hand_roll()
    hs.wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        hand_roll()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(R):
        graph.replay()
    torch.cuda.synchronize()
    gwall = (time.perf_counter() - t0) / R
    t0 = time.perf_counter()
    for _ in range(R):
        ctl.iterate()
    torch.cuda.synchronize()
    iwall = (time.perf_counter() - t0) / R
    launch = m.get_launch()
    progress(f"hand form: {R} batches of {N} x {H}: rollout {hwall * 1e3:.3f} ms, steps {swall * 1e3:.3f} ms")
    return {
        "value": N * H / hwall, "unit": "env-steps/s", "rollouts": N, "horizon": H,
        "ms_per_rollout_batch": hwall * 1e3, "gpu_event_ms_per_rollout_batch": hgpu,
        "step_launches_ms_per_rollout_batch": swall * 1e3,
        "step_launches_gpu_event_ms_per_rollout_batch": sgpu,
        "vs_step_launches": swall / hwall,
        "graph_replay_ms_per_rollout_batch": gwall * 1e3,
        "ms_per_mppi_iteration": iwall * 1e3,
        "mean_contacts_per_world_step": hc_w, "max_contacts_per_world_step": hmax,
        "capacity_overflows": hover,
        "persistent_kernel": launch[3], "rollout_block": launch[2], "launch": "autotuned",
        "scene": "16 hinge dofs in 4 fingers (capsule links, fingertip spheres, position "
                 "actuators) + free 5 cm cube, nv 22, condim 6, h 2 ms, sigma 0.1 rad",
    }


def cpu_leg(args, scene, state_q, state_v):
    """The FP64 oracle as it stands on a bounded sample of the settled pile:
    worlds split statically over the machine's CPU share (threads), and a second,
    smaller sample on one thread."""
    qn, vn = state_q.cpu().numpy(), state_v.cpu().numpy()
    nw = qn.shape[0]
    host = host_info()
    threads = min(CPU_SHARE, host["affinity_cpus"])
    rng = np.random.default_rng(0)
    out = {"unit": "env-steps/s", "kind": "oracle", "host": host}
    if args.cpu_worlds > 0:
        sample = np.sort(rng.choice(nw, size=min(args.cpu_worlds, nw), replace=False))
        rate, dt = cpu_baseline(scene, qn, vn, sample, args.cpu_steps, threads)
        progress(f"cpu baseline ({threads} threads): {dt:.1f} s")
        out.update({"value": rate, "cores": threads,
                    "sample": f"{len(sample)} worlds x {args.cpu_steps} steps of the same settled pile "
                              f"(FP64 oracle, {threads} threads, {dt:.1f} s wall)"})
    if args.cpu1_worlds > 0:
        sample1 = np.sort(rng.choice(nw, size=min(args.cpu1_worlds, nw), replace=False))
        rate1, dt1 = cpu_baseline(scene, qn, vn, sample1, args.cpu_steps, 1)
        progress(f"cpu baseline (1 thread): {dt1:.1f} s")
        out["one_core"] = {"value": rate1, "cores": 1,
                           "sample": f"{len(sample1)} worlds x {args.cpu_steps} steps ({dt1:.1f} s wall)"}
        if "value" not in out:
            out.update({"value": rate1, "cores": 1, "sample": out["one_core"]["sample"]})
    return out


if __name__ == "__main__":
    main()
