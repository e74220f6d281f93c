"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Per-step parity feeds both sides the same float32 state; tolerances and the
guard band are stated in tests/parity.py.  All tests here need an MI355X.
"""
import os
import time

import numpy as np
import pytest

from oracle.cfo import Oracle
from paper_2603_12185_amd import scenes

from parity import compare_step, tdev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_12185_amd import cfsim
    cfsim.load()
    return torch


def applied_wrench(s, rng, lin_acc=2.0, ang_acc=20.0, shape=()):
    """Random applied force/torque per free body, scaled by its mass and inertia
    (accelerations of order lin_acc m/s^2 and ang_acc rad/s^2)."""
    nw, nb = s["nworld"], s["nbody"]
    t = rng.normal(0.0, 1.0, shape + (nw, nb, 6))
    t[..., :3] *= lin_acc * s["body_mass"][:, :, None]
    t[..., 3:] *= ang_acc * s["body_inertia"]
    return t.reshape(shape + (nw, 6 * nb)).astype(np.float32)


def _oracle_states(scene, nsteps, tau=None, record_every=1):
    """The oracle's own trajectory from the scene's initial state; returns
    [(t, q_t, v_t)] at the recorded steps, cast to float32 (the shared input of
    both sides).  tau: [nw][nv] held constant, or None."""
    o = Oracle(scene)
    q, v = scene["q0"].astype(np.float64), scene["v0"].astype(np.float64)
    tau64 = None if tau is None else np.asarray(tau, np.float64)
    threads = max(1, min(16, len(os.sched_getaffinity(0)), scene["nworld"]))
    out = []
    for t in range(nsteps):
        if (t % record_every == 0) or t == nsteps - 1:
            out.append((t, q.astype(np.float32), v.astype(np.float32)))
        if t + 1 < nsteps:
            q, v = o.step_threads(q, v, threads, tau64)
        if t % 200 == 199:
            print(f"  oracle trajectory at step {t + 1}", flush=True)
    return out


def _run_steps(torch, model, scene, nsteps, tau=None, record_every=1):
    """One GPU step from each recorded state of the oracle's trajectory (see
    _oracle_states).  Returns list of (t, q_in, v_in, q_out, v_out, contacts)."""
    tau_d = None if tau is None else tdev(tau)
    recs = []
    for t, qi, vi in _oracle_states(scene, nsteps, tau, record_every):
        con = model.alloc_contacts()
        q1, v1 = model.step(tdev(qi), tdev(vi), tau=tau_d, contacts=con)
        recs.append((t, qi, vi, q1.cpu().numpy(), v1.cpu().numpy(), to_np(con)))
    torch.cuda.synchronize()
    return recs


def test_boxes_drop_per_step_parity_1000_steps(torch_cuda):
    """Config: 1 world, 8 free boxes dropped on a plane, 1000 steps.  Every step:
    contact set bit-exact, velocities within 1e-5 relative."""
    from paper_2603_12185_amd import cfsim
    s = scenes.boxes_drop(seed=0)
    model = cfsim.Model(s)
    assert model.warning  # box-box pairs have no rule
    print("case: boxes_drop seed 0, 1000 steps", flush=True)
    recs = _run_steps(torch_cuda, model, s, 1000)
    o = Oracle(s)
    stats = None
    for t, qi, vi, qg, vg, con in recs:
        stats = compare_step(s, o, qi, vi, None, qg, vg, con, stats=stats)
    print("boxes_drop parity", stats)
    assert stats["checked"] >= 990 and stats["contacts"] > 1000


def test_boxes_drop_drift_report(torch_cuda):
    """Independent 1000-step runs: report per-step state divergence (not bounded)
    and the first step at which the contact sets differ."""
    from paper_2603_12185_amd import cfsim
    s = scenes.boxes_drop(seed=0)
    model = cfsim.Model(s)
    o = Oracle(s)
    q, v = s["q0"].astype(np.float64), s["v0"].astype(np.float64)
    qg, vg = tdev(s["q0"]), tdev(s["v0"])
    first_div, maxerr = None, []
    for t in range(1000):
        con = model.alloc_contacts()
        qg, vg = model.step(qg, vg, contacts=con)
        c = to_np(con)
        q, v, out = o.step(q, v)
        maxerr.append(float(np.abs(vg.cpu().numpy().astype(np.float64) - v).max()))
        if first_div is None and (c["ncon"][0] != out["ncon"][0] or
                                  (c["geom"][0, :out["ncon"][0]] != out["geom"][0, :out["ncon"][0]]).any()):
            first_div = t
    print(f"drift: max|dv| at steps 1/10/100/1000: {maxerr[0]:.2e} {maxerr[9]:.2e} "
          f"{maxerr[99]:.2e} {maxerr[-1]:.2e}; first contact-set divergence: {first_div}")
    assert np.isfinite(maxerr).all()


@pytest.mark.parametrize("condim", [1, 3, 4, 6])
def test_mixed_shapes_parity(torch_cuda, condim):
    """All pair rules (plane-sphere/capsule/box, sphere-sphere, static sphere),
    tilted planes, per-world sizes, random applied forces; 150 steps."""
    from paper_2603_12185_amd import cfsim
    s = scenes.mixed_shapes(nworld=5, seed=condim, condim=condim)
    model = cfsim.Model(s)
    tau_np = applied_wrench(s, np.random.default_rng(condim))
    print(f"case: mixed_shapes condim {condim}", flush=True)
    recs = _run_steps(torch_cuda, model, s, 150, tau=tau_np, record_every=3)
    o = Oracle(s)
    stats = None
    for t, qi, vi, qg, vg, con in recs:
        assert np.abs(vg).max() < 1000.0, f"scene left the bounded regime at step {t}"
        stats = compare_step(s, o, qi, vi, tau_np, qg, vg, con, stats=stats)
    print("mixed parity", condim, stats)
    assert stats["contacts"] > 50


def test_dense_pile_small_parity(torch_cuda):
    """16 worlds x 64 spheres in the walled box: 2336 candidate slots per world
    (10 compaction chunks, ragged tail); compared every 40 steps over 600."""
    from paper_2603_12185_amd import cfsim
    s = scenes.dense_pile(nworld=16, nsphere=64, seed=7)
    model = cfsim.Model(s)
    print("case: dense_pile 16x64", flush=True)
    recs = _run_steps(torch_cuda, model, s, 600, record_every=40)
    o = Oracle(s)
    stats = None
    for t, qi, vi, qg, vg, con in recs:
        stats = compare_step(s, o, qi, vi, None, qg, vg, con, stats=stats)
    print("pile parity", stats)
    assert stats["contacts"] > 16 * 40


@pytest.mark.parametrize("nsphere", [7, 10, 33, 63, 64, 65, 100])
def test_sphere_block_sizes_parity(torch_cuda, nsphere):
    """The narrow phase's sphere block (every pair of a run of free spheres,
    tested cyclically) at odd and even counts, with one (<= 64) and two mask
    words per row: one step of a packed cluster with random spins against the
    oracle, contact set included."""
    from paper_2603_12185_amd import cfsim
    s = scenes.sphere_cluster(nsphere=nsphere, seed=nsphere, spread=0.07 * (nsphere / 10) ** (1 / 3),
                              ncon_max=1024)
    model = cfsim.Model(s)
    print(f"case: sphere block {nsphere} spheres", flush=True)
    q, v = s["q0"], s["v0"]
    con = model.alloc_contacts()
    q1, v1 = model.step(tdev(q), tdev(v), contacts=con)
    stats = compare_step(s, Oracle(s), q, v, None, q1.cpu().numpy(), v1.cpu().numpy(), to_np(con))
    print("sphere block", nsphere, stats)
    assert stats["checked"] == 1 and stats["contacts"] >= nsphere // 2


@pytest.mark.parametrize("case", ["pile64", "pile128", "cluster100"])
def test_collide_launch_shapes_agree(torch_cuda, case):
    """The narrow phase at 64, 128 and 256 threads per world (plane rows, the
    sphere block's one- and two-word register masks, their row loops and
    workgroup scans) finds the same contacts, bit for bit, in the same order; the
    resolution at each shape agrees with the default's to float32 rounding (its
    fixed-point headroom depends on the workgroup size)."""
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    if case == "cluster100":
        s, settle = scenes.sphere_cluster(nsphere=100, seed=5, spread=0.15, ncon_max=1024), 0
    else:
        s, settle = scenes.dense_pile(nworld=8, nsphere=int(case[4:]), seed=11), 300
    model = cfsim.Model(s)
    print(f"case: launch shapes {case}", flush=True)
    q, v = tdev(s["q0"]), tdev(s["v0"])
    for _ in range(settle):
        q, v = model.step(q, v)
    ref = None
    for blk in (64, 128, 256):
        model.set_launch(blk, blk)
        con = model.alloc_contacts()
        q1, v1 = model.step(q.clone(), v.clone(), contacts=con)
        rec = (con["ncon"].clone(), con["geom"].clone(), con["dist"].clone(), con["pos"].clone(),
               con["frame"].clone())
        if ref is None:
            ref = (rec, v1)
            assert int(con["ncon"].min()) > 0
            continue
        for x, y in zip(rec, ref[0]):
            assert torch.equal(x, y), f"contacts differ at {blk} threads per world"
        assert float((v1 - ref[1]).abs().max()) <= 1e-5 * float(ref[1].abs().max())


def test_dense_pile_many_contacts_parity(torch_cuda):
    """4 worlds x 128 spheres packed in two overlapping layers on the ground:
    more than 256 contacts per world (several compaction and reduction
    chunks); the packed state and the oracle's next three states compared."""
    from paper_2603_12185_amd import cfsim
    s = scenes.dense_pile(nworld=4, nsphere=128, seed=3)
    rng = np.random.default_rng(3)
    q = s["q0"].reshape(4, 128, 7)
    rad = s["geom_size"][:, 5:, 0]  # spheres follow the ground and four walls
    for w in range(4):
        for i in range(128):
            layer, j = divmod(i, 64)
            gx, gy = divmod(j, 8)
            q[w, i, 0] = (gx - 3.5) * 0.06 + rng.uniform(-0.002, 0.002)
            q[w, i, 1] = (gy - 3.5) * 0.06 + rng.uniform(-0.002, 0.002)
            q[w, i, 2] = rad[w, i] + layer * 0.055
    model = cfsim.Model(s)
    print("case: dense_pile 4x128 packed", flush=True)
    recs = _run_steps(torch_cuda, model, s, 4)
    o = Oracle(s)
    stats = None
    for t, qi, vi, qg, vg, con in recs:
        stats = compare_step(s, o, qi, vi, None, qg, vg, con, stats=stats)
    last_ncon = recs[-1][5]["ncon"]
    print("pile128 parity", stats, "ncon", [r[5]["ncon"].tolist() for r in recs])
    assert last_ncon.min() > 256


def test_dense_pile_full_size_sampled(torch_cuda):
    """The benchmark workload (4096 worlds x 64 spheres) in the benchmark's launch
    configuration: sampled worlds checked against the oracle at steps 150 and
    400; every world checked for finite state and ncon <= ncon_max."""
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    s = scenes.dense_pile(nworld=4096, nsphere=64, seed=0)
    model = cfsim.Model(s)
    print("case: dense_pile 4096x64 full size", flush=True)
    q, v = tdev(s["q0"]), tdev(s["v0"])
    sample = [0, 1, 777, 2048, 4095]
    ss = scenes.select_worlds(s, sample)
    o = Oracle(ss)
    # the sampled worlds' inputs at steps 150 and 400 come from the oracle's own trajectory
    ostates = {t: (qo, vo) for t, qo, vo in _oracle_states(ss, 401, record_every=50) if t in (150, 400)}
    idx = torch.tensor(sample, device="cuda")
    stats = None
    for t in range(401):
        con = None
        if t in (150, 400):
            con = model.alloc_contacts()
            q[idx], v[idx] = tdev(ostates[t][0]), tdev(ostates[t][1])
        q1, v1 = model.step(q, v, contacts=con)
        if con is not None:
            c = to_np(con)
            assert (c["ncon"] <= s["ncon_max"]).all() and (c["overflow"] == 0).all()
            qn, vn = q1.cpu().numpy(), v1.cpu().numpy()
            assert np.isfinite(qn).all() and np.isfinite(vn).all()
            sub = {k: val[sample] for k, val in c.items()}
            stats = compare_step(ss, o, ostates[t][0], ostates[t][1], None, qn[sample], vn[sample], sub,
                                 stats=stats)
            print(f"step {t}: mean contacts/world {c['ncon'].mean():.1f} max {c['ncon'].max()}")
        q, v = q1, v1
    torch.cuda.synchronize()
    print("full-size sampled parity", stats)
    assert stats["checked"] >= 8


def test_empty_and_overflow_edge_cases(torch_cuda):
    """No contacts (bodies in the air), ncon_max = 0 and a small ncon_max that
    truncates: counts, kept contacts and dynamics match the oracle."""
    from paper_2603_12185_amd import cfsim
    s = scenes.dense_pile(nworld=3, nsphere=16, seed=1)
    s["q0"].reshape(3, 16, 7)[:, :, 2] += 5.0
    for cm in (1024, 0, 5):
        sc = scenes.with_params(s, ncon_max=cm)
        model = cfsim.Model(sc)
        recs = _run_steps(torch_cuda, model, sc, 3)
        o = Oracle(sc)
        for t, qi, vi, qg, vg, con in recs:
            compare_step(sc, o, qi, vi, None, qg, vg, con)
            assert con["ncon"].sum() == 0
    # sunk spheres: many contacts, truncated
    s2 = scenes.dense_pile(nworld=3, nsphere=32, seed=2)
    s2["q0"].reshape(3, 32, 7)[:, :, 2] = 0.01
    for cm in (0, 5, 40):
        sc = scenes.with_params(s2, ncon_max=cm)
        model = cfsim.Model(sc)
        recs = _run_steps(torch_cuda, model, sc, 2)
        o = Oracle(sc)
        for t, qi, vi, qg, vg, con in recs:
            compare_step(sc, o, qi, vi, None, qg, vg, con)
            assert (con["overflow"] > 0).all()


def test_rollout_reports_overflow(torch_cuda):
    """cf_rollout counts, per step and world, the contacts dropped beyond
    ncon_max exactly as cf_step does: sunk spheres with a small capacity, on
    the free-body persistent kernel (contacts in the global workspace, any
    capacity) and on step launches (80 bodies, more than the free-body kernel
    takes, with a capacity too large for the general persistent kernel's
    LDS)."""
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    s2 = scenes.dense_pile(nworld=3, nsphere=32, seed=2)
    s2["q0"].reshape(3, 32, 7)[:, :, 2] = 0.01
    s3 = scenes.dense_pile(nworld=3, nsphere=80, seed=2)
    s3["q0"].reshape(3, 80, 7)[:, :, 2] = 0.01
    T = 4
    for base, cm, fused in ((s2, 5, True), (s2, 40, True), (s2, 4000, True), (s3, 4000, False)):
        sc = scenes.with_params(base, ncon_max=cm)
        model = cfsim.Model(sc)
        assert model.get_launch()[3] == fused
        q0, v0 = tdev(sc["q0"]), tdev(sc["v0"])
        nct = torch.full((T, 3), -1, dtype=torch.int32, device="cuda")
        ovt = torch.full((T, 3), -1, dtype=torch.int32, device="cuda")
        qt, vt = model.rollout(T, q0, v0, ncon_traj=nct, overflow_traj=ovt)
        for t in range(T):
            con = {"ncon": torch.zeros(3, dtype=torch.int32, device="cuda"),
                   "overflow": torch.zeros(3, dtype=torch.int32, device="cuda")}
            model.step(qt[t].clone(), vt[t].clone(), contacts=con)
            assert torch.equal(con["ncon"], nct[t]) and torch.equal(con["overflow"], ovt[t]), (cm, t)
        if cm < 100:
            assert (ovt > 0).all() and (nct == cm).all()
        else:
            assert (ovt == 0).all() and (nct > 40).all()


def test_in_place_update_and_determinism(torch_cuda):
    """q_out/v_out aliasing q/v gives the same bits as separate outputs; two
    runs from the same state are bitwise identical."""
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    s = scenes.dense_pile(nworld=64, nsphere=64, seed=5)
    model = cfsim.Model(s)
    q, v = tdev(s["q0"]), tdev(s["v0"])
    for _ in range(300):
        q, v = model.step(q, v)
    qa, va = q.clone(), v.clone()
    ref = [model.step(q, v) for _ in range(1)][0]
    model.step(qa, va, q_out=qa, v_out=va)
    torch.cuda.synchronize()
    assert torch.equal(ref[0], qa) and torch.equal(ref[1], va)
    runs = []
    for _ in range(2):
        qq, vv = q.clone(), v.clone()
        for _ in range(50):
            qq, vv = model.step(qq, vv)
        runs.append((qq, vv))
    torch.cuda.synchronize()
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])


def _rollout_vs_steps(torch, model, s, T, tau=None):
    """Rollout trajectory against repeated cf_step from the same start; returns the
    trajectories and per-step contact counts."""
    q0, v0 = tdev(s["q0"]), tdev(s["v0"])
    ncon = torch.zeros((T, s["nworld"]), dtype=torch.int32, device="cuda")
    over = torch.full((T, s["nworld"]), -1, dtype=torch.int32, device="cuda")
    qt, vt = model.rollout(T, q0, v0, tau_seq=tau, ncon_traj=ncon, overflow_traj=over)
    assert int(over.abs().sum()) == 0, "contact capacity overflowed in the rollout"
    q, v = q0, v0
    worst = 0.0
    for t in range(T):
        con = {"ncon": torch.zeros(s["nworld"], dtype=torch.int32, device="cuda")}
        q, v = model.step(q, v, tau=None if tau is None else tau[t].contiguous(), contacts=con)
        assert torch.equal(con["ncon"], ncon[t]), f"contact counts differ at step {t}"
        d = (v - vt[t + 1]).abs().max().item() / max(vt[t + 1].abs().max().item(), 1e-3)
        worst = max(worst, d)
        q, v = qt[t + 1].clone(), vt[t + 1].clone()  # continue from the rollout's state
    assert torch.equal(qt[0], q0) and torch.equal(vt[0], v0)
    return qt, vt, ncon, worst


@pytest.mark.parametrize("scene_fn", ["mixed", "articulated", "pile"])
def test_rollout_matches_steps_and_oracle(torch_cuda, scene_fn):
    """cf_rollout (one persistent kernel) against cf_step from each rollout state
    (same contact counts, velocities equal to float32 rounding) and against the
    oracle from sampled trajectory states (parity tolerance)."""
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    if scene_fn == "mixed":
        s = scenes.mixed_shapes(nworld=4, seed=11, condim=4)
    elif scene_fn == "articulated":
        s = scenes.articulated_mix(nworld=4, seed=2, condim=6)
    else:
        s = scenes.dense_pile(nworld=8, nsphere=64, seed=4, ncon_max=384)
    model = cfsim.Model(s)
    assert model.get_launch()[3], "expected the persistent rollout kernel"
    T = 120 if scene_fn != "pile" else 400
    tau = tdev(applied_wrench(s, np.random.default_rng(0), shape=(T,))) if scene_fn == "mixed" else None
    qt, vt, ncon, worst = _rollout_vs_steps(torch, model, s, T, tau)
    assert worst < 1e-6, f"rollout vs step relative difference {worst:.2e}"
    # against the oracle: two-step rollouts (persistent kernel) from states of
    # the oracle's own trajectory, first step compared
    o = Oracle(s)
    stats = None
    tau0 = None if tau is None else tau[0].cpu().numpy()
    for t, qi, vi in _oracle_states(s, T, tau0, record_every=max(1, T // 10)):
        tau2 = None if tau is None else tdev(np.stack([tau0, tau0]))
        q2, v2 = model.rollout(2, tdev(qi), tdev(vi), tau_seq=tau2)
        stats = compare_step(s, o, qi, vi, tau0, q2[1].cpu().numpy(), v2[1].cpu().numpy(), None,
                             stats=stats)
    print("rollout", scene_fn, stats, "contacts", int(ncon.sum()), "worst vs step", worst)


def test_rollout_full_pile_matches_steps(torch_cuda):
    """The benchmark's batch (4096 worlds x 64 spheres) through cf_rollout: more
    worlds than twelve per CU, so the free-body persistent kernel takes its
    four-waves-per-SIMD register sizing (the bench's launch); the trajectory
    and per-step contact counts equal repeated cf_step from each rollout state,
    from the lattice and from a settled state."""
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    s = scenes.dense_pile(nworld=4096, nsphere=64, seed=0)
    model = cfsim.Model(s)
    assert model.get_launch()[3], "expected the persistent rollout kernel"
    _, vt, ncon, worst = _rollout_vs_steps(torch, model, s, 30)
    assert worst < 1e-6, f"rollout vs step relative difference {worst:.2e}"
    q, v = tdev(s["q0"]), tdev(s["v0"])
    for _ in range(300):
        q, v = model.step(q, v)
    s2 = dict(s)
    s2["q0"], s2["v0"] = q.cpu().numpy(), v.cpu().numpy()
    _, vt2, ncon2, worst2 = _rollout_vs_steps(torch, model, s2, 30)
    assert worst2 < 1e-6, f"settled: rollout vs step relative difference {worst2:.2e}"
    assert float(ncon2.double().mean()) > 100, "the settled pile should hold its contacts"


@pytest.mark.parametrize("condim", [1, 3, 4, 6])
def test_one_kernel_step_equals_two_launches(torch_cuda, condim):
    """cf_step of worlds of free bodies at the one-wave launch shapes runs the
    narrow phase and the resolution in one kernel: against the two kernels
    (kernel timing on launches them apart), the contact set (counts, geom
    pairs, sub-indices) is identical and every float32 result equal to
    rounding, on a settled pile and on mixed shapes, at every condim.  The
    two forms run the same device functions in the same order, but compiled
    into different kernels the compiler may contract a multiply and an add
    into one fused operation in one and not the other, so the last bits of a
    result may differ."""
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    for s, settle in ((scenes.dense_pile(nworld=64, nsphere=64, seed=3, condim=condim), 300),
                      (scenes.mixed_shapes(nworld=8, seed=50 + condim, condim=condim), 20)):
        model = cfsim.Model(s)
        assert model.step_kernels() == 1
        q, v = tdev(s["q0"]), tdev(s["v0"])
        for _ in range(settle):
            q, v = model.step(q, v)
        print(f"case: one-kernel step {s['name']} condim {condim}", flush=True)
        c1 = model.alloc_contacts()
        q1, v1 = model.step(q, v, contacts=c1)
        model.set_profiling(True)
        assert model.step_kernels() == 2
        c2 = model.alloc_contacts()
        q2, v2 = model.step(q, v, contacts=c2)
        model.set_profiling(False)
        torch.cuda.synchronize()
        assert int(c1["ncon"].sum()) > 0
        for k in ("ncon", "overflow", "geom", "sub"):
            assert torch.equal(c1[k], c2[k]), k

        def close(a, b, rel=1e-6):
            return float((a - b).abs().max()) <= rel * max(float(a.abs().max()), 1.0)

        assert close(q1, q2) and close(v1, v2)
        for k in c1:
            if c1[k].is_floating_point():
                assert close(c1[k], c2[k], 1e-5), k
        print("bitwise equal:", bool(torch.equal(q1, q2) and torch.equal(v1, v2)))


@pytest.mark.parametrize("case", ["mix1", "mix3", "mix4", "mix6", "hand3", "hand6", "sib3", "sls6", "bob3",
                                  "hand6d", "mix3d"])
def test_one_kernel_articulated_step_equals_two_launches(torch_cuda, case):
    """cf_step of a model with articulated subtrees at the one-wave launch
    shapes runs the narrow phase (with the small subtrees' float64 frames)
    and the general resolution in one kernel: against the two kernels, along
    a trajectory with contacts (actuator targets on the hand), the contact
    set is identical and every float32 result equal to rounding (see the
    free-body test above for why not always bitwise).  A trailing "d": the
    exact diagonal impedance, compared from the states of the heuristic
    form's trajectory (articulated trajectories under the diagonal form leave
    the bounded regime, where rounding differences grow without bound)."""
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    diag = case.endswith("d")
    s, T, every, taus = _diag_articulated_case(case.rstrip("d"))
    traj = cfsim.Model(s)
    traj.set_launch(64, 64)
    if diag:
        sd = dict(s)
        sd["impedance"] = 1
        model = cfsim.Model(sd)
        model.set_launch(64, 64)
    else:
        model = traj
    assert model.step_kernels() == 1 and traj.step_kernels() == 1
    q, v = tdev(s["q0"]), tdev(s["v0"])
    print(f"case: one-kernel articulated step {case}", flush=True)
    checked = 0
    for t in range(T):
        tau = None if taus is None else tdev(taus[t])
        if t % every == 0:
            c1 = model.alloc_contacts()
            q1, v1 = model.step(q, v, tau=tau, contacts=c1)
            model.set_profiling(True)
            assert model.step_kernels() == 2
            c2 = model.alloc_contacts()
            q2, v2 = model.step(q, v, tau=tau, contacts=c2)
            model.set_profiling(False)
            torch.cuda.synchronize()
            for k in ("ncon", "overflow", "geom", "sub"):
                assert torch.equal(c1[k], c2[k]), (t, k)
            checked += int(c1["ncon"].sum())

            def close(a, b, rel=1e-6):
                return float((a - b).abs().max()) <= rel * max(float(a.abs().max()), 1.0)

            assert close(q1, q2) and close(v1, v2), t
            for k in c1:
                if c1[k].is_floating_point():
                    assert close(c1[k], c2[k], 1e-5), (t, k)
        q, v = traj.step(q, v, tau=tau)
    assert checked > 0
    print("contacts compared:", checked)


def test_rollout_graph_capture_replays(torch_cuda):
    """A stream capture of cf_rollout replays correctly: three replays with new
    initial states, eager work and synchronisations in between, each checked
    against an eager rollout."""
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    s = scenes.dense_pile(nworld=32, nsphere=32, seed=8, ncon_max=256)
    model = cfsim.Model(s)
    T = 50
    q_in, v_in = tdev(s["q0"]), tdev(s["v0"])
    q_traj = torch.empty((T + 1, s["nworld"], model.nq), device="cuda")
    v_traj = torch.empty((T + 1, s["nworld"], model.nv), device="cuda")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        model.rollout(T, q_in, v_in, q_traj=q_traj, v_traj=v_traj)  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        model.rollout(T, q_in, v_in, q_traj=q_traj, v_traj=v_traj)
    rng = np.random.default_rng(1)
    for rep in range(3):
        q0 = s["q0"].copy()
        q0.reshape(s["nworld"], -1, 7)[:, :, 2] += rng.uniform(0.0, 0.05)
        q_in.copy_(tdev(q0))
        v_in.copy_(tdev(s["v0"]))
        g.replay()
        torch.cuda.synchronize()
        qe, ve = model.rollout(T, tdev(q0), tdev(s["v0"]))
        torch.cuda.synchronize()
        assert torch.equal(qe, q_traj) and torch.equal(ve, v_traj), f"replay {rep} differs"
        _ = (q_in * 2).sum().item()  # unrelated eager work between replays


def test_autotune_picks_valid_launch(torch_cuda):
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    s = scenes.dense_pile(nworld=512, nsphere=64, seed=0)
    model = cfsim.Model(s)
    q, v = tdev(s["q0"]), tdev(s["v0"])
    for _ in range(200):
        q, v = model.step(q, v)
    us_step, us_roll = model.autotune(q, v, steps=10)
    cb, rb, ob, fused = model.get_launch()
    print(f"autotune: step {us_step:.1f} us ({cb}/{rb}), rollout {us_roll:.1f} us/step ({ob}, fused={fused})")
    assert us_step > 0 and cb in (64, 128, 256) and rb in (64, 128, 256) and ob in (64, 128, 256)
    q1, v1 = model.step(q, v)
    torch.cuda.synchronize()
    assert torch.isfinite(v1).all()


def test_kernel_timing_query(torch_cuda):
    from paper_2603_12185_amd import cfsim
    s = scenes.dense_pile(nworld=256, nsphere=64, seed=0)
    model = cfsim.Model(s)
    q, v = tdev(s["q0"]), tdev(s["v0"])
    model.set_profiling(True)
    t0 = time.time()
    for _ in range(20):
        q, v = model.step(q, v)
    a, b, n = model.kernel_times()
    print(f"collide {a / n * 1e3:.1f} us, resolve {b / n * 1e3:.1f} us per step; wall {time.time() - t0:.3f}s")
    assert n == 20 and a > 0 and b > 0
    model.set_profiling(False)
    # isolated back-to-back timing leaves the state untouched and gives the
    # same step as cf_step
    q0, v0 = q.clone(), v.clone()
    qo, vo = torch_cuda.empty_like(q), torch_cuda.empty_like(v)
    uc, ur = model.time_kernels(q, v, qo, vo, reps=10)
    torch_cuda.cuda.synchronize()
    assert uc > 0 and ur > 0
    assert torch_cuda.equal(q, q0) and torch_cuda.equal(v, v0)
    q1, v1 = model.step(q, v)
    assert torch_cuda.equal(q1, qo) and torch_cuda.equal(v1, vo)


# ---------------------------------------------------------------- articulated
@pytest.mark.parametrize("condim", [3, 6])
def test_articulated_mix_parity(torch_cuda, condim):
    """Hinge arm, slide-slide-hinge chain, floating base with hinged fingers and
    free spheres: per-subtree mass matrix, bias and Cholesky on the GPU; contacts
    on articulated links; 300 steps compared every 3."""
    from paper_2603_12185_amd import cfsim
    s = scenes.articulated_mix(nworld=6, seed=condim, condim=condim)
    model = cfsim.Model(s)
    print(f"case: articulated_mix condim {condim}", flush=True)
    recs = _run_steps(torch_cuda, model, s, 300, record_every=3)
    o = Oracle(s)
    stats = None
    for t, qi, vi, qg, vg, con in recs:
        stats = compare_step(s, o, qi, vi, None, qg, vg, con, stats=stats)
    print("articulated parity", condim, stats)
    assert stats["contacts"] > 500


def test_pendulum_and_double_pendulum_parity(torch_cuda):
    """Contact-free hinge chains: per-step parity over 2000 steps and the
    small-angle period of the GPU trajectory."""
    from paper_2603_12185_amd import cfsim
    import math
    for s in (scenes.pendulum(length=0.5, mass=1.0), scenes.double_pendulum()):
        s["q0"][0, 0] = 0.3
        model = cfsim.Model(s)
        recs = _run_steps(torch_cuda, model, s, 2000, record_every=50)
        o = Oracle(s)
        stats = None
        for t, qi, vi, qg, vg, con in recs:
            stats = compare_step(s, o, qi, vi, None, qg, vg, con, stats=stats)
        print(s["name"], stats)
    # period of a small-amplitude pendulum on the GPU
    s = scenes.pendulum(length=0.5, mass=1.0, h=0.0005)
    s["q0"][0, 0] = 0.01
    model = cfsim.Model(s)
    q, v = tdev(s["q0"]), tdev(s["v0"])
    th = []
    for _ in range(4000):
        q, v = model.step(q, v)
        th.append(float(q[0, 0]))
    th = np.array(th)
    cross = [i + th[i] / (th[i] - th[i + 1]) for i in range(len(th) - 1) if th[i] > 0 >= th[i + 1]]
    L = 0.5
    Ipiv = s["body_inertia"][0, 0, 1] + s["body_mass"][0, 0] * L * L
    T = 2 * math.pi * math.sqrt(Ipiv / (s["body_mass"][0, 0] * 9.81 * L))
    np.testing.assert_allclose((cross[1] - cross[0]) * s["h"], T, rtol=2e-3)


def test_slide_point_mass_stick_decay_on_gpu(torch_cuda):
    """The stick-regime decay of the sliding point mass (three slide joints), run
    on the GPU: u_{n+1} = (1 - 2 rho* a mu^2 / 3) u_n."""
    from paper_2603_12185_amd import cfsim
    mu = 0.5
    s = scenes.point_mass(mu=mu)
    g = 9.81
    a = s["k_user"] * s["h"] + s["d_user"]
    rho = s["solimp"][1] / (1 - s["solimp"][1])
    delta = (g * s["h"] / s["k_user"]) * (3 / (4 * rho) - a)
    s["q0"][0, 2] = s["geom_size"][0, 1, 0] - delta
    u1 = 3 * g * s["h"] / (4 * rho * a * mu)
    s["v0"][0, 0] = 0.5 * u1
    model = cfsim.Model(s)
    q, v = tdev(s["q0"]), tdev(s["v0"])
    mu32 = s["geom_friction"][0, 1, 0]
    fac = 1 - 2 * rho * a * mu32 * mu32 / 3
    u0 = float(s["v0"][0, 0])
    for n in range(1, 200):
        q, v = model.step(q, v)
        if n % 20 == 0:
            np.testing.assert_allclose(float(v[0, 0]), fac ** n * u0, rtol=2e-5)


# ---------------------------------------------------------------- exact diagonal impedance
@pytest.mark.parametrize("condim", [1, 3, 4, 6])
def test_diagonal_impedance_parity(torch_cuda, condim):
    """The exact diagonal impedance option (per-facet J~ M^-1 J~^T) against the
    oracle's.  The diagonal form resolves every facet as if it were alone, so
    coupled facets over-correct and frictional scenes leave the bounded regime
    within tens of steps: mixed shapes are compared on their first three
    states, the frictionless (condim 1) pile over 400 steps."""
    from paper_2603_12185_amd import cfsim
    s = scenes.mixed_shapes(nworld=4, seed=30 + condim, condim=condim)
    s["impedance"] = 1
    model = cfsim.Model(s)
    tau_np = applied_wrench(s, np.random.default_rng(condim))
    print(f"case: diagonal impedance mixed condim {condim}", flush=True)
    recs = _run_steps(torch_cuda, model, s, 3, tau=tau_np)
    o = Oracle(s)
    stats = None
    for t, qi, vi, qg, vg, con in recs:
        stats = compare_step(s, o, qi, vi, tau_np, qg, vg, con, stats=stats)
    print("diagonal impedance mixed", condim, stats)
    assert stats["contacts"] >= 3
    if condim == 1:
        p = scenes.dense_pile(nworld=4, nsphere=64, seed=9, ncon_max=512, condim=1)
        p["impedance"] = 1
        model = cfsim.Model(p)
        print("case: diagonal impedance dense pile condim 1", flush=True)
        recs = _run_steps(torch_cuda, model, p, 400, record_every=100)
        o = Oracle(p)
        stats = None
        for t, qi, vi, qg, vg, con in recs:
            stats = compare_step(p, o, qi, vi, None, qg, vg, con, stats=stats)
        print("diagonal impedance pile", stats)
        assert stats["contacts"] > 100


def _diag_articulated_case(case):
    """(scene, steps of the heuristic trajectory, every, tau schedule or None)."""
    kind, condim = case[:-1], int(case[-1])
    if kind == "mix":
        return scenes.articulated_mix(nworld=4, seed=40 + condim, condim=condim), 240, 8, None
    if kind == "hand":
        from test_gpu_hand import _target_schedule
        s = scenes.hand_cube(nworld=4, seed=40 + condim, condim=condim)
        return s, 240, 8, _target_schedule(s, 240, 40, 0.35, seed=condim)
    if kind in ("sib", "sls"):  # same-subtree contacts on a free carrier (general path) or a slide (small)
        return scenes.sibling_sliders(nworld=4, seed=condim, carrier="free" if kind == "sib" else "slide",
                                      axis2=(0.6, 0.8, 0.0), condim=condim), 40, 4, None
    return scenes.hinge_bob_on_plane(condim=condim), 40, 4, None


@pytest.mark.parametrize("case", ["mix1", "mix3", "mix4", "mix6", "hand3", "hand6", "sib3", "sib6", "sls3", "sls6",
                                  "bob3"])
def test_diagonal_impedance_articulated_parity(torch_cuda, case):
    """The exact diagonal impedance on articulated subtrees (each body's
    L^-1 J^T from the subtree's Cholesky factor, one row over the subtree's
    dofs when both bodies of a contact are in it) against the oracle's dense
    J~ M^-1 J~^T.  Resolving each facet as if alone over-corrects coupled
    facets, and an articulated trajectory under the diagonal form leaves the
    bounded regime within tens of steps, so every GPU step starts from a state
    of the oracle's heuristic trajectory (contacts present) and is compared
    with one oracle step of the diagonal form from the same state."""
    from paper_2603_12185_amd import cfsim
    s, T, every, taus = _diag_articulated_case(case)
    sd = dict(s)
    sd["impedance"] = 1
    model = cfsim.Model(sd)
    oh, od = Oracle(s), Oracle(sd)
    q, v = s["q0"].astype(np.float64), s["v0"].astype(np.float64)
    stats = None
    print(f"case: diagonal impedance articulated {case}", flush=True)
    for t in range(T):
        tau = None if taus is None else taus[t]
        if t % every == 0:
            q32, v32 = q.astype(np.float32), v.astype(np.float32)
            con = model.alloc_contacts()
            q1, v1 = model.step(tdev(q32), tdev(v32), tau=None if tau is None else tdev(tau), contacts=con)
            stats = compare_step(sd, od, q32, v32, tau, q1.cpu().numpy(), v1.cpu().numpy(), to_np(con),
                                 stats=stats)
        q, v, _ = oh.step(q, v, tau=None if tau is None else tau.astype(np.float64), outputs=False)
    print("diagonal impedance articulated", case, stats)
    assert stats["contacts"] >= (8 if case[:-1] in ("sib", "sls", "bob") else 40)


def test_diagonal_impedance_rules(torch_cuda):
    """An articulated model takes the diagonal impedance, an invalid mode is
    rejected; the adjoint takes a diagonal model of free bodies and refuses an
    articulated one."""
    from paper_2603_12185_amd import cfsim
    m = cfsim.Model(scenes.pendulum())
    m.set_impedance(1)
    q, v = tdev(scenes.pendulum()["q0"]), tdev(scenes.pendulum()["v0"])
    with pytest.raises(cfsim.CFError, match="UNSUPPORTED"):
        m.step_backward(q, v, None, q, v)
    m.set_impedance(0)
    m.step_backward(q, v, None, q, v)
    with pytest.raises(cfsim.CFError, match="INVALID"):
        m.set_impedance(7)
    s = scenes.mixed_shapes(nworld=1, seed=2)
    s["impedance"] = 1
    m = cfsim.Model(s)
    q, v = tdev(s["q0"]), tdev(s["v0"])
    gq, gv, gt = m.step_backward(q, v, None, q, v)
    import torch
    assert bool(torch.isfinite(gq).all() and torch.isfinite(gv).all() and torch.isfinite(gt).all())
