"""GPU parity of the actuated hand-and-cube scene (16 hinge dofs in four
subtrees, capsule links, fingertip spheres, box-capsule / box-sphere /
plane contacts, 6D friction) against the FP64 oracle, its batched rollouts,
and the MPPI controller built on them.  All tests need an MI355X.
"""
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


def _target_schedule(s, nsteps, every, amp, seed):
    """Finger targets [nsteps][nw][nv]: the initial pose plus a uniform offset
    redrawn every `every` steps."""
    rng = np.random.default_rng(seed)
    base = scenes.hand_targets(s)
    out = np.empty((nsteps,) + base.shape, np.float32)
    cur = base.copy()
    for t in range(nsteps):
        if t % every == 0 and t > 0:
            cur = base.copy()
            cur[:, 6:] += rng.uniform(-amp, amp, cur[:, 6:].shape).astype(np.float32)
        out[t] = cur
    return out


@pytest.mark.parametrize("condim", [3, 6])
def test_hand_parity(torch_cuda, condim):
    """One GPU step from each recorded state of the oracle's own trajectory
    (targets redrawn every 40 steps), compared with the oracle's step."""
    from paper_2603_12185_amd import cfsim
    s = scenes.hand_cube(nworld=4, seed=condim, condim=condim)
    model = cfsim.Model(s)
    o = Oracle(s)
    T = 400
    taus = _target_schedule(s, T, 40, 0.35, seed=condim)
    q, v = s["q0"].astype(np.float64), s["v0"].astype(np.float64)
    stats = None
    box_contacts = 0
    print(f"case: hand_cube condim {condim}", flush=True)
    for t in range(T):
        q32, v32, tau = q.astype(np.float32), v.astype(np.float32), taus[t]
        if t % 4 == 0:
            con = model.alloc_contacts()
            q1, v1 = model.step(tdev(q32), tdev(v32), tau=tdev(tau), contacts=con)
            c = to_np(con)
            stats = compare_step(s, o, q32, v32, tau, q1.cpu().numpy(), v1.cpu().numpy(), c, stats=stats)
            for w in range(s["nworld"]):
                ga = c["geom"][w, :c["ncon"][w], 0]
                box_contacts += int((s["geom_type"][ga] == scenes.BOX).sum())
        q, v, _ = o.step(q, v, tau=tau.astype(np.float64), outputs=False)
    print("hand parity", condim, stats, "box contacts", box_contacts)
    assert stats["contacts"] > 200 and box_contacts > 20


def test_hand_full_size_sampled(torch_cuda):
    """The hand's batch at full size (2048 worlds, condim 6) in the launch
    shape the bench's autotuner picks for it (one wave per world, one kernel
    per step): every world driven by its own target schedule; at steps 60, 120
    and 199 the sampled worlds take the oracle's own trajectory states and
    their step is compared with the oracle's; every world stays finite and
    within its contact capacity."""
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    s = scenes.hand_cube(nworld=2048, seed=5, condim=6)
    model = cfsim.Model(s)
    model.set_launch(64, 64)
    assert model.step_kernels() == 1
    T, checks = 200, (60, 120, 199)
    taus = _target_schedule(s, T, 40, 0.35, seed=5)
    sample = [0, 1, 1023, 2047]
    ss = scenes.select_worlds(s, sample)
    o = Oracle(ss)
    print("case: hand_cube 2048 worlds full size", flush=True)
    qo, vo = ss["q0"].astype(np.float64), ss["v0"].astype(np.float64)
    ostates = {}
    for t in range(T):
        if t in checks:
            ostates[t] = (qo.astype(np.float32), vo.astype(np.float32))
        qo, vo, _ = o.step(qo, vo, tau=taus[t][sample].astype(np.float64), outputs=False)
    idx = torch.tensor(sample, device="cuda")
    q, v = tdev(s["q0"]), tdev(s["v0"])
    stats = None
    for t in range(T):
        con = None
        tau = tdev(taus[t])
        if t in checks:
            con = model.alloc_contacts()
            q[idx], v[idx] = tdev(ostates[t][0]), tdev(ostates[t][1])
        q1, v1 = model.step(q, v, tau=tau, contacts=con)
        if con is not None:
            c = to_np(con)
            assert (c["ncon"] <= s["ncon_max"]).all() and (c["overflow"] == 0).all()
            qn, vn = q1.cpu().numpy(), v1.cpu().numpy()
            assert np.isfinite(qn).all() and np.isfinite(vn).all()
            sub = {k: val[sample] for k, val in c.items()}
            stats = compare_step(ss, o, ostates[t][0], ostates[t][1], taus[t][sample], qn[sample], vn[sample],
                                 sub, stats=stats)
            print(f"step {t}: mean contacts/world {c['ncon'].mean():.2f} max {c['ncon'].max()}")
        q, v = q1, v1
    torch.cuda.synchronize()
    print("hand full-size sampled parity", stats)
    assert stats["checked"] >= len(checks) * len(sample) // 2 and stats["contacts"] > 0


def test_hand_rollout_matches_steps(torch_cuda):
    """cf_rollout with per-step finger targets (persistent kernel) against
    cf_step from every rollout state: same contact counts, velocities equal to
    float32 rounding."""
    from paper_2603_12185_amd import cfsim
    torch = torch_cuda
    s = scenes.hand_cube(nworld=64, seed=9)
    model = cfsim.Model(s)
    assert model.get_launch()[3], "expected the persistent rollout kernel"
    T = 100
    tau = tdev(_target_schedule(s, T, 10, 0.2, seed=4))
    q0, v0 = tdev(s["q0"]), tdev(s["v0"])
    ncon = torch.zeros((T, s["nworld"]), dtype=torch.int32, device="cuda")
    over = torch.full((T, s["nworld"]), -1, dtype=torch.int32, device="cuda")
    qt, vt = model.rollout(T, q0, v0, tau_seq=tau, ncon_traj=ncon, overflow_traj=over)
    assert int(over.abs().sum()) == 0, "contact capacity overflowed in the rollout"
    worst = 0.0
    for t in range(T):
        con = {"ncon": torch.zeros(s["nworld"], dtype=torch.int32, device="cuda")}
        q, v = model.step(qt[t].clone(), vt[t].clone(), tau=tau[t].contiguous(), contacts=con)
        assert torch.equal(con["ncon"], ncon[t]), f"contact counts differ at step {t}"
        worst = max(worst, (v - vt[t + 1]).abs().max().item() / max(vt[t + 1].abs().max().item(), 1e-3))
    print("hand rollout vs steps: worst relative velocity difference", worst,
          "contacts per world-step", float(ncon.double().mean()))
    assert worst < 1e-5
    assert int(ncon.max()) > 0


def test_actuators_validation(torch_cuda):
    from paper_2603_12185_amd import cfsim
    s = scenes.hand_cube(nworld=2)
    model = cfsim.Model(s)
    bad = np.zeros(model.nv, np.float32)
    bad[0] = 1.0  # the cube's free dof
    with pytest.raises(cfsim.CFError):
        model.set_actuators(bad, None)
    with pytest.raises(cfsim.CFError):
        model.set_actuators(np.full(model.nv, -1.0, np.float32), None)
    model.set_actuators(None, None)  # removes them: the input is a force again
    q, v = tdev(s["q0"]), tdev(s["v0"])
    q1, v1 = model.step(q, v)
    assert bool(torch_cuda.isfinite(v1).all())


def test_mppi_iteration(torch_cuda):
    """MPPI with 256 rollouts of 20 steps: the weights are a distribution, the
    nominal sequence moves by the weighted noise, the plant stays finite, and
    the cube turns toward the target yaw over 150 iterations."""
    from paper_2603_12185_amd import mpc
    torch = torch_cuda
    ctl = mpc.HandMPPI(nroll=256, H=20, sigma=0.1, target_yaw=0.4, seed=1)
    yaw0 = ctl.cube_yaw()
    costs = []
    for it in range(150):
        costs.append(ctl.iterate())
        if it % 50 == 0:
            print(f"  mppi iteration {it}: weighted cost {costs[-1]:.4f}, yaw {ctl.cube_yaw():.4f}", flush=True)
    torch.cuda.synchronize()
    assert all(np.isfinite(costs)) and bool(torch.isfinite(ctl.q).all())
    print("mppi: yaw", yaw0, "->", ctl.cube_yaw(), "cost", costs[0], "->", costs[-1])
    assert ctl.cube_yaw() - yaw0 > 0.02
