"""Two further references for the checkpointed trajectory adjoint (a
force-matching loss over frames of a velocity-Verlet trajectory of the binary
LJ mixture, gradients for x0, v0 and theta):

(i)  the FP64 reverse sweep replayed on the GPU's own forward states: the
     positions the GPU reached at every step are recorded, and the oracle's
     adjoint runs on them, once on the FP32 pair set of each state and once
     with the FP64 cut-off test u <= rc^2.  Both must match the GPU gradients
     to the parity bar (the GPU forward and backward run through the same
     pair sets, so only FP64 summation order and the FP32 rounding of the
     forward state separate them);
(ii) a fully FP64 end-to-end run (FP64 forward trajectory, FP64 adjoint):
     the GPU gradient's distance to it grows with the trajectory length, since
     the FP32 trajectory separates from the FP64 one exponentially (the
     dynamics are chaotic).  Reported against the length, not asserted."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1804_07598_amd import inputs

pytestmark = pytest.mark.gpu

RC, SKIN, PER = 2.5, 0.3, (1, 1, 1)
MIX = inputs.LJ_MIXTURE
TOL = 1e-5


def np_(t):
    return t.detach().cpu().numpy()


def rel_max(g, ref):
    return float(np.abs(g - ref).max() / math.sqrt((ref ** 2).mean()))


def gpu_case(n, K, frame_every, ckpt_every, seed=5, zero_targets=False):
    """GPU gradients of the frame-averaged force MSE (targets from the FP64
    oracle trajectory at theta_tgt = 1.05 theta, or zero), the GPU's frame
    forces, and the GPU's positions at every step of the same forward pass
    (recorded by repeating it step by step with the same rebuilds at the
    checkpoints)."""
    import torch
    from paper_1804_07598_amd.adjoint import LJTrajFn
    from paper_1804_07598_amd.sim import ParticleSim
    s = inputs.lj_lattice(n, 1.2, 1.0, seed, mixture=True)
    dt = np.float32(0.005)
    theta = np.float32(np.array(MIX["eps"] + MIX["sig"])).astype(np.float64)
    theta_t = 1.05 * theta
    frames = list(range(frame_every, K + 1, frame_every))
    if zero_targets:
        targets = np.zeros((len(frames), n, 3))
    else:
        _, Ft, _ = O.lj_traj(s.pos, s.vel, s.box, PER, RC, float(dt), K, theta_t[:3],
                             theta_t[3:], s.typ)
        targets = np.stack([Ft[k] for k in frames])
    sim = ParticleSim(s.pos, s.box, PER, vel=s.vel, typ=s.typ, r_cut=RC, skin=SKIN)
    x0 = torch.tensor(s.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    v0 = torch.tensor(s.vel, dtype=torch.float64, device="cuda", requires_grad=True)
    th = torch.tensor(theta, device="cuda", requires_grad=True)
    Fk = LJTrajFn.apply(x0, v0, th, sim, float(dt), K, frame_every, ckpt_every, 2)
    loss = ((Fk - torch.tensor(targets, device="cuda")) ** 2).mean()
    loss.backward()
    grads = (np_(x0.grad), np_(v0.grad), np_(th.grad))
    # the forward again, one step at a time, recording positions
    eps, sig = tuple(theta[:3]), tuple(theta[3:])
    sim.set_particles(s.pos, s.vel)
    xs = np.empty((K + 1, n, 3), np.float32)
    xs[0] = s.pos
    for k in range(K):
        if k > 0 and k % ckpt_every == 0:
            sim.build_verlet()
        sim.step(1, dt=float(dt), eps=eps, sig=sig, n_types=2)
        xs[k + 1] = np_(sim.get()[0])
    sim.check()
    sim.close()
    fbar = np.zeros((K + 1, n, 3), np.float64)
    Fk = np_(Fk)
    for q, k in enumerate(frames):
        fbar[k] = 2.0 * (Fk[q] - targets[q]) / targets.size
    return s, theta, dt, frames, targets, grads, xs, fbar


@pytest.mark.parametrize("n,K,fe,ce", [(2048, 40, 20, 20), (1500, 60, 20, 20),
                                      (1024, 200, 20, 20)])
def test_fp64_adjoint_on_gpu_states(n, K, fe, ce):
    s, theta, dt, frames, targets, (gx, gv, gt), xs, fbar = gpu_case(n, K, fe, ce)
    # FP64 sweep on the FP32 pair set of each recorded state
    ox, ov, ot = O.lj_traj_adjoint_f32(xs, s.box, PER, O.radius2(RC), float(dt), fbar,
                                       theta[:3], theta[3:], s.typ)
    assert rel_max(gx, ox) <= TOL and rel_max(gv, ov) <= TOL
    assert np.all(np.abs(gt - ot) <= TOL * np.abs(ot)), (gt, ot)
    # the FP64 oracle adjoint (FP64 cut-off test) on the same states
    px, pv, pt = O.lj_traj_adjoint(xs.astype(np.float64), s.box, PER, RC, float(dt), fbar,
                                   theta[:3], theta[3:], s.typ)
    print(f"n={n} K={K}: vs FP32-set sweep x {rel_max(gx, ox):.2e} v {rel_max(gv, ov):.2e}; "
          f"vs FP64-cut-off sweep x {rel_max(gx, px):.2e} v {rel_max(gv, pv):.2e} "
          f"theta {np.max(np.abs(gt - pt) / np.abs(pt)):.2e}")
    assert rel_max(gx, px) <= TOL and rel_max(gv, pv) <= TOL
    assert np.all(np.abs(gt - pt) <= TOL * np.abs(pt)), (gt, pt)


def test_fp64_adjoint_on_gpu_states_full_size_segment():
    """The bench's configuration (32,768-atom mixture, checkpoints and loss
    frames every 20 steps), one segment: the FP64 sweep on the FP32 pair sets
    of the GPU's own states against the GPU gradients (loss: mean squared
    frame force, so no FP64 trajectory is needed for targets)."""
    s, theta, dt, frames, targets, (gx, gv, gt), xs, fbar = gpu_case(32768, 20, 20, 20,
                                                                      zero_targets=True)
    ox, ov, ot = O.lj_traj_adjoint_f32(xs, s.box, PER, O.radius2(RC), float(dt), fbar,
                                       theta[:3], theta[3:], s.typ)
    print(f"n=32768 K=20: x {rel_max(gx, ox):.2e} v {rel_max(gv, ov):.2e} "
          f"theta {np.max(np.abs(gt - ot) / np.abs(ot)):.2e}")
    assert rel_max(gx, ox) <= TOL and rel_max(gv, ov) <= TOL
    assert np.all(np.abs(gt - ot) <= TOL * np.abs(ot)), (gt, ot)


def test_report_fp64_end_to_end_error_vs_length():
    """(ii): printed, not asserted (beyond finiteness)."""
    rows = []
    for K in (10, 20, 40, 80, 160):
        s, theta, dt, frames, targets, (gx, gv, gt), xs, _ = gpu_case(1024, K, min(10, K), 20)
        x64, F64, v64 = O.lj_traj(s.pos, s.vel, s.box, PER, RC, float(dt), K, theta[:3],
                                  theta[3:], s.typ)
        fbar = np.zeros(x64.shape, np.float64)
        for q, k in enumerate(frames):
            fbar[k] = 2.0 * (F64[k] - targets[q]) / targets.size
        ex, ev, et = O.lj_traj_adjoint(x64, s.box, PER, RC, float(dt), fbar, theta[:3],
                                       theta[3:], s.typ)
        d = xs[-1].astype(np.float64) - x64[-1]
        d -= s.box.astype(np.float64) * np.round(d / s.box.astype(np.float64))  # minimum image
        dx = float(np.abs(d).max())
        rows.append((K, dx, rel_max(gx, ex), rel_max(gv, ev), float(np.max(np.abs(gt - et) /
                                                                            np.abs(et)))))
        assert np.isfinite(gx).all() and np.isfinite(gt).all()
    print("\nK   max|x_gpu - x_fp64|   dL/dx0 err (of RMS)   dL/dv0 err   dL/dtheta err (rel)")
    for r in rows:
        print(f"{r[0]:<4d}{r[1]:>12.2e}{r[2]:>20.2e}{r[3]:>15.2e}{r[4]:>18.2e}")
