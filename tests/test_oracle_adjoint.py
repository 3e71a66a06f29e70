"""Pins of the oracle's Lennard-Jones adjoint (forces of section 4.1,
differentiated) against things other than itself: central finite differences
of the oracle's own forces and trajectories, an independent dense FP64
implementation differentiated by torch autograd, and exact identities
(homogeneity in eps; joint scaling of positions and sigma)."""
import numpy as np
import pytest
import torch

import oracle

EPS = (1.0, 1.5, 0.5)   # AA, AB, BB
SIG = (1.0, 0.8, 0.88)
RC = 2.5


def _system(nside=5, a=1.12, jitter=0.08, seed=0, mixture=True):
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(*[np.arange(nside)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5
    x = g * a + rng.uniform(-jitter, jitter, g.shape)
    L = np.full(3, nside * a)
    typ = rng.permutation(np.arange(len(x)) % 2).astype(np.int32) if mixture else None
    return x, L, typ


def _pairset(x, L, per, rc=RC):
    d = x[:, None, :] - x[None, :, :]
    for a in range(3):
        if per[a]:
            d[..., a] -= L[a] * np.rint(d[..., a] / L[a])
    r2 = (d ** 2).sum(-1)
    np.fill_diagonal(r2, np.inf)
    return r2 <= rc * rc


def _lamF(x, L, per, lam, typ, eps=EPS, sig=SIG):
    F, _ = oracle.lj_forces_f64(x, L, per, RC, eps, sig, typ)
    return float((lam * F).sum())


@pytest.mark.parametrize("per", [(1, 1, 1), (0, 0, 0)])
def test_vjp_positions_match_central_differences(per):
    x, L, typ = _system()
    rng = np.random.default_rng(1)
    lam = rng.normal(size=x.shape)
    gx, _ = oracle.lj_vjp_f64(x, L, per, RC, lam, EPS, SIG, typ)
    h = 1e-6
    base = _pairset(x, L, per)
    checked = 0
    for q in rng.choice(x.size, 40, replace=False):
        i, a = divmod(int(q), 3)
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        if not (np.array_equal(_pairset(xp, L, per), base) and
                np.array_equal(_pairset(xm, L, per), base)):
            continue  # the cut-off would be crossed: not differentiable here
        fd = (_lamF(xp, L, per, lam, typ) - _lamF(xm, L, per, lam, typ)) / (2 * h)
        assert abs(fd - gx[i, a]) <= 1e-6 * np.abs(gx).max(), (i, a, fd, gx[i, a])
        checked += 1
    assert checked >= 30


def test_vjp_parameters_match_central_differences():
    x, L, typ = _system(seed=2)
    per = (1, 1, 1)
    lam = np.random.default_rng(3).normal(size=x.shape)
    _, gt = oracle.lj_vjp_f64(x, L, per, RC, lam, EPS, SIG, typ)
    theta = np.array(EPS + SIG)
    for p in range(6):
        h = 1e-6 * theta[p]
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd = (_lamF(x, L, per, lam, typ, tp[:3], tp[3:]) -
              _lamF(x, L, per, lam, typ, tm[:3], tm[3:])) / (2 * h)
        assert abs(fd - gt[p]) <= 1e-6 * max(abs(gt[p]), 1e-3), (p, fd, gt[p])


def test_vjp_eps_homogeneity():
    # forces are linear in the well depths jointly: sum_p eps_p dL/deps_p = lam . F
    x, L, typ = _system(seed=4)
    per = (1, 1, 1)
    lam = np.random.default_rng(5).normal(size=x.shape)
    _, gt = oracle.lj_vjp_f64(x, L, per, RC, lam, EPS, SIG, typ)
    lhs = float(np.dot(EPS, gt[:3]))
    rhs = _lamF(x, L, per, lam, typ)
    assert abs(lhs - rhs) <= 1e-12 * (abs(rhs) + np.abs(gt).max())


@pytest.mark.parametrize("eps", [EPS, (1.0, 0.0, 0.5), (0.0, 0.0, 0.0)])
def test_vjp_eps_derivative_is_the_unit_depth_force(eps):
    # the force is linear in each well depth separately, so dL/deps_k is
    # lam . F with only the type-k pairs on, at unit depth, whatever eps is
    # (eps_k = 0 included, where the pair force itself vanishes)
    x, L, typ = _system(seed=8)
    per = (1, 1, 1)
    lam = np.random.default_rng(9).normal(size=x.shape)
    _, gt = oracle.lj_vjp_f64(x, L, per, RC, lam, eps, SIG, typ)
    for k in range(3):
        unit = tuple(1.0 if q == k else 0.0 for q in range(3))
        ref = _lamF(x, L, per, lam, typ, unit, SIG)
        assert abs(gt[k] - ref) <= 1e-12 * (abs(ref) + 1.0), (k, gt[k], ref)
    if eps[1] == 0.0:
        assert gt[1] != 0.0


def test_vjp_joint_scaling_of_positions_and_sigma():
    # each pair force s(u) r is homogeneous of degree -1 in (r, sigma) jointly, so
    # in an open box sum_k x_k . dL/dx_k + sum_p sig_p dL/dsig_p = -lam . F
    x, L, typ = _system(seed=6)
    per = (0, 0, 0)
    lam = np.random.default_rng(7).normal(size=x.shape)
    gx, gt = oracle.lj_vjp_f64(x, L, per, RC, lam, EPS, SIG, typ)
    lhs = float((x * gx).sum() + np.dot(SIG, gt[3:]))
    rhs = -_lamF(x, L, per, lam, typ)
    assert abs(lhs - rhs) <= 1e-10 * (np.abs(x * gx).sum() + np.abs(np.array(SIG) * gt[3:]).sum())


# --- independent dense implementation, differentiated by torch autograd ------

def _torch_forces(x, L, per, eps, sig, typ):
    d = x[:, None, :] - x[None, :, :]
    Lt = torch.as_tensor(L, dtype=torch.float64)
    pm = torch.as_tensor(per, dtype=torch.float64)
    d = d - pm * Lt * torch.round(d.detach() / Lt)
    u = (d * d).sum(-1)
    n = x.shape[0]
    mask = (u.detach() <= RC * RC) & ~torch.eye(n, dtype=torch.bool)
    t = torch.as_tensor(typ, dtype=torch.long)
    k = t[:, None] + t[None, :]
    e, s_ = eps[k], sig[k]
    us = torch.where(mask, u, torch.ones_like(u))
    s = 24 * e * (2 * s_ ** 12 / us ** 7 - s_ ** 6 / us ** 4)
    s = torch.where(mask, s, torch.zeros_like(s))
    return (s[..., None] * d).sum(1)


def test_vjp_matches_torch_autograd_of_dense_forces():
    x, L, typ = _system(seed=8)
    per = (1, 1, 1)
    lam = np.random.default_rng(9).normal(size=x.shape)
    xt = torch.tensor(x, requires_grad=True)
    et = torch.tensor(EPS, dtype=torch.float64, requires_grad=True)
    st = torch.tensor(SIG, dtype=torch.float64, requires_grad=True)
    F = _torch_forces(xt, L, per, et, st, typ)
    F_or, _ = oracle.lj_forces_f64(x, L, per, RC, EPS, SIG, typ)
    assert np.abs(F.detach().numpy() - F_or).max() <= 1e-10 * np.abs(F_or).max()
    (F * torch.as_tensor(lam)).sum().backward()
    gx, gt = oracle.lj_vjp_f64(x, L, per, RC, lam, EPS, SIG, typ)
    assert np.abs(xt.grad.numpy() - gx).max() <= 1e-10 * np.abs(gx).max()
    ref = np.concatenate([et.grad.numpy(), st.grad.numpy()])
    assert np.abs(ref - gt).max() <= 1e-10 * np.abs(gt).max()


def test_vjp_fp32_set_variant_agrees_with_fp64_variant():
    x, L, typ = _system(seed=10)
    x32 = x.astype(np.float32)
    L32 = L.astype(np.float32)
    per = (1, 1, 1)
    x64 = x32.astype(np.float64)
    lam = np.random.default_rng(11).normal(size=x.shape)
    g32, t32 = oracle.lj_vjp(x32, L32, per, np.float32(RC * RC), lam, EPS, SIG, typ)
    g64, t64 = oracle.lj_vjp_f64(x64, L32.astype(np.float64), per, RC, lam, EPS, SIG, typ)
    assert np.abs(g32 - g64).max() <= 1e-11 * np.abs(g64).max()
    assert np.abs(t32 - t64).max() <= 1e-11 * np.abs(t64).max()


# --- trajectories -------------------------------------------------------------

def _velocities(n, seed, T=1.0):
    v = np.random.default_rng(seed).normal(0.0, np.sqrt(T), (n, 3))
    return v - v.mean(0)


def _traj_loss(x0, v0, L, per, dt, K, frames, targets, typ, eps=EPS, sig=SIG):
    xs, Fs, _ = oracle.lj_traj(x0, v0, L, per, RC, dt, K, eps, sig, typ)
    n = len(x0)
    loss = sum(((Fs[k] - targets[q]) ** 2).sum() for q, k in enumerate(frames))
    return loss / (3 * n * len(frames)), xs, Fs


def _fbar(Fs, frames, targets):
    K1, n, _ = Fs.shape
    fb = np.zeros_like(Fs)
    for q, k in enumerate(frames):
        fb[k] = 2.0 * (Fs[k] - targets[q]) / (3 * n * len(frames))
    return fb


def _traj_problem(seed=12, K=24, frames=(8, 16, 24)):
    x0, L, typ = _system(seed=seed)
    per = (1, 1, 1)
    v0 = _velocities(len(x0), seed + 1)
    dt = 0.005
    tgt_eps = tuple(1.05 * e for e in EPS)
    tgt_sig = tuple(1.05 * s for s in SIG)
    _, Ft, _ = oracle.lj_traj(x0, v0, L, per, RC, dt, K, tgt_eps, tgt_sig, typ)
    targets = [Ft[k] for k in frames]
    return x0, v0, L, per, typ, dt, K, list(frames), targets


def test_trajectory_adjoint_matches_central_differences():
    x0, v0, L, per, typ, dt, K, frames, targets = _traj_problem()
    loss, xs, Fs = _traj_loss(x0, v0, L, per, dt, K, frames, targets, typ)
    xb, vb, gt = oracle.lj_traj_adjoint(xs, L, per, RC, dt, _fbar(Fs, frames, targets), EPS,
                                        SIG, typ)

    def sets(xs_):
        return [_pairset(x, L, per) for x in xs_]

    base = sets(xs)
    rng = np.random.default_rng(13)
    h = 1e-6
    checked = 0
    for which, grad in (("x", xb), ("v", vb)):
        for q in rng.choice(x0.size, 12, replace=False):
            i, a = divmod(int(q), 3)
            res = []
            ok = True
            for sgn in (1, -1):
                xx, vv = x0.copy(), v0.copy()
                (xx if which == "x" else vv)[i, a] += sgn * h
                lo, xs_, _ = _traj_loss(xx, vv, L, per, dt, K, frames, targets, typ)
                ok &= all(np.array_equal(p, q_) for p, q_ in zip(sets(xs_), base))
                res.append(lo)
            if not ok:
                continue
            fd = (res[0] - res[1]) / (2 * h)
            assert abs(fd - grad[i, a]) <= 2e-5 * np.abs(grad).max(), (which, i, a, fd, grad[i, a])
            checked += 1
    assert checked >= 16
    theta = np.array(EPS + SIG)
    for p in range(6):
        hp = 1e-6 * theta[p]
        res = []
        for sgn in (1, -1):
            t = theta.copy()
            t[p] += sgn * hp
            lo, xs_, _ = _traj_loss(x0, v0, L, per, dt, K, frames, targets, typ, t[:3], t[3:])
            res.append(lo)
        fd = (res[0] - res[1]) / (2 * hp)
        assert abs(fd - gt[p]) <= 2e-5 * np.abs(gt).max(), (p, fd, gt[p])


def test_trajectory_adjoint_matches_torch_autograd():
    x0, v0, L, per, typ, dt, K, frames, targets = _traj_problem(seed=20, K=12, frames=(6, 12))
    loss, xs, Fs = _traj_loss(x0, v0, L, per, dt, K, frames, targets, typ)
    xb, vb, gt = oracle.lj_traj_adjoint(xs, L, per, RC, dt, _fbar(Fs, frames, targets), EPS,
                                        SIG, typ)
    xt = torch.tensor(x0, requires_grad=True)
    vt = torch.tensor(v0, requires_grad=True)
    et = torch.tensor(EPS, dtype=torch.float64, requires_grad=True)
    st = torch.tensor(SIG, dtype=torch.float64, requires_grad=True)
    Lt = torch.as_tensor(L)
    x, v = xt, vt
    F = _torch_forces(x, L, per, et, st, typ)
    n = len(x0)
    tl = torch.zeros((), dtype=torch.float64)
    for k in range(1, K + 1):
        v = v + 0.5 * dt * F
        x = x + dt * v
        x = x - Lt * torch.floor(x.detach() / Lt)
        F = _torch_forces(x, L, per, et, st, typ)
        v = v + 0.5 * dt * F
        if k in frames:
            tl = tl + ((F - torch.as_tensor(targets[frames.index(k)])) ** 2).sum()
    tl = tl / (3 * n * len(frames))
    assert abs(float(tl.detach()) - loss) <= 1e-10 * loss
    tl.backward()
    assert np.abs(xt.grad.numpy() - xb).max() <= 1e-9 * np.abs(xb).max()
    assert np.abs(vt.grad.numpy() - vb).max() <= 1e-9 * np.abs(vb).max()
    ref = np.concatenate([et.grad.numpy(), st.grad.numpy()])
    assert np.abs(ref - gt).max() <= 1e-9 * np.abs(gt).max()


def test_trajectory_adjoint_of_zero_steps_is_the_force_vjp():
    x0, L, typ = _system(seed=30)
    per = (1, 1, 1)
    lam = np.random.default_rng(31).normal(size=x0.shape)
    xb, vb, gt = oracle.lj_traj_adjoint(x0[None], L, per, RC, 0.005, lam[None], EPS, SIG, typ)
    gx, gt1 = oracle.lj_vjp_f64(x0, L, per, RC, lam, EPS, SIG, typ)
    assert np.array_equal(xb, gx) and np.array_equal(gt, gt1)
    assert not vb.any()


# --- trajectories with FP32 particle state -----------------------------------

def _f32_problem(seed=40, K=40):
    x0, L, typ = _system(seed=seed)
    v0 = _velocities(len(x0), seed + 1)
    return (x0.astype(np.float32), v0.astype(np.float32), L.astype(np.float32), (1, 1, 1), typ,
            K)


def test_fp32_state_trajectory_follows_fp64_trajectory():
    x32, v32, L32, per, typ, K = _f32_problem()
    xs, vs, Fs, nb = oracle.lj_traj_f32(x32, v32, L32, per, RC * RC, 0.005, K, 0.15 ** 2, 0,
                                        EPS, SIG, typ)
    xs64, Fs64, vs64 = oracle.lj_traj(x32.astype(np.float64), v32.astype(np.float64),
                                      L32.astype(np.float64), per, RC, 0.005, K, EPS, SIG, typ)
    for k in (1, K // 2, K):
        d = xs[k].astype(np.float64) - xs64[k]
        d -= L32 * np.round(d / L32)
        assert np.abs(d).max() < 1e-5, k
        assert np.abs(vs[k] - vs64[k]).max() < 1e-4, k
        assert np.abs(Fs[k] - Fs64[k]).max() < 1e-3 * np.abs(Fs64[k]).max(), k


def test_fp32_state_wraps_only_at_rebuilds():
    x32, v32, L32, per, typ, K = _f32_problem(seed=42, K=30)
    v32 = v32 + np.float32([-4.0, 0.0, 0.0])  # a common drift: many leave through x = 0
    always = oracle.lj_traj_f32(x32, v32, L32, per, RC * RC, 0.005, K, 0.0, 0, EPS, SIG, typ)
    never = oracle.lj_traj_f32(x32, v32, L32, per, RC * RC, 0.005, K, 1e30, 0, EPS, SIG, typ)
    every = oracle.lj_traj_f32(x32, v32, L32, per, RC * RC, 0.005, K, 1e30, 7, EPS, SIG, typ)
    assert always[3] == K + 1 and never[3] == 1 and every[3] == 1 + (K - 1) // 7
    xa, xn = always[0], never[0]
    assert xa.min() >= 0 and np.all(xa < L32)                 # wrapped at every step
    assert xn.min() < 0 or np.any(xn >= L32)                  # some particle left the box
    d = xn.astype(np.float64) - xa
    assert np.abs(d - L32 * np.round(d / L32)).max() < 1e-5   # same motion modulo L


def test_fp32_state_adjoint_equals_fp64_adjoint_on_the_same_states():
    x32, v32, L32, per, typ, K = _f32_problem(seed=44, K=20)
    xs, vs, Fs, nb = oracle.lj_traj_f32(x32, v32, L32, per, RC * RC, 0.005, K, 0.15 ** 2, 0,
                                        EPS, SIG, typ)
    fb = np.random.default_rng(45).normal(size=xs.shape) * 1e-3
    dt = float(np.float32(0.005))
    a = oracle.lj_traj_adjoint_f32(xs, L32, per, RC * RC, dt, fb, EPS, SIG, typ)
    b = oracle.lj_traj_adjoint(xs.astype(np.float64), L32.astype(np.float64), per, RC, dt, fb,
                               EPS, SIG, typ)
    for u, w in zip(a, b):
        assert np.abs(u - w).max() <= 1e-10 * np.abs(w).max()
