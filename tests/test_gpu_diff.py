"""The differentiable quadrotor edge rollout (kpx_diff_* through the C ABI)
against the float64 oracle: per-edge losses, the adjoint gradient against the
oracle's complex-step gradient and against central differences of the GPU's
own loss, checkpoint-boundary and degenerate edges, the autograd wrapper, and
projected-gradient polishing step by step.

Tolerances, derived from float32 arithmetic over at most 40 RK4 steps: the
loss is a sum of O(40) terms of size up to ~20 (the thrust effort), each
carrying a few float32 roundings (2^-24 ~ 6e-8) amplified by the rollout's
sensitivity, so 1e-5 relative to max(1, |L|) leaves an order of magnitude of
margin.  The gradient is compared per edge in the max norm, relative 1e-4 of
the oracle gradient's max norm (the bound asked of the adjoint).  Central
differences with h = 1e-3 are held to 1e-3 relative against the float64
oracle loss on the CPU (test_oracle_diff); differences of the float32 GPU loss
carry the loss's own rounding, a few tens of ulp(L) for a sum of ~60 terms,
divided by h, so here they get 1e-3 of the gradient's norm plus 16 ulp(L) / h:
a check of the adjoint's sign and size against the kernel's own forward."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

E_PARITY = 1000  # several 256-edge tiles and a ragged tail
LR = 0.01


@pytest.fixture(scope="module")
def kpx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_02846_amd as K

    K.lib()
    return K


def _dev(x0, u, n):
    import torch

    return (torch.from_numpy(np.ascontiguousarray(x0.T)).cuda(),
            torch.from_numpy(np.ascontiguousarray(u.T)).cuda(),
            torch.from_numpy(np.ascontiguousarray(n, dtype=np.int32)).cuda())


def _run(R, x0, u, n, want_grad=True):
    import torch

    xd, ud, nd = _dev(x0, u, n)
    loss, grad = R.loss_grad(xd, ud, nd, want_grad)
    torch.cuda.synchronize()
    return loss.cpu().numpy(), (grad.cpu().numpy().T if grad is not None else None)


@pytest.fixture(scope="module")
def scene(kpx, ora):
    from paper_2602_02846_amd.diff import Rollout

    b = W.diff_workload(0, n_edges=E_PARITY)
    return b, Rollout(b.problem, b.dt), ora.DiffProblem(b.problem, b.dt)


def _check_loss(ora, D, b, loss, idx):
    for e in idx:
        ref = ora.diff_loss(D, b.x0[e], b.u[e], int(b.n[e]))
        assert abs(loss[e] - ref) <= 1e-5 * max(1.0, abs(ref)), (e, loss[e], ref)


def _check_grad(ora, D, x0, u, n, grad, idx, rel=1e-4):
    worst = 0.0
    for e in idx:
        ref = ora.diff_grad(D, x0[e], u[e], int(n[e]))
        err = np.max(np.abs(grad[e] - ref)) / np.max(np.abs(ref))
        worst = max(worst, err)
        assert err <= rel, (e, int(n[e]), err, grad[e], ref)
    return worst


def test_loss_matches_oracle(scene, ora):
    b, R, D = scene
    loss, grad = _run(R, b.x0, b.u, b.n)
    loss_only, none = _run(R, b.x0, b.u, b.n, want_grad=False)
    assert none is None
    np.testing.assert_array_equal(loss, loss_only)
    _check_loss(ora, D, b, loss, range(E_PARITY))


def test_gradient_matches_oracle(scene, ora):
    b, R, D = scene
    _, grad = _run(R, b.x0, b.u, b.n)
    worst = _check_grad(ora, D, b.x0, b.u, b.n, grad, range(0, E_PARITY, 3))
    print(f"max-norm relative gradient error {worst:.2e}")


def test_gradient_matches_central_differences_of_the_gpu_loss(scene):
    b, R, _ = scene
    idx = np.arange(0, 64)
    _, grad = _run(R, b.x0[idx], b.u[idx], b.n[idx])
    h = np.float32(1e-3)
    E = len(idx)
    # one launch per sign and control: the +-h copies of all edges side by side
    x0 = np.repeat(b.x0[idx][None], 32, 0).reshape(-1, 12)
    n = np.repeat(b.n[idx][None], 32, 0).reshape(-1)
    u = np.repeat(b.u[idx][None], 32, 0).reshape(32, E, 16)
    for j in range(16):
        u[2 * j, :, j] += h
        u[2 * j + 1, :, j] -= h
    loss, _ = _run(R, x0, u.reshape(-1, 16), n, want_grad=False)
    loss = loss.reshape(32, E).astype(np.float64)
    step = (u[0::2, :, :] - u[1::2, :, :])[np.arange(16), :, np.arange(16)].astype(np.float64)
    fd = ((loss[0::2] - loss[1::2]) / step).T  # E x 16
    for e in range(E):
        floor = 16 * np.spacing(np.float32(max(1.0, abs(loss[0, e])))) / float(h)
        err = np.max(np.abs(fd[e] - grad[e]))
        assert err <= 1e-3 * np.max(np.abs(grad[e])) + floor, (e, err, fd[e], grad[e])


@pytest.mark.parametrize("n", [4, 5, 7, 8, 9, 15, 16, 17, 24, 31, 32, 33, 39, 40])
def test_checkpoint_boundaries(scene, ora, n):
    b, R, D = scene
    idx = np.arange(64)
    nn = np.full(64, n, np.int32)
    loss, grad = _run(R, b.x0[idx], b.u[idx], nn)
    for e in range(0, 64, 4):
        ref = ora.diff_loss(D, b.x0[e], b.u[e], n)
        assert abs(loss[e] - ref) <= 1e-5 * max(1.0, abs(ref))
    _check_grad(ora, D, b.x0[idx], b.u[idx], nn, grad, range(0, 64, 4))


def test_unequal_inertias_exercise_the_gyroscopic_terms(kpx, ora):
    from paper_2602_02846_amd.diff import Rollout

    b = W.diff_workload(3, n_edges=300)
    b.problem.dyn_params[1:4] = [0.008, 0.011, 0.019]
    R = Rollout(b.problem, b.dt)
    D = ora.DiffProblem(b.problem, b.dt)
    loss, grad = _run(R, b.x0, b.u, b.n)
    _check_loss(ora, D, b, loss, range(0, 300, 2))
    _check_grad(ora, D, b.x0, b.u, b.n, grad, range(0, 300, 5))


def test_scene_without_boxes_and_other_weights(kpx, ora):
    from paper_2602_02846_amd.diff import Rollout

    b = W.diff_workload(4, n_edges=260)
    b.problem.boxes = np.zeros((0, 6), np.float32)
    kw = dict(goal=[0.3, 0.6, 0.4], w_ctrl=0.05, w_goal=3.0)
    R = Rollout(b.problem, b.dt, **kw)
    D = ora.DiffProblem(b.problem, b.dt, **kw)
    loss, grad = _run(R, b.x0, b.u, b.n)
    _check_loss(ora, D, b, loss, range(0, 260, 2))
    _check_grad(ora, D, b.x0, b.u, b.n, grad, range(0, 260, 5))


def test_path_length_term_matches_oracle(kpx, ora):
    """The loss with the path length weighted in, and its gradient through
    the speeds at every RK4 stage state."""
    from paper_2602_02846_amd.diff import Rollout

    b = W.diff_workload(5, n_edges=260)
    kw = dict(w_len=2.0)
    R = Rollout(b.problem, b.dt, **kw)
    D = ora.DiffProblem(b.problem, b.dt, **kw)
    loss, grad = _run(R, b.x0, b.u, b.n)
    _check_loss(ora, D, b, loss, range(0, 260, 2))
    worst = _check_grad(ora, D, b.x0, b.u, b.n, grad, range(0, 260, 5))
    print(f"max-norm relative gradient error with the length term {worst:.2e}")
    # the term matters: without it most of these gradients would miss the
    # tolerance they meet
    D0 = ora.DiffProblem(b.problem, b.dt)
    far = 0
    idx = range(0, 260, 5)
    for e in idx:
        g0 = ora.diff_grad(D0, b.x0[e], b.u[e], int(b.n[e]))
        far += np.max(np.abs(grad[e] - g0)) / np.max(np.abs(g0)) > 1e-4
    assert far >= 0.8 * len(idx), far


def test_degenerate_edges(scene):
    import torch

    b, R, _ = scene
    n = b.n[:300].copy()
    n[[0, 7, 299]] = [3, 41, -5]  # outside 4..40
    loss, grad = _run(R, b.x0[:300], b.u[:300], n)
    assert np.isnan(loss[[0, 7, 299]]).all()
    assert (grad[[0, 7, 299]] == 0).all()
    assert np.isfinite(loss[1:7]).all()
    # an empty batch does nothing
    e = torch.empty((12, 0), device="cuda"), torch.empty((16, 0), device="cuda")
    loss, grad = R.loss_grad(e[0], e[1], torch.empty(0, dtype=torch.int32, device="cuda"))
    assert loss.numel() == 0 and grad.numel() == 0


def test_autograd_function(scene):
    import torch

    from paper_2602_02846_amd.diff import edge_loss

    b, R, _ = scene
    x0, u, n = _dev(b.x0[:500], b.u[:500], b.n[:500])
    u = u.clone().requires_grad_(True)
    wts = torch.linspace(0.5, 1.5, 500, device="cuda")
    L = edge_loss(u, R, x0, n)
    (L * wts).sum().backward()
    loss, grad = R.loss_grad(x0, u.detach(), n)
    torch.cuda.synchronize()
    assert torch.equal(L.detach(), loss)
    torch.testing.assert_close(u.grad, grad * wts.unsqueeze(0), rtol=0, atol=0)


def test_polish_matches_oracle_steps(scene, ora):
    import torch

    b, R, D = scene
    m = 200
    x0, u, n = _dev(b.x0[:m], b.u[:m], b.n[:m])
    before, _ = R.loss_grad(x0, u, n, want_grad=False)
    after = R.polish(x0, u, n, steps=3, lr=LR)
    torch.cuda.synchronize()
    before, after, up = before.cpu().numpy(), after.cpu().numpy(), u.cpu().numpy().T
    lo = np.asarray(b.problem.u_lo[:4], np.float32)
    hi = np.asarray(b.problem.u_hi[:4], np.float32)
    assert (up >= np.tile(lo, 4)).all() and (up <= np.tile(hi, 4)).all()
    lr = float(np.float32(LR))
    for e in range(0, m, 4):
        v = b.u[e].astype(np.float64)
        for _ in range(3):  # projected gradient steps in float64
            v = np.clip(v - lr * ora.diff_grad(D, b.x0[e], v, int(b.n[e])), np.tile(lo, 4), np.tile(hi, 4))
        scale = np.tile(hi - lo, 4)
        assert np.max(np.abs(up[e] - v) / scale) <= 1e-5, (e, up[e], v)
        ref = ora.diff_loss(D, b.x0[e], up[e], int(b.n[e]))
        assert abs(after[e] - ref) <= 1e-5 * max(1.0, abs(ref))
    assert (after <= before + 1e-5 * np.maximum(1.0, np.abs(before))).all()
    assert after.mean() < before.mean()


def _margin(ora, b, x):
    """Distance of state x to the nearest boundary of the valid set (state
    bounds, workspace, box faces): where it is below float32 resolution the
    float32 and float64 rollouts may judge the step differently."""
    p = b.problem
    lo, hi = np.asarray(p.x_lo[:12], np.float64), np.asarray(p.x_hi[:12], np.float64)
    d = [np.min(np.abs(x - lo)), np.min(np.abs(x - hi)),
         np.min(np.abs(x[:3] - np.asarray(p.ws_lo[:3], np.float64))),
         np.min(np.abs(x[:3] - np.asarray(p.ws_hi[:3], np.float64)))]
    d += [abs(ora.box_sd(bx, x[:3])) for bx in np.asarray(p.boxes).reshape(-1, 6)]
    return min(d)


def _check_validity(ora, D, b, u, n, bad, idx):
    exact = 0
    for e in idx:
        ref = ora.diff_first_invalid(D, b.x0[e], u[e], int(n[e]))
        if bad[e] == ref:
            exact += 1
            continue
        _, st = ora.diff_loss(D, b.x0[e], u[e], int(n[e]), states=True)
        k = min(k for k in (int(bad[e]), ref) if k > 0)
        assert _margin(ora, b, st[k]) < 1e-5, (e, int(bad[e]), ref)
    return exact


def test_validity_matches_oracle(scene, ora):
    import torch

    b, R, D = scene
    x0, u, n = _dev(b.x0, b.u, b.n)
    loss, bad = R.polish(x0, u, n, steps=0, validity=True)
    ref_loss, _ = R.loss_grad(x0, u, n, want_grad=False)
    torch.cuda.synchronize()
    assert torch.equal(loss, ref_loss)
    bad = bad.cpu().numpy()
    assert ((bad >= 0) & (bad <= b.n)).all()
    assert 0 < (bad > 0).sum() < len(bad)  # both kinds occur in the workload
    exact = _check_validity(ora, D, b, b.u, b.n, bad, range(E_PARITY))
    assert exact >= E_PARITY - 2


def test_polished_edges_are_rejudged_by_the_oracle(scene, ora):
    import torch

    b, R, D = scene
    m = 400
    x0, u, n = _dev(b.x0[:m], b.u[:m], b.n[:m])
    nn = b.n[:m].copy()
    nn[5] = 2  # unsupported: -1
    n = torch.from_numpy(nn).cuda()
    loss, bad = R.polish(x0, u, n, steps=3, lr=LR, validity=True)
    torch.cuda.synchronize()
    bad, up = bad.cpu().numpy(), u.cpu().numpy().T
    assert bad[5] == -1 and np.isnan(loss[5].item())
    keep = [e for e in range(m) if e != 5]
    exact = _check_validity(ora, D, b, up, nn, bad, keep)
    assert exact >= len(keep) - 2
    print(f"valid after 3 polish steps: {(bad[keep] == 0).sum()} of {len(keep)}")


def test_rejects_tensors_that_do_not_fit(scene):
    import torch

    b, R, _ = scene
    x0, u, n = _dev(b.x0[:100], b.u[:100], b.n[:100])
    loss = torch.empty(100, device="cuda")
    grad = torch.empty((16, 100), device="cuda")
    for bad in ((x0[:, :50], u, n), (x0, u[:8], n), (x0.T.contiguous().T, u, n),
                (x0.double(), u, n), (x0, u, n.long())):
        with pytest.raises(ValueError):
            R.loss_grad_into(*bad, loss, grad)
    with pytest.raises(ValueError):
        R.loss_grad_into(x0, u, n, loss[:50], grad)
    with pytest.raises(ValueError):
        R.loss_grad_into(x0, u, n, loss, grad[:, :50])
    with pytest.raises(ValueError):
        R.polish(x0, u.clone(), n, steps=1, loss=loss[:10])
    R.loss_grad_into(x0, u, n, loss, grad)  # the right shapes still run
    torch.cuda.synchronize()
    assert torch.isfinite(loss).all()
