"""The fitting loop's own kernels (loss gradient, Adam update) against
PyTorch references computed on the CPU, and a short native fit against the
same fit driven by PyTorch autograd and torch.optim.Adam around the library's
forward and backward."""
import numpy as np
import pytest
import torch

import paper_2602_20063_amd as shm
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def ref_loss(out, dirs, tr, tn, w_value):
    """The value + normal objective in FP64 on the CPU; rows whose output is
    not finite contribute nothing but count in the means."""
    Q = out.shape[0]
    ok = torch.isfinite(out).all(dim=1)
    o = out[ok]
    w = dirs[ok] / dirs[ok].norm(dim=1, keepdim=True)
    m = o[:, :1] * w - o[:, 1:]
    n = m / m.norm(dim=1, keepdim=True)
    return (w_value * ((o[:, 0] - tr[ok]) ** 2).sum() + ((n - tn[ok]) ** 2).sum()) / Q


def test_loss_grad_matches_autograd():
    rng = np.random.default_rng(7)
    Q = 5003
    dirs = workloads.uniform_dirs(Q, rng) * rng.uniform(0.5, 2.0, (Q, 1)).astype(np.float32)
    dirs[17] = 0.0
    out = np.concatenate([1.0 + 0.2 * rng.standard_normal((Q, 1)), 0.1 * rng.standard_normal((Q, 3))], axis=1)
    out = out.astype(np.float32)
    out[17] = np.nan  # the query of a zero direction
    tr = (1.0 + 0.2 * rng.standard_normal(Q)).astype(np.float32)
    tn = rng.standard_normal((Q, 3))
    tn = (tn / np.linalg.norm(tn, axis=1, keepdims=True)).astype(np.float32)
    w_value = 37.0
    g = torch.empty((Q, 4), device=DEV)
    shm.shm_fit_loss_grad(torch.as_tensor(out).to(DEV), torch.as_tensor(dirs).to(DEV), torch.as_tensor(tr).to(DEV),
                          torch.as_tensor(tn).to(DEV), Q, w_value, g)
    got = g.cpu().numpy()
    o64 = torch.as_tensor(out, dtype=torch.float64).requires_grad_(True)
    ref_loss(o64, torch.as_tensor(dirs, dtype=torch.float64), torch.as_tensor(tr, dtype=torch.float64),
             torch.as_tensor(tn, dtype=torch.float64), w_value).backward()
    ref = np.nan_to_num(o64.grad.numpy())
    assert (got[17] == 0).all()
    scale = np.abs(ref).max(axis=0)
    assert (np.abs(got - ref).max(axis=0) <= 2e-5 * scale).all(), (np.abs(got - ref).max(axis=0), scale)


def test_fused_forward_loss_grad_matches_two_steps():
    """The fused kernel equals the forward query followed by the loss
    gradient, on a random LUT with a ragged query count and a zero
    direction."""
    rng = np.random.default_rng(9)
    N, Q = 24, 7777
    lut = torch.as_tensor(workloads.random_lut(N, rng)).to(DEV)[None].contiguous()
    dirs = workloads.uniform_dirs(Q, rng)
    dirs[5] = 0.0
    d = torch.as_tensor(dirs).to(DEV)
    tr = torch.as_tensor((1.0 + 0.1 * rng.standard_normal(Q)).astype(np.float32)).to(DEV)
    tn = rng.standard_normal((Q, 3))
    tn = torch.as_tensor((tn / np.linalg.norm(tn, axis=1, keepdims=True)).astype(np.float32)).to(DEV)
    out = torch.empty((Q, 4), device=DEV)
    shm.shm_query_value_grad(lut, shm.SHM_F32, shm.SHM_LAYOUT_TEXEL, N, 1, d, Q, out)
    g2 = torch.empty((Q, 4), device=DEV)
    shm.shm_fit_loss_grad(out, d, tr, tn, Q, 5.0, g2)
    g1 = torch.full((Q, 4), float("nan"), device=DEV)
    shm.shm_fit_forward_loss_grad(lut, N, d, tr, tn, Q, 5.0, g1)
    a, b = g1.cpu().numpy(), g2.cpu().numpy()
    assert (a[5] == 0).all() and np.isfinite(a).all()
    assert (np.abs(a - b).max(axis=0) <= 1e-6 * np.abs(b).max(axis=0)).all()


def test_adam_matches_torch_adam():
    rng = np.random.default_rng(8)
    N = 6
    p0 = rng.standard_normal((1, 6, N + 2, N + 2, 4)).astype(np.float32)
    grads = [rng.standard_normal(p0.shape).astype(np.float32) * s for s in (1.0, 0.01, 3.0, 1e-4)]
    lr_v, lr_d = 1e-2, 3e-3
    p = torch.as_tensor(p0).to(DEV)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    val = torch.tensor(p0[..., :1], requires_grad=True)
    der = torch.tensor(p0[..., 1:], requires_grad=True)
    opt = torch.optim.Adam([{"params": [val], "lr": lr_v}, {"params": [der], "lr": lr_d}], betas=(0.9, 0.999),
                           eps=1e-8, foreach=False)
    for t, gr in enumerate(grads, start=1):
        shm.shm_adam_step(p, torch.as_tensor(gr).to(DEV), m, v, p.numel() // 4, t, lr_v, lr_d)
        val.grad = torch.as_tensor(gr[..., :1]).clone()
        der.grad = torch.as_tensor(gr[..., 1:]).clone()
        opt.step()
        ref = torch.cat([val.detach(), der.detach()], dim=-1).numpy()
        got = p.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-6 * (1.0 + np.abs(ref).max()), (t, np.abs(got - ref).max())


@pytest.mark.parametrize("fused", [True, False])
def test_native_fit_matches_torch_loop(fused):
    """20 steps at N = 16 on 30,000 directions sorted by cell: the native
    loop (one fused kernel per step, or the three-kernel step) and the
    autograd + torch.optim.Adam loop end at the same LUT."""
    N, Q = 16, 30000
    r = workloads.rng_for(4)
    dirs = torch.as_tensor(workloads.uniform_dirs(Q, r)).to(DEV)
    keys = shm.cell_keys(N, dirs)
    dirs = dirs[torch.argsort(keys.to(torch.int64) & 0xFFFFFFFF, stable=True)].contiguous()
    tv, tg = workloads.fbm_target_torch(dirs, seed=5)
    tv, tg = tv.float(), tg.float()
    w = dirs / dirs.norm(dim=1, keepdim=True)
    tn = tv[:, None] * w - tg
    tn = (tn / tn.norm(dim=1, keepdim=True)).contiguous()
    lut0 = torch.zeros((1, 6, N + 2, N + 2, 4), device=DEV)
    lut0[..., 0] = 1.0
    w_value, lr_v, lr_d, steps = 1000.0, 1e-3, 3e-4, 20
    fit = shm.LutFit(lut0.clone(), dirs, tv, tn, w_value=w_value, lr_value=lr_v, lr_deriv=lr_d, fused=fused)
    for _ in range(steps):
        fit.step()
    val = lut0[..., :1].clone().requires_grad_(True)
    der = lut0[..., 1:].clone().requires_grad_(True)
    opt = torch.optim.Adam([{"params": [val], "lr": lr_v}, {"params": [der], "lr": lr_d}], betas=(0.9, 0.999),
                           eps=1e-8)
    bctx = shm.BackwardContext(N, 1, dirs, Q)
    losses = []
    for _ in range(steps):
        opt.zero_grad(set_to_none=True)
        o = shm.HermiteQuery.apply(torch.cat([val, der], dim=-1).contiguous(), dirs, bctx)
        n = o[:, :1] * w - o[:, 1:]
        n = n / n.norm(dim=1, keepdim=True)
        loss = w_value * ((o[:, 0] - tv) ** 2).mean() + ((n - tn) ** 2).sum(dim=1).mean()
        loss.backward()
        opt.step()
        losses.append(loss.item())
    torch.cuda.synchronize()
    ref = torch.cat([val.detach(), der.detach()], dim=-1)
    d = (fit.lut - ref).abs().max().item()
    assert d <= 1e-4 * ref.abs().max().item(), d
    assert losses[-1] < 0.7 * losses[0]  # and the fit makes progress


def fit_problem(N, Q, seed, zero=()):
    """A random LUT, Q unsorted directions (some zero) and fBm targets."""
    rng = np.random.default_rng(seed)
    lut = torch.as_tensor(workloads.random_lut(N, rng)).to(DEV)[None].contiguous()
    d = workloads.uniform_dirs(Q, rng)
    d[list(zero)] = 0.0
    dirs = torch.as_tensor(d).to(DEV)
    at = d.copy()
    at[list(zero)] = (0.0, 0.0, 1.0)  # targets of the zero directions: any finite values
    at = torch.as_tensor(at).to(DEV)
    tv, tg = workloads.fbm_target_torch(at, seed=seed)
    w = at / at.norm(dim=1, keepdim=True)
    tn = tv.float()[:, None] * w - tg.float()
    tn = tn / tn.norm(dim=1, keepdim=True)
    return lut, dirs, tv.float().contiguous(), tn.contiguous()


@pytest.mark.parametrize("N,Q", [(16, 20011), (37, 50000), (3, 30011)])  # (3, 30011): ~300 queries per cell, dense tiles
def test_fused_step_matches_three_kernel_step(N, Q):
    """The one-kernel fitting step against the three-kernel step (forward +
    loss gradient, LUT-only backward, Adam) from the same LUT, over 4 steps:
    unsorted directions with zero ones among them, tiles that overhang the
    face (N + 2 not a multiple of 15).  Same sums in the same order, so the
    moments agree to rounding and the parameters to far below an Adam step."""
    lut, dirs, tv, tn = fit_problem(N, Q, seed=N, zero=(3, Q - 1))
    a = shm.LutFit(lut.clone(), dirs, tv, tn, w_value=30.0, lr_value=1e-3, lr_deriv=3e-4, fused=True)
    b = shm.LutFit(lut.clone(), dirs, tv, tn, w_value=30.0, lr_value=1e-3, lr_deriv=3e-4, fused=False)
    for step in range(1, 5):
        a.step()
        b.step()
        torch.cuda.synchronize()
        same = torch.equal(a.lut, b.lut) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)
        dm = (a.m - b.m).abs().max().item()
        dp = (a.lut - b.lut).abs().max().item()
        print(f"N={N} step {step}: bitwise {same}, max |dm| {dm:.3g} of {b.m.abs().max().item():.3g}, max |dp| {dp:.3g}")
        assert dm <= 1e-5 * b.m.abs().max().item(), (step, dm)
        assert dp <= 1e-6, (step, dp)
        assert (b.lut != lut).float().mean().item() > 0.99  # nearly every texel moved
    assert a.lut.data_ptr() != b.lut.data_ptr() and a.lut.data_ptr() == a.bufs[0].data_ptr()  # 4 steps: back to buffer 0


def test_fused_step_without_queries_is_adam_with_zero_gradient():
    """Q = 0: no query list, the gradient is zero, Adam still moves the
    parameters by its moments."""
    N = 20
    rng = np.random.default_rng(2)
    p0 = torch.as_tensor(workloads.random_lut(N, rng)).to(DEV)[None].contiguous()
    m0 = torch.as_tensor(rng.standard_normal(p0.shape).astype(np.float32) * 1e-3).to(DEV)
    v0 = torch.as_tensor(rng.uniform(0, 1e-6, p0.shape).astype(np.float32)).to(DEV)
    empty = torch.empty((0, 3), device=DEV)
    ws = torch.empty(max(shm.shm_backward_workspace(N, 1, 0), 256), dtype=torch.uint8, device=DEV)
    out, m1, v1 = torch.full_like(p0, float("nan")), m0.clone(), v0.clone()
    shm.shm_fit_step(p0, out, m1, v1, N, empty, empty, empty, 0, 1.0, 3, 1e-3, 3e-4, 0.9, 0.999, 1e-8, ws, False)
    p2, m2, v2 = p0.clone(), m0.clone(), v0.clone()
    shm.shm_adam_step(p2, torch.zeros_like(p0), m2, v2, p0.numel() // 4, 3, 1e-3, 3e-4)
    torch.cuda.synchronize()
    print("bitwise", torch.equal(out, p2), torch.equal(m1, m2), torch.equal(v1, v2))
    for x, y in ((out, p2), (m1, m2), (v1, v2)):
        assert (x - y).abs().max().item() <= 1e-7 * (1.0 + y.abs().max().item())


def test_fused_steps_replay_from_a_graph():
    """Two one-kernel steps (t = 1, 2) captured in a HIP graph (through
    torch.cuda.graph) and replayed three times, with eager work and
    synchronisations between the replays: after every replay the LUT and the
    moments equal, bit for bit, those of the same step sequence run eagerly."""
    N, Q = 24, 30011
    lut, dirs, tv, tn = fit_problem(N, Q, seed=11, zero=(5,))
    kw = dict(w_value=30.0, lr_value=1e-3, lr_deriv=3e-4, fused=True)
    g_fit = shm.LutFit(lut.clone(), dirs, tv, tn, **kw)
    e_fit = shm.LutFit(lut.clone(), dirs, tv, tn, **kw)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g_fit.step()
        g_fit.step()
    assert g_fit.cur == 0 and g_fit.t == 2
    for rep in range(3):
        graph.replay()
        junk = torch.randn(1 << 20, device=DEV).sum()  # eager work between replays
        torch.cuda.synchronize()
        e_fit.t = 0  # the graph holds steps 1 and 2
        e_fit.step()
        e_fit.step()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(g_fit.lut, e_fit.lut), rep
        assert torch.equal(g_fit.m, e_fit.m) and torch.equal(g_fit.v, e_fit.v), rep
        assert not torch.equal(g_fit.lut, lut)


@pytest.mark.parametrize("fused", [True, False])
def test_fit_checkpoint_resume(tmp_path, fused):
    """Five steps without stopping equal three steps, a checkpoint written
    with torch.save and read back with weights_only=True into a new fit, and
    two more steps: the same LUT and moments, bit for bit."""
    N, Q = 20, 25013
    lut, dirs, tv, tn = fit_problem(N, Q, seed=12)
    kw = dict(w_value=30.0, lr_value=1e-3, lr_deriv=3e-4, fused=fused)
    a = shm.LutFit(lut.clone(), dirs, tv, tn, **kw)
    for _ in range(5):
        a.step()
    b = shm.LutFit(lut.clone(), dirs, tv, tn, **kw)
    for _ in range(3):
        b.step()
    path = tmp_path / "fit.pt"
    torch.save(b.state_dict(), path)
    c = shm.LutFit(torch.zeros_like(lut), dirs, tv, tn, **kw)
    c.load_state_dict(torch.load(path, weights_only=True))
    for _ in range(2):
        c.step()
    torch.cuda.synchronize()
    assert torch.equal(a.lut, c.lut) and torch.equal(a.m, c.m) and torch.equal(a.v, c.v) and c.t == 5
