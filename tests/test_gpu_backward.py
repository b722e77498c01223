"""GPU adjoint vs the FP64 oracle gradient and central finite differences."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.helpers import azint, norm_err, oracle_matrix

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def grad_scale(m, U, gI, gW):
    """Per-pixel scale sum_b A_bp (|gI_b| / U_b + |gW_b|) of the adjoint."""
    return oracle.integrate_vjp(m, U, np.abs(gI) if gI is not None else None,
                                np.abs(gW) if gW is not None else None)


@pytest.mark.parametrize("g", [(100, 100, 50.0, 50.0, 100), (37, 53, 10.25, 40.5, 61),
                               (64, 48, -5.0, 70.0, 40), (31, 29, 15.5, 14.5, 300),
                               (1, 17, 0.5, 8.5, 5)])
@pytest.mark.parametrize("grads", ["I", "W", "IW"])
def test_backward_vs_oracle(g, grads, dev):
    h, w, cy, cx, npt = g
    say("backward", g, grads)
    az = azint()
    plan = az.Plan(h, w, npt, center=(cy, cx), device=dev)
    m = oracle_matrix(h, w, cy, cx, npt)
    rng = np.random.default_rng(h + w)
    x = rng.uniform(0, 1, size=h * w)
    gI = rng.standard_normal(npt) if "I" in grads else None
    gW = rng.standard_normal(npt) if "W" in grads else None
    _, _, U = oracle.integrate(m, x)
    t = lambda a: None if a is None else torch.from_numpy(a).to(dev)
    _, _, Ud = plan.integrate(t(x))
    gx = plan.backward(Ud, t(gI), t(gW)).cpu().numpy()
    ref = oracle.integrate_vjp(m, U, gI, gW)
    assert norm_err(gx, ref, grad_scale(m, U, gI, gW)) <= 1e-12


def test_c4_adjoint_fd_and_oracle(dev):
    """The 1000x1000 adjoint workload: random upstream gradient (seed 3); the
    GPU gradient against the oracle gradient and against central differences
    of the GPU forward on 64 random pixels (h = 1e-6).  The map is linear, so
    the differences carry no truncation error; each perturbation only moves
    the <= 4 bins the pixel touches, and the difference is formed there."""
    say("c4")
    az = azint()
    inst = synth.c4_instance()
    g = inst.geom
    npt = inst.npt
    x = inst.extra["x"]
    gI = inst.grad
    plan = az.Plan(g.h, g.w, npt, center=(g.center_y, g.center_x), device=dev)
    m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, npt)
    xd = torch.from_numpy(x).to(dev)
    I, W, U = plan.integrate(xd)
    gId = torch.from_numpy(gI).to(dev)
    gx = plan.backward(U, gId).cpu().numpy()
    Io, Wo, Uo = oracle.integrate(m, x)
    ref = oracle.integrate_vjp(m, Uo, gI)
    assert norm_err(gx, ref, grad_scale(m, Uo, gI, None)) <= 1e-12
    # central differences of the GPU forward on 64 pixels
    h = synth.C4["fd_h"]
    I0 = I.cpu().numpy()
    coords = inst.extra["fd_coords"]
    csc_data, csc_bins, colptr = plan.export_csc()
    Ip, Im = torch.empty_like(I), torch.empty_like(I)
    for p in coords:
        bins = csc_bins[colptr[p]:colptr[p + 1]]
        xp = xd.clone()
        xp[p] += h
        plan.integrate(xp, out=(Ip, torch.empty_like(W), torch.empty_like(U)))
        xm = xd.clone()
        xm[p] -= h
        plan.integrate(xm, out=(Im, torch.empty_like(W), torch.empty_like(U)))
        dp = Ip.cpu().numpy()[bins]
        dm = Im.cpu().numpy()[bins]
        fd = float(np.dot(gI[bins], dp - dm)) / (2 * h)
        # rounding of I at each touched bin, amplified by 1/(2h)
        bound = 4 * 2.3e-16 * float(np.dot(np.abs(gI[bins]), np.abs(I0[bins]))) / (2 * h)
        assert abs(fd - gx[p]) <= bound + 1e-9 * abs(gx[p]), (p, fd, gx[p], bound)
        # only those bins moved
        others = np.setdiff1d(np.arange(npt), bins)
        assert np.array_equal(Ip.cpu().numpy()[others], I0[others])


def test_dot_product_identity(dev):
    say("dot product identity")
    az = azint()
    plan = az.Plan(300, 310, 280, center=(150.5, 140.2), device=dev)
    rng = np.random.default_rng(1)
    x = torch.from_numpy(rng.uniform(0, 1, 300 * 310)).to(dev)
    gI = torch.from_numpy(rng.standard_normal(280)).to(dev)
    gW = torch.from_numpy(rng.standard_normal(280)).to(dev)
    I, W, U = plan.integrate(x)
    gx = plan.backward(U, gI, gW)
    lhs = float((gI * I).sum() + (gW * W).sum())
    rhs = float((gx * x).sum())
    scale = float((gI.abs() * I.abs()).sum() + (gW.abs() * W.abs()).sum())
    assert abs(lhs - rhs) <= 1e-13 * scale


@pytest.mark.parametrize("shape", [(256,), (16, 16)])
def test_autograd_function_gradcheck(shape, dev):
    """gradcheck of the autograd function on a flat image and on an (h, w)
    image, whose gradient must come back in the image's own shape."""
    say("gradcheck", shape)
    az = azint()
    plan = az.Plan(16, 16, 12, center=(8.3, 7.9), device=dev)
    x = torch.rand(shape, dtype=torch.float64, device=dev, requires_grad=True)

    def f(x):
        I, W, _ = az.Integrate1d.apply(x, plan, 0.0)
        return I, W

    # W ~ 30 here: its rounding (~4e-15) over 2*eps gives ~2e-9 of FD noise
    assert torch.autograd.gradcheck(f, (x,), eps=1e-6, atol=2e-8, rtol=1e-7)
    I, W, _ = az.Integrate1d.apply(x, plan, 0.0)
    (g,) = torch.autograd.grad(I.sum() + W.sum(), x)
    assert g.shape == x.shape


def test_backward_wrt_raw_with_corrections(dev):
    say("backward wrt raw")
    az = azint()
    inst = synth.instance_hw(50, 40, 9, npt=30, corrections=True, grad=True)
    g = inst.geom
    plan = az.Plan(g.h, g.w, 30, device=dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(dev)
    plan.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
    I, W, U = plan.integrate_raw(t(inst.raw))
    graw = plan.backward(U, t(inst.grad), wrt_raw=True).cpu().numpy()
    m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, 30)
    x = oracle.correct(inst.raw, inst.dark, inst.flat, inst.solid, inst.polar)
    _, _, Uo = oracle.integrate(m, x)
    norm = oracle.azint_oracle.correction_norm(inst.flat, inst.solid, inst.polar)
    ref = oracle.integrate_vjp(m, Uo, inst.grad, norm=norm)
    scale = grad_scale(m, Uo, inst.grad, None) / norm
    assert norm_err(graw, ref, scale) <= 1e-12


def test_backward_f32(dev):
    say("backward f32")
    az = azint()
    plan = az.Plan(120, 130, 100, dtype=torch.float32, device=dev)
    m = oracle_matrix(120, 130, 60.0, 65.0, 100)
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, 120 * 130).astype(np.float32)
    gI = rng.standard_normal(100).astype(np.float32)
    I, W, U = plan.integrate(torch.from_numpy(x).to(dev))
    gx = plan.backward(U, torch.from_numpy(gI).to(dev)).cpu().numpy().astype(np.float64)
    m32 = dict(m)
    m32["coef"] = m["coef"].astype(np.float32).astype(np.float64)
    U32 = U.cpu().numpy().astype(np.float64)
    ref = oracle.integrate_vjp(m32, U32, gI.astype(np.float64))
    assert norm_err(gx, ref, grad_scale(m32, U32, gI.astype(np.float64), None)) <= 2.0 ** -22


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_first_bin_adjoint_bits_equal_per_entry_adjoint(dtype, dev):
    """One-dimensional plans run the adjoint from each pixel's first bin (its
    bins are consecutive); a batch that also holds a 2-D plan reads the
    per-entry bin ids of the CSC for all its pixels.  The products are added
    in the same order either way, so the 1-D instances' gradients must agree
    bit for bit."""
    say("first-bin vs per-entry adjoint", dtype)
    az = azint()
    shapes = [(90, 100, 44.6, 50.2, 40), (31, 29, 15.5, 14.5, 300), (1, 17, 0.5, 8.5, 5),
              (257, 263, 128.5, 131.5, 256)]
    plans = [az.Plan(h, w, n, center=(cy, cx), dtype=dtype, layout="pixel")
             for (h, w, cy, cx, n) in shapes]
    two = az.Plan(40, 50, 20, npt_azim=8, dtype=dtype, layout="pixel")
    batch = az.Batch(plans[:2] + [two] + plans[2:], device=dev)
    npd = np.float64 if dtype == torch.float64 else np.float32
    rng = np.random.default_rng(31)
    xs = [rng.uniform(0, 1, size=p.npix).astype(npd) for p in plans[:2] + [two] + plans[2:]]
    x = torch.from_numpy(np.concatenate(xs)).to(dev)
    I, W, U = batch.forward(x)
    gI = torch.from_numpy(rng.standard_normal(batch.npt).astype(npd)).to(dev)
    gW = torch.from_numpy(rng.standard_normal(batch.npt).astype(npd)).to(dev)
    gx = batch.backward(U, gI, gW)
    torch.cuda.synchronize()
    po, bo = batch.pix_off, batch.bin_off
    order = [0, 1, None, 2, 3]
    for k, j in enumerate(order):
        if j is None:
            continue
        p = plans[j]
        p.upload(dev)
        gk = p.backward(U[bo[k]:bo[k + 1]].contiguous(), gI[bo[k]:bo[k + 1]].contiguous(),
                        gW[bo[k]:bo[k + 1]].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(gk, gx[po[k]:po[k + 1]]), shapes[j]
