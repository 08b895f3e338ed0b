"""Parity of the straight-through (differentiable) coder on the GPU with the FP64 oracle.

The forward must be the codec: the same stream bytes as gsc_encode_frame, yhat = q * step of
that stream, ahat equal to the GPU decoder's output for it. The loss and the gradient of every
Gaussian attribute (through torch.autograd) are compared with the oracle's closed form. A
quantized coefficient that the FP32 transform rounds to the other side of a decision boundary
than the FP64 oracle (a rounding tie, verified as such) changes yhat by one step; the entries
it reaches through T^T (its subtree in that channel) are then left out of the comparison.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2606_05650_amd import gsc, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GROUPED = synth.quant_steps(synth.STEPS_GROUPED)
REL_TOL = 1e-5
TIE_FRAC = 1e-4


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _ties(pos, attr, J, steps, q_gpu, leaf):
    """Coefficients whose GPU decision differs from the oracle's: checked to be rounding ties
    of the FP32 coefficient; returns the mask of (voxel, channel) entries they reach."""
    dev = _dev()
    ref = orc.encode_frame(pos, attr, J, steps, 0.5, want_y=True)
    nv, C = q_gpu.shape
    diff = q_gpu != ref["Q"]
    assert diff.mean() <= TIE_FRAC
    affected = np.zeros((nv, C), dtype=bool)
    if not diff.any():
        return affected, 0
    coef = torch.empty((max(pos.shape[0], 1), C), dtype=torch.float32, device=dev)
    gsc.encode_frame(torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev),
                     gsc.make_params(J, C, steps), coef_f32=coef).check()
    Y32 = coef[:nv].cpu().numpy().astype(np.float64)
    Y64 = ref["Y"]
    for v, c in zip(*np.nonzero(diff)):
        assert abs(int(q_gpu[v, c]) - int(ref["Q"][v, c])) == 1
        t = abs(Y64[v, c]) / float(steps[c]) + 0.5
        assert abs(t - round(t)) <= abs(Y32[v, c] - Y64[v, c]) / float(steps[c]) + 1e-12
        e = np.zeros((nv, 1))
        e[v, 0] = 1.0
        affected[orc.raht_inverse(leaf, J, e)[:, 0] != 0, c] = True
    return affected, int(diff.sum())


def _run(pos, attr, J, lam):
    from paper_2606_05650_amd.ste import SteCoder, rd_loss
    dev = _dev()
    C = attr.shape[1]
    p = gsc.make_params(J, C, GROUPED)
    tp = torch.from_numpy(pos).to(dev)
    ta = torch.from_numpy(attr).to(dev).requires_grad_(True)
    steps = torch.from_numpy(GROUPED).to(dev)
    yhat, ahat, aref = SteCoder.apply(ta, tp, p)
    loss, dist, rate = rd_loss(yhat, ahat, aref, steps, lam)
    loss.backward()
    torch.cuda.synchronize()
    return dict(yhat=yhat.detach().cpu().numpy(), ahat=ahat.detach().cpu().numpy(),
                aref=aref.cpu().numpy(), grad=ta.grad.cpu().numpy(), dist=float(dist),
                rate=float(rate))


def _compare(pos, attr, J, lam):
    print(f"case n={pos.shape[0]} J={J} lambda={lam}", flush=True)
    g = _run(pos, attr, J, lam)
    o = orc.ste_grad(pos, attr, J, GROUPED, 0.5, lam)
    nv, C = o["nv"], attr.shape[1]
    assert g["yhat"].shape == (nv, C)
    q_gpu = np.rint(g["yhat"].astype(np.float64) / GROUPED).astype(np.int32)
    assert np.array_equal(q_gpu.astype(np.float64) * GROUPED, g["yhat"].astype(np.float64))
    aff, nties = _ties(pos, attr, J, GROUPED, q_gpu, o["leaf"])
    ok = ~aff
    # voxel means and the decoded rows
    sc = np.abs(o["aref"]).max(axis=0)
    assert (np.abs(g["aref"] - o["aref"]).max(axis=0) / sc).max() <= REL_TOL
    assert np.array_equal(g["yhat"][ok], o["yhat"][ok])
    assert (np.where(ok, np.abs(g["ahat"] - o["ahat"]), 0).max(axis=0) / sc).max() <= REL_TOL
    # loss
    assert abs(g["dist"] - o["dist"]) <= 1e-3 * o["dist"] + 4 * nties * 0.25 / (nv * C)
    assert abs(g["rate"] - o["rate"]) <= 1e-5 * o["rate"] + lam * nties
    # gradient of every Gaussian attribute not reached by a tie
    vof = o["voxel_of"]
    okg = ok[vof]
    gmax = np.abs(o["grad"]).max(axis=0)
    cnt = np.bincount(vof, minlength=nv)[vof][:, None]
    tol = REL_TOL * gmax + 2.0 / (nv * C) * 2 * REL_TOL * sc / cnt
    err = np.where(okg, np.abs(g["grad"] - o["grad"]) - tol, 0)
    assert err.max() <= 0, f"gradient error exceeds the bound by {err.max():.3g}"
    assert okg.mean() >= 0.9
    return g, o


@pytest.mark.parametrize("n,J,lam,dups", [
    (2000, 11, 0.01, False),
    (2000, 11, 0.0, False),
    (3000, 4, 0.01, True),
    (20_000, 9, 0.01, False),
    (1, 6, 0.01, False),
])
def test_ste_gradient_matches_oracle(n, J, lam, dups):
    if dups:
        pos, attr = synth.make_duplicates_frame(n, seed=40, grid=8)
    else:
        pos, attr = synth.make_frame(n, seed=41 + n % 7)
    _compare(pos, attr, J, lam)


def test_ste_gradient_500k_depth11():
    pos, attr = synth.make_frame(500_000, seed=4)
    _compare(pos, attr, 11, 0.01)


def test_ste_forward_is_the_codec():
    dev = _dev()
    pos, attr = synth.make_frame(30_000, seed=42)
    J, C = 10, attr.shape[1]
    p = gsc.make_params(J, C, GROUPED)
    tp, ta = torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev)
    f = gsc.ste_forward(tp, ta, p)
    e = gsc.encode_frame(tp, ta, p)
    torch.cuda.synchronize()
    f.encoded.check()
    e.check()
    assert f.encoded.to_bytes() == e.to_bytes()
    nv = e.n_vox()
    blob = np.frombuffer(e.to_bytes(), dtype=np.uint8)
    h = gsc.parse_header(blob)
    Q = blob[int(h["coef_offset"]):].view(np.int32).reshape(nv, C)
    assert np.array_equal(f.yhat[:nv].cpu().numpy(), (Q * GROUPED).astype(np.float32))
    d = gsc.decode_frame(e.stream, J, C, nv)
    torch.cuda.synchronize()
    assert torch.equal(f.ahat[:nv], d.attr[:nv])


def test_ste_backward_repeatable_and_checks_workspace():
    dev = _dev()
    pos, attr = synth.make_frame(5000, seed=43)
    J, C = 9, attr.shape[1]
    p = gsc.make_params(J, C, GROUPED)
    tp, ta = torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev)
    f = gsc.ste_forward(tp, ta, p)
    f.encoded.check()
    nv = f.encoded.n_vox()
    gy = torch.randn((nv, C), device=dev)
    ga = torch.randn((nv, C), device=dev)
    g1, i1 = gsc.ste_backward(f, gy, ga)
    g2, i2 = gsc.ste_backward(f, gy, ga)
    torch.cuda.synchronize()
    assert int(i1[0]) == 0 and int(i2[0]) == 0 and torch.equal(g1, g2)
    # a workspace that holds a plain encode is refused on the device, without touching output
    e = gsc.encode_frame(tp, ta, p)
    e.check()
    plain = gsc.SteForward(f.yhat, f.ahat, f.aref, e, f.n)
    out = torch.full((5000, C), 7.0, device=dev)
    _, i3 = gsc.ste_backward(plain, gy, ga, out=out)
    torch.cuda.synchronize()
    assert int(i3[0]) == 1 and bool((out == 7.0).all())


def test_padded_layer_matches_without_host_synchronization():
    """SteCoderPadded gives SteCoder's outputs, loss and gradient, and a whole training step with
    it (forward, loss, backward) makes no host synchronization: torch's sync-debug mode, set to
    raise, lets it through (it raises on the synchronizing layer)."""
    from paper_2606_05650_amd.ste import SteCoder, SteCoderPadded, rd_loss
    dev = _dev()
    pos, attr = synth.make_frame(20_000, seed=43)
    J, lam = 9, 0.01
    n, C = attr.shape
    print(f"case n={n} J={J} padded layer", flush=True)
    p = gsc.make_params(J, C, GROUPED)
    tp = torch.from_numpy(pos).to(dev)
    steps = torch.from_numpy(GROUPED).to(dev)
    ta = torch.from_numpy(attr).to(dev).requires_grad_(True)
    yhat, ahat, aref = SteCoder.apply(ta, tp, p)
    loss, _, _ = rd_loss(yhat, ahat, aref, steps, lam)
    loss.backward()
    torch.cuda.synchronize()
    nv = yhat.shape[0]
    want_loss, want_grad = float(loss), ta.grad.clone()

    tb = torch.from_numpy(attr).to(dev).requires_grad_(True)

    def step():
        y, a, r, nvt = SteCoderPadded.apply(tb, tp, p)
        l, _, _ = rd_loss(y, a, r, steps, lam, nv=nvt)
        l.backward()
        return y, a, r, nvt, l

    y, a, r, nvt, l = step()
    torch.cuda.synchronize()
    assert int(nvt.item()) == nv
    assert y.shape == (n, C)
    assert torch.equal(y[:nv], yhat.detach()) and torch.equal(a[:nv], ahat.detach())
    assert torch.equal(r[:nv], aref)
    assert not y[nv:].any() and not a[nv:].any() and not r[nv:].any()
    assert abs(float(l) - want_loss) <= 1e-5 * abs(want_loss)
    torch.testing.assert_close(tb.grad, want_grad, rtol=1e-5, atol=1e-9)
    first_grad = tb.grad.clone()

    # the same step again with every torch-side host synchronization turned into an error
    tb.grad = None
    torch.cuda.set_sync_debug_mode("error")
    try:
        out = step()
        with pytest.raises(RuntimeError):
            tb.grad = None
            SteCoder.apply(tb, tp, p)  # cuts its outputs to Nv rows: synchronizes
    finally:
        torch.cuda.set_sync_debug_mode("default")
    torch.cuda.synchronize()
    assert int(out[3].item()) == nv and float(out[4]) == float(l)
    tb.grad = None
    step()
    torch.cuda.synchronize()
    assert torch.equal(tb.grad, first_grad)
