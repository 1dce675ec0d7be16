"""The C interface driven the way a PyTorch caller drives it: the problem is
created on a torch stream, the data, start point and results cross as device
pointers of torch tensors (on_device = 1) enqueued on that same stream, and the
outcome is bitwise the one of the host-pointer path on the library's own
stream."""
import numpy as np
import pytest

from paper_2002_02328_amd import binding, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _setup(g, w):
    g.set_psf_gaussian(w.kxy, w.kz, w.sigma_xy, w.sigma_z)
    g.set_params(w.lam, w.delta, w.eta, w.kappa)


@pytest.mark.parametrize("prec", [binding.FP32, binding.FP64])
def test_torch_stream_and_device_pointers_match_host_path(prec):
    assert torch.cuda.is_available()
    shape = (12, 45, 100)
    w = inputs.tiny(shape, seed=21, kxy=5, kz=5, nblocks=4)
    nz, ny, nx = shape
    dt = np.float64 if prec == binding.FP64 else np.float32
    tdt = torch.float64 if prec == binding.FP64 else torch.float32
    y = (w.xbar + w.noise).astype(dt)
    x0 = np.clip(y, 0.0, 1.0).astype(dt)

    # host pointers, the library's own stream
    h = binding.Problem(nx, ny, nz, prec)
    _setup(h, w)
    h.set_data(y)
    h.set_blocks(w.nslices)
    h.set_x0(x0)
    rh = h.run(25, grad_rtol=0.0, check_every=25)
    xh, dh, qh, sh = h.get_state()
    h.close()

    # device pointers of torch tensors, everything on one torch stream
    s = torch.cuda.Stream()
    g = binding.Problem(nx, ny, nz, prec, stream=s.cuda_stream)
    _setup(g, w)
    with torch.cuda.stream(s):
        ty = torch.from_numpy(y).to("cuda", non_blocking=False)
        tx0 = torch.from_numpy(x0).to("cuda")
        tx = torch.full(shape, float("nan"), dtype=tdt, device="cuda")
        g.set_data(ty.data_ptr(), on_device=True)
        g.set_blocks(w.nslices)
        g.set_x0(tx0.data_ptr(), on_device=True)
        rg = g.run(25, grad_rtol=0.0, check_every=25)
        g.get_x(out_ptr=tx.data_ptr())
        # work the caller enqueues on the stream after a call sees its results
        tsum = tx.sum()
    s.synchronize()
    xg = tx.cpu().numpy()
    assert np.array_equal(xg, xh)
    assert rg["f"] == rh["f"] and rg["grad_norm"] == rh["grad_norm"]
    assert float(tsum) == pytest.approx(float(xh.astype(np.float64).sum()), rel=1e-5)
    # the state read back through the interface agrees as well
    xs, ds, qs, ss = g.get_state()
    assert np.array_equal(xs, xh) and np.array_equal(ds, dh) and np.array_equal(qs, qh) and ss == sh
    g.close()
    # the caller's stream is left alive: it still takes work
    with torch.cuda.stream(s):
        z = torch.ones(4, device="cuda") * 2
    s.synchronize()
    assert float(z.sum()) == 8.0
