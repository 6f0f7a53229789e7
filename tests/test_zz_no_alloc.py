"""The no-allocation image loss (vbm_image_loss_static) against the workspace one (vbm_image_loss),
called through the C ABI: two calls in a row, the second on a smaller batch, for L1 and for
L1 + D-SSIM; the fixed scratch keeps the last call's contents, so the second call also shows that
nothing stale leaks into a later result.  Beyond its fixed size the call is refused, launching
nothing."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import loss as oloss
from tests.gpu_common import dev, say

pytestmark = pytest.mark.gpu


def _batch(dims, seed):
    rng = np.random.default_rng(seed)
    imgs = [rng.uniform(size=(3, h, w)).astype(np.float32) for w, h in dims]
    tgts = [np.clip(i + 0.1 * rng.normal(size=i.shape), 0, 1).astype(np.float32) for i in imgs]
    x = torch.from_numpy(np.concatenate([i.reshape(-1) for i in imgs])).to(dev())
    y = torch.from_numpy(np.concatenate([t.reshape(-1) for t in tgts])).to(dev())
    return imgs, tgts, x, y


def _static(lib, x, y, dims, kind, lam, g, loss):
    from paper_2601_09417_amd import _lib as L
    d = np.ascontiguousarray(np.asarray(dims, np.int32).reshape(-1, 2))
    st = lib.vbm_image_loss_static(x.data_ptr(), y.data_ptr(), d.ctypes.data_as(C.POINTER(C.c_int32)), d.shape[0],
                                   kind, lam, g.data_ptr(), loss.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return st, L


def _workspace(lib, x, y, dims, kind, lam, g, loss):
    d = np.ascontiguousarray(np.asarray(dims, np.int32).reshape(-1, 2))
    nb = lib.vbm_image_loss_workspace_size(d.ctypes.data_as(C.POINTER(C.c_int32)), d.shape[0], kind)
    ws = torch.empty(max(int(nb), 1), dtype=torch.uint8, device=dev())
    st = lib.vbm_image_loss(x.data_ptr(), y.data_ptr(), d.ctypes.data_as(C.POINTER(C.c_int32)), d.shape[0], kind, lam,
                            g.data_ptr(), loss.data_ptr(), ws.data_ptr(), ws.numel(),
                            torch.cuda.current_stream().cuda_stream)
    return st, nb


@pytest.mark.parametrize("kind", [0, 1])
def test_static_scratch_loss_matches_workspace_loss(kind):
    from paper_2601_09417_amd import _lib as L
    lib = L.load()
    lam = 0.2
    name = "l1" if kind == 0 else "l1_dssim"
    big = [(320, 240), (320, 240), (131, 77), (640, 480)]
    small = [(37, 29), (64, 48)]
    for call, dims in enumerate((big, small)):
        imgs, tgts, x, y = _batch(dims, 10 * kind + call)
        g_s, g_w = torch.full_like(x, np.nan), torch.full_like(x, np.nan)
        l_s = torch.full((1,), np.nan, device=dev())
        l_w = torch.full((1,), np.nan, device=dev())
        st, _ = _static(lib, x, y, dims, kind, lam, g_s, l_s)
        assert st == 0, lib.vbm_last_error()
        st, nb = _workspace(lib, x, y, dims, kind, lam, g_w, l_w)
        assert st == 0, lib.vbm_last_error()
        torch.cuda.synchronize()
        say(f"  {name} call {call}: {len(dims)} views, {nb} bytes of scratch; loss {float(l_s):.6f}")
        # the same kernels in the same order on the same values: identical bit for bit
        assert torch.equal(l_s, l_w) and torch.equal(g_s, g_w)
        # and within the loss tolerances of the oracle
        ref_loss, ref_g = oloss.loss_and_grad(imgs, tgts, name)
        assert abs(float(l_s) - ref_loss) <= 1e-5 * abs(ref_loss)
        rg = np.concatenate([a.reshape(-1) for a in ref_g])
        assert np.abs(g_s.cpu().numpy() - rg).max() <= 1e-4 * np.abs(rg).max()


def test_static_scratch_loss_refuses_beyond_its_size():
    from paper_2601_09417_amd import _lib as L
    lib = L.load()
    dims = [(2048, 1024)]                       # D-SSIM: 2M pixels x 36 bytes > 64 MiB
    x = torch.zeros(8, device=dev())
    g = torch.full_like(x, 7.0)
    loss = torch.full((1,), 7.0, device=dev())
    st, _ = _static(lib, x, x, dims, 1, 0.2, g, loss)
    assert st == -5, st                          # VBM_ERR_CAPACITY
    assert "64" in lib.vbm_last_error().decode() or "scratch" in lib.vbm_last_error().decode()
    torch.cuda.synchronize()
    assert torch.all(g == 7.0) and float(loss) == 7.0         # nothing was launched
    # L1 of the same size needs a few KiB and runs
    big = torch.rand(3 * 2048 * 1024, device=dev())
    tgt = torch.rand_like(big)
    gb = torch.empty_like(big)
    lb = torch.zeros(1, device=dev())
    st, _ = _static(lib, big, tgt, dims, 0, 0.2, gb, lb)
    assert st == 0
    torch.cuda.synchronize()
    ref = float((big - tgt).abs().double().mean())
    assert abs(float(lb) - ref) <= 1e-5 * ref
