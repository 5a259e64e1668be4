"""The allocation-free binning entry point (mot_bin_points_noalloc) through the C ABI:
bit for bit the results of mot_bin_points, on two calls in a row (the second smaller, so
it runs on scratch the first one filled), with and without the sub-key, and the size
limit refused before any device work."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _call_noalloc(mot, x, s, o, n, T, sub_dim):
    import torch
    dev = torch.device("cuda")
    npts, d = x.shape
    tpd = (n + T - 1) // T
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    cell = torch.full((max(npts, 1), d), -7, dtype=torch.int32, device=dev)
    perm = torch.full((max(npts, 1),), -7, dtype=torch.int32, device=dev)
    toff = torch.full((tpd ** d + 1,), -7, dtype=torch.int32, device=dev)
    sh = np.ascontiguousarray(np.broadcast_to(s, (d,)), dtype=np.float64)
    oh = np.ascontiguousarray(np.broadcast_to(o, (d,)), dtype=np.float64)
    ip = ctypes.POINTER(ctypes.c_int32)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = mot.lib().mot_bin_points_noalloc(d, npts, ctypes.cast(xd.data_ptr(), dp), sh.ctypes.data_as(dp),
                                          oh.ctypes.data_as(dp), n, T, sub_dim,
                                          ctypes.cast(cell.data_ptr(), ip), ctypes.cast(perm.data_ptr(), ip),
                                          ctypes.cast(toff.data_ptr(), ip), mot.current_stream())
    assert rc == mot.OK, rc
    torch.cuda.synchronize()
    return cell.cpu().numpy()[:npts], perm.cpu().numpy()[:npts], toff.cpu().numpy()


@pytest.mark.parametrize("sub_dim", [1, -1])
def test_noalloc_binning_equals_mot_bin_points(sub_dim):
    from paper_2208_03120_amd import mot
    r = np.random.Generator(np.random.PCG64(140 + sub_dim))
    for npts, n, T in [(150_000, 128, 5), (40_000, 64, 5)]:  # second call smaller
        x = r.uniform(-0.3, 0.3, size=(npts, 3))
        x[:5] = np.round(x[:5] * 64) / 64
        s = np.full(3, n / 2.0)
        o = n / 2.0 + r.uniform(-0.5, 0.5, size=3)
        cell, perm, toff = _call_noalloc(mot, x, s, o, n, T, sub_dim)
        rcell, rperm, rtoff = mot.bin_points(x, s, o, n, T, sub_dim=sub_dim)
        np.testing.assert_array_equal(cell, rcell)
        np.testing.assert_array_equal(perm, rperm)
        np.testing.assert_array_equal(toff, rtoff)


def test_noalloc_binning_size_limit():
    from paper_2208_03120_amd import mot
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    one = np.ones(3)
    # refused on the host, before any pointer is touched
    rc = mot.lib().mot_bin_points_noalloc(3, (1 << 20) + 1, ctypes.cast(1, dp), one.ctypes.data_as(dp),
                                          one.ctypes.data_as(dp), 64, 5, 1, ctypes.cast(1, ip),
                                          ctypes.cast(1, ip), ctypes.cast(1, ip), None)
    assert rc == mot.ELIMIT
