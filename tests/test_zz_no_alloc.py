"""The entry point that allocates no device memory (perm_bbfg_noalloc) against
perm_bbfg through the C ABI: same plan and kernels, so the same bits, on two
calls in a row (the second with a smaller input, so it runs on what the first
left in the shared scratch array), with host and device buffers, and its edge
cases.  It also checks that the calls allocate no device memory."""
import numpy as np
import pytest

from paper_2309_07027_amd import binding as B
from paper_2309_07027_amd import inputs as I

pytestmark = pytest.mark.gpu


def _device_bytes_in_use():
    import torch
    free, total = torch.cuda.mem_get_info()
    return total - free


def test_noalloc_matches_perm_bbfg_twice_second_smaller():
    import torch
    B.init()
    A30, M30 = I.c2a()
    A14, M14 = I.random_instance(np.random.default_rng(8), 14, m=9)
    ref30, i30 = B.perm_bbfg(A30, M30, with_info=True)
    ref14, i14 = B.perm_bbfg(A14, M14, with_info=True)
    torch.cuda.synchronize()
    used0 = _device_bytes_in_use()
    got30, n30 = B.perm_bbfg_noalloc(A30, M30, with_info=True)
    got14, n14 = B.perm_bbfg_noalloc(A14, M14, with_info=True)
    torch.cuda.synchronize()
    assert _device_bytes_in_use() == used0
    assert got30 == ref30 and got14 == ref14          # same plan and kernels: same bits
    assert abs(got30 - ref30) <= 1e-10 * abs(ref30)
    assert n30["rel_err_est"] == i30["rel_err_est"] and n14["kappa"] == i14["kappa"]
    assert n30["n_units"] == i30["n_units"] and n30["n_addends"] == 2 ** 29


def test_noalloc_device_buffers_and_edges():
    import torch
    B.init()
    A, M = I.c2c()
    ref = B.perm_bbfg(A, M)
    At = torch.from_numpy(A).to("cuda")
    assert B.perm_bbfg_noalloc(At, M) == ref
    # bunched rows, zero-multiplicity rows, the empty permanent, n = 1
    rng = np.random.default_rng(9)
    for n in (1, 2, 5, 17):
        Ar, Mr = I.random_instance(rng, n, m=4)
        assert B.perm_bbfg_noalloc(Ar, Mr) == B.perm_bbfg(Ar, Mr), n
    Z = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    assert B.perm_bbfg_noalloc(Z, [2, 0, 1, 0]) == B.perm_bbfg(Z, [2, 0, 1, 0])
    assert B.perm_bbfg_noalloc(np.zeros((0, 0), dtype=complex), np.zeros(0, dtype=np.int32)) == 1
    with pytest.raises(B.BBFGError) as e:
        B.perm_bbfg_noalloc(np.ones((49, 49), dtype=complex))
    assert e.value.code == B.BBFG_ERANGE
    with pytest.raises(B.BBFGError) as e:
        B.perm_bbfg_noalloc(np.ones((3, 3), dtype=complex), [1, 1, 2])
    assert e.value.code == B.BBFG_EINVAL
