"""Halo faces of a split box on the GPU: pm_halo_pack gathers exactly the
(moment, cell) elements of the face map (pm_halo_plan, checked on the CPU
against the reflection parities), and pm_halo_unpack scatters a buffer
back into exactly those elements, leaving every other value unchanged."""
import numpy as np
import pytest

import paper_2004_02833_amd as pm

from gpu_util import gpu_init, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TDT = {pm.PM_FP64: torch.float64, pm.PM_FP32: torch.float32, pm.PM_BF16: torch.bfloat16}


def read_all(V, shape):
    return np.stack([pm.pm_read(i) for i in range(V)]).reshape(V, -1)


@pytest.mark.parametrize("N,shape,prec", [(3, (6, 5, 64), pm.PM_FP64), (7, (4, 6, 96), pm.PM_FP32),
                                          (3, (5, 4, 7), pm.PM_BF16), (2, (1, 3, 160), pm.PM_FP64)])
def test_halo_pack_unpack(N, shape, prec):
    say("case halo", N, shape, prec)
    nz, ny, nx = shape
    V = (N + 1) ** 2
    rng = np.random.default_rng(5 + N)
    dev = torch.device("cuda", 0)
    gpu_init(N, shape, 0.1, 0.02, rng.uniform(0, 1, shape), rng.uniform(0, 1, shape), None, prec)
    try:
        pm.pm_bind_stream(torch.cuda.current_stream(dev).cuda_stream)
        for i in range(V):
            pm.pm_write(i, rng.normal(size=shape))
        for parity, dirs in ((0, 7), (1, 7), (1, 6), (0, 5)):
            n, mom, cell = pm.pm_halo_plan(N, nx, ny, nz, parity, dirs, with_index=True)
            state = read_all(V, shape)
            buf = torch.empty(n, dtype=TDT[prec], device=dev)
            pm.pm_halo_pack(parity, buf.data_ptr(), dirs)
            got = buf.double().cpu().numpy()
            assert np.array_equal(got, state[mom, cell])
            # unpack a changed buffer: exactly the face elements change
            new = (-2.0 * buf.double() + 1.0).to(TDT[prec])
            pm.pm_halo_unpack(parity, new.data_ptr(), dirs)
            after = read_all(V, shape)
            want = state.copy()
            want[mom, cell] = new.double().cpu().numpy()
            assert np.array_equal(after, want)
            # and the original buffer restores the state bit for bit
            pm.pm_halo_unpack(parity, buf.data_ptr(), dirs)
            assert np.array_equal(read_all(V, shape), state)
    finally:
        pm.pm_finalize()
        pm.pm_bind_stream(0)
