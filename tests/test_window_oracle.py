"""The windowed oracle used for full-size GPU parity is exact: on a small
periodic grid, the central block of a periodic window run equals the
full-domain run bit for bit when the window margin is at least 3 cells per
step (and differs when it is not)."""
import numpy as np

from oracle import c_oracle

from gpu_util import window_index, window_oracle


def test_window_oracle_matches_full_domain():
    c_oracle.build(force=False)
    N, shape, B, k = 3, (22, 20, 24), 4, 2
    rng = np.random.default_rng(5)
    sa = rng.uniform(0, 0.5, shape)
    ss = rng.uniform(0, 1, shape)
    q = rng.uniform(0, 1, shape)
    u = rng.normal(size=(16,) + shape)
    h, dt = 1 / 24, 0.5 / 24
    full = c_oracle.run(N, shape, h, dt, sa, ss, q, u, k)
    for corner in ((0, 0, 0), (9, 15, 21)):
        R = 3 * k
        ix = window_index(shape, corner, B, R)
        got = window_oracle(N, shape, h, dt, sa, ss, q, u[(slice(None),) + np.ix_(*ix)], corner, B, R, k)
        cz, cy, cx = (np.arange(corner[d], corner[d] + B) % shape[d] for d in range(3))
        want = full[(slice(None),) + np.ix_(cz, cy, cx)]
        assert np.array_equal(got, want)
    # a margin below the dependence radius is visibly wrong
    R = 1
    ix = window_index(shape, (0, 0, 0), B, R)
    sub = np.ix_(*ix)
    bad = c_oracle.run(N, (B + 2 * R,) * 3, h, dt, sa[sub], ss[sub], q[sub],
                       u[(slice(None),) + sub], k)[:, R:R + B, R:R + B, R:R + B]
    assert not np.allclose(bad, full[:, :B, :B, :B], rtol=1e-6, atol=1e-9)
