"""Seeded synthetic inputs for the P_N step (shared by the tests, the oracle
runs and the benchmark; holds none of the method's arithmetic).

Each recipe returns a Workload: the medium (sigma_a, sigma_s, q as cell-centred
[z, y, x] float64 arrays), the grid, the time step and a generator of the
initial moments, one moment plane at a time so that large grids never need a
full FP64 copy of the state in host memory.

Domain [0, 1)^3, periodic, h = 1/n, cell centres (c + 1/2) h; distances are
periodic minimum-image distances; Gaussians are exp(-d^2 / (2 w^2)).
The paper uses no public dataset: its workloads are block sizes and a reactor
geometry, so these recipes stand in for them.

  p3_pulse     P3, 32^3, 64 steps: Gaussian pulse, blockwise random medium
  p7_lattice   P7, 128^3, 400 steps: 7^3 block lattice of absorbers, centre source
  p39_smooth   P39, 64^3, 100 steps: smooth random medium, 3 pulses + noise
  p39_large    the p39_smooth recipe at 160^3, 50 steps
  p7_adjoint   P7, 64^3, 200 steps, checkpoints every 20: gradient workload
  reactor      P19, 500^3: stand-in for the reactor-vessel showcase
"""
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np


@dataclass
class Workload:
    name: str
    N: int
    n: int                      # cells per direction (cubic box)
    nsteps: int
    sigma_a: np.ndarray
    sigma_s: np.ndarray
    q: Optional[np.ndarray]
    moment_fn: Callable[[int], np.ndarray]
    seed: int
    checkpoint: int = 0
    target: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    @property
    def V(self):
        return (self.N + 1) ** 2

    @property
    def shape(self):
        return (self.n, self.n, self.n)

    @property
    def h(self):
        return 1.0 / self.n

    @property
    def dt(self):
        return 0.5 * self.h

    def moment(self, i):
        """Initial value of moment i (canonical index l^2 + l + m), [z, y, x]."""
        return self.moment_fn(i)

    def initial(self):
        """All initial moments, shape (V, n, n, n) float64 (small grids only)."""
        return np.stack([self.moment(i) for i in range(self.V)])

    def moment_device(self, i, device):
        """Initial moment i as a float64 torch tensor on `device`.  Recipes
        with a `device_moment_fn` draw their noise there (large grids);
        otherwise the host plane is copied."""
        import torch
        fn = self.extra.get("device_moment_fn")
        if fn is not None:
            return fn(i, device)
        return torch.from_numpy(self.moment(i)).to(device)


def _device_zeros(n):
    """Zero initial moments made on the device (no host plane to copy)."""
    def fn(i, device):
        import torch
        return torch.zeros((n, n, n), dtype=torch.float64, device=device)
    return fn


def _coords(n):
    c = (np.arange(n) + 0.5) / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return x, y, z


def _periodic_d2(n, centre):
    x, y, z = _coords(n)
    d2 = np.zeros_like(x)
    for a, c in zip((x, y, z), centre):
        d = np.abs(a - c)
        d = np.minimum(d, 1.0 - d)
        d2 += d * d
    return d2


def gaussian(n, centre, width):
    return np.exp(-_periodic_d2(n, centre) / (2.0 * width * width))


def blockwise(n, block, values):
    """Piecewise-constant field on cubes of `block` cells; values[bz, by, bx]."""
    idx = np.arange(n) // block
    return values[np.ix_(idx, idx, idx)]


def p3_pulse(seed=0, n=32, N=3, nsteps=64):
    """P3 pulse: sigma_s ~ U[0,1], sigma_a ~ U[0,0.5] per 4^3 block, q = 0,
    zeroth moment a Gaussian (w = 0.1) at a centre ~ U[0,1)^3, others 0."""
    rng = np.random.default_rng(seed)
    nb = -(-n // 4)
    ss = blockwise(n, 4, rng.uniform(0.0, 1.0, (nb, nb, nb)))
    sa = blockwise(n, 4, rng.uniform(0.0, 0.5, (nb, nb, nb)))
    centre = rng.uniform(0.0, 1.0, 3)
    g = gaussian(n, centre, 0.1)

    def moment(i):
        return g.copy() if i == 0 else np.zeros((n, n, n))

    return Workload("p3_pulse", N, n, nsteps, sa, ss, None, moment, seed,
                    extra={"centre": centre.tolist()})


def p7_lattice(seed=1, n=128, N=7, nsteps=400):
    """7x7x7 block lattice, block index b_d = floor(7 c_d / n).  Blocks with an
    even index sum are absorbers (sigma_a = 10, sigma_s = 0) with probability
    1/2 each; all others sigma_a = 0, sigma_s = 1.  q = 1 on the centre block
    (3,3,3), whose index sum is odd.  Initial state zero."""
    rng = np.random.default_rng(seed)
    b = (7 * np.arange(n)) // n
    bz, by, bx = np.meshgrid(b, b, b, indexing="ij")
    keep = rng.uniform(size=(7, 7, 7)) < 0.5
    absorber = ((bx + by + bz) % 2 == 0) & keep[bz, by, bx]
    sa = np.where(absorber, 10.0, 0.0)
    ss = np.where(absorber, 0.0, 1.0)
    q = ((bx == 3) & (by == 3) & (bz == 3)).astype(np.float64)

    def moment(i):
        return np.zeros((n, n, n))

    return Workload("p7_lattice", N, n, nsteps, sa, ss, q, moment, seed,
                    extra={"device_moment_fn": _device_zeros(n)})


def smooth_field(n, rng, modes=8, kmax=4):
    """f = clip(0.5 + 0.25 g, 0, 1), g = sum_k a_k cos(2 pi n_k . x + phi_k)."""
    x, y, z = _coords(n)
    g = np.zeros((n, n, n))
    for _ in range(modes):
        while True:
            kv = rng.integers(-kmax, kmax + 1, 3)
            if np.any(kv != 0):
                break
        a = rng.uniform(0.0, 1.0)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        g += a * np.cos(2.0 * np.pi * (kv[0] * x + kv[1] * y + kv[2] * z) + ph)
    return np.clip(0.5 + 0.25 * g, 0.0, 1.0)


def p39_smooth(seed=2, n=64, N=39, nsteps=100, name="p39_smooth"):
    """sigma_a = 0.1 + 0.4 f (smooth random f in [0,1]), sigma_s = 1 - sigma_a,
    q = 0; zeroth moment = sum of 3 Gaussians (w = 0.05) at centres ~ U[0,1)^3;
    every higher moment i.i.d. N(0, 1e-3^2), drawn per moment from the
    generator seeded with (seed, i)."""
    rng = np.random.default_rng(seed)
    f = smooth_field(n, rng)
    sa = 0.1 + 0.4 * f
    ss = 1.0 - sa
    centres = rng.uniform(0.0, 1.0, (3, 3))
    g = sum(gaussian(n, c, 0.05) for c in centres)

    def moment(i):
        if i == 0:
            return g.copy()
        return np.random.default_rng([seed, i]).normal(0.0, 1e-3, (n, n, n))

    return Workload(name, N, n, nsteps, sa, ss, None, moment, seed,
                    extra={"centres": centres.tolist()})


def p39_aniso(seed=2, n=64, N=39, nsteps=100, asym=0.8):
    """The p39_smooth recipe with anisotropic (forward-peaked) scattering:
    Henyey-Greenstein phase function of asymmetry 0.8, whose Legendre
    moments are g_l = 0.8^l, so degree l has c_l = sigma_a + (1 - g_l) sigma_s."""
    w = p39_smooth(seed=seed, n=n, N=N, nsteps=nsteps, name="p39_aniso")
    w.extra["scattering"] = [asym ** l for l in range(1, N + 1)]
    return w


def p39_large(seed=2, n=160, N=39, nsteps=50):
    """The p39_smooth recipe at 160^3.  Drawing 6.5e9 normals on the host
    takes about a minute, so the N(0, 1e-3^2) noise of moments i >= 1 is
    drawn on the GPU by torch's generator seeded with seed * 100003 + i;
    `moment(i)` returns the same values on the host (via the device)."""
    w = p39_smooth(seed=seed, n=n, N=N, nsteps=nsteps, name="p39_large")
    g0 = w.moment_fn(0)

    def device_moment(i, device):
        import torch
        if i == 0:
            return torch.from_numpy(g0).to(device)
        gen = torch.Generator(device=device)
        gen.manual_seed(seed * 100003 + i)
        return 1e-3 * torch.randn((n, n, n), generator=gen, dtype=torch.float64, device=device)

    w.extra["device_moment_fn"] = device_moment
    w.moment_fn = lambda i: device_moment(i, "cuda").cpu().numpy() if i else g0.copy()
    return w


def p7_adjoint(seed=3, n=64, N=7, nsteps=200, checkpoint=20):
    """Gradient workload: the p3_pulse medium recipe (4^3 blocks, sigma_s ~
    U[0,1], sigma_a ~ U[0,0.5]) and a Gaussian pulse (w = 0.1); the target is
    u_0(T) of the same run with sigma_a scaled by (1 + U[-0.1, 0.1]) per 4^3
    block.  Returns the workload; the target must be computed by a forward
    run with `perturbed_sigma_a`."""
    w = p3_pulse(seed=seed, n=n, N=N, nsteps=nsteps)
    rng = np.random.default_rng([seed, 99])
    nb = -(-n // 4)
    factor = blockwise(n, 4, 1.0 + rng.uniform(-0.1, 0.1, (nb, nb, nb)))
    w.name = "p7_adjoint"
    w.checkpoint = checkpoint
    w.extra["perturbed_sigma_a"] = w.sigma_a * factor
    return w


def reactor(seed=4, n=500, N=19, nsteps=20, name="reactor"):
    """Stand-in for the reactor-vessel showcase: a cube of n^3 cells of
    0.2 cm (n = 500: 1 m) with an outer concrete shell, a water box and a
    core of vertical fuel rods 5 cells (1 cm) thick.  Printed: rods 1 cm
    thick, q0 = 2, Sigma_a = 10 in water and 5 in concrete, Sigma_s = 1.
    Not printed (readings): concrete shell 10 % of the edge on every side,
    core = the central 50 % of the edge in x and y and 70 % in z, square rod
    lattice with a pitch of 3 rod widths, rods with Sigma_a = 0 and the
    source q = 2, Sigma_s = 1 everywhere, initial state zero.  `seed` only
    shifts the rod lattice by up to one pitch."""
    rng = np.random.default_rng(seed)
    c = np.arange(n)
    shell = max(1, int(round(0.1 * n)))
    rod = max(1, int(round(n / 100)))            # 1 cm on a 1 m box
    pitch = 3 * rod
    off = int(rng.integers(0, pitch))
    core_xy = (c >= n // 4) & (c < n - n // 4)
    core_z = (c >= int(0.15 * n)) & (c < n - int(0.15 * n))
    in_rod = ((c - n // 4 + off) % pitch) < rod
    z, y, x = np.meshgrid(c, c, c, indexing="ij", sparse=True)
    concrete = ((x < shell) | (x >= n - shell) | (y < shell) | (y >= n - shell) |
                (z < shell) | (z >= n - shell))
    rods = core_xy[x] & core_xy[y] & core_z[z] & in_rod[x] & in_rod[y]
    sa = np.where(concrete, 5.0, np.where(rods, 0.0, 10.0))
    ss = np.ones((n, n, n))
    q = np.where(rods & ~concrete, 2.0, 0.0)

    def moment(i):
        return np.zeros((n, n, n))

    w = Workload(name, N, n, nsteps, sa, ss, q, moment, seed,
                 extra={"rod": rod, "pitch": pitch, "shell": shell, "offset": off,
                        "device_moment_fn": _device_zeros(n)})
    return w


RECIPES = {
    "p3_pulse": p3_pulse,
    "p7_lattice": p7_lattice,
    "p39_smooth": p39_smooth,
    "p39_large": p39_large,
    "p39_aniso": p39_aniso,
    "p7_adjoint": p7_adjoint,
    "reactor": reactor,
}
