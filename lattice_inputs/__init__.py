"""Seeded synthetic inputs for the periodic 2D lattice Schroedinger problem.

This module is the only code shared by the CPU oracle and the GPU path.  It
holds no arithmetic of the MB4 method: it only draws the on-site potential
(disorder plus defect sites) and the initial wavepacket from seeds, so both
sides integrate exactly the same problem.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: the i-th draw of a (seed, stream) pair is the SplitMix64 output
function applied to ``key(seed, stream) + (i + 1) * GAMMA``, where GAMMA is
the golden-ratio increment of that paper.  A uniform double in [0, 1) takes
the top 53 bits of the 64-bit output.

Site order is x fastest: site = y * nx + x (the paper's ((j-1) Nx + i)
ordering of Sec. 2.1, zero-based).
"""
from __future__ import annotations

from dataclasses import asdict, dataclass, field, replace
import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

STREAM_DISORDER = 0
STREAM_DEFECTS = 1
STREAM_AMPLITUDE = 2
STREAM_PHASE = 3
STREAM_NONLINEARITY = 4


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (variant 13 of Stafford's mixers)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    """Key of one (seed, stream) pair: a SplitMix64 output of the packed pair."""
    s = np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    with np.errstate(over="ignore"):
        packed = (s * GAMMA) ^ np.uint64(stream)
    return _mix64(packed)[0]


def draw_u64(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Draws start .. start+n-1 of the (seed, stream) counter-based sequence."""
    key = stream_key(seed, stream)
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(key + idx * GAMMA)


def draw_uniform(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of each draw."""
    u = draw_u64(seed, stream, n, start) >> np.uint64(11)
    return u.astype(np.float64) * (1.0 / 9007199254740992.0)


@dataclass
class LatticeProblem:
    """One synthetic workload: lattice, potential recipe, wavepacket, step."""

    name: str
    nx: int
    ny: int
    t_hop: float = 1.0
    diag_shift: float = 0.0
    disorder_w: float = 1.0        # V_j ~ Uniform[-W/2, W/2]
    defect_count: int = 0          # number of distinct defect sites
    defect_v: float = 50.0         # potential at a defect (replaces disorder)
    g: float = 1.0                 # nonlinearity: i psi' = (A + g|psi|^2) psi
    sigma: float = 3.0             # wavepacket width in sites
    kx: float = math.pi / 4
    ky: float = 0.0
    h: float = 0.01
    steps: int = 1000
    seed: int = 1
    energy_every: int = 0          # log energy every this many steps (0: ends only)
    initial: str = "wavepacket"    # "wavepacket", "cosine" (1 + 2 cos x + 2 cos y) or
                                   # "random" (independent amplitude and phase per site)
    normalise: bool = True         # scale the initial state to sum |psi|^2 = 1
    origin_v: float | None = None  # potential at site 0 (the grid origin), if set
    centre: tuple | None = None    # wavepacket centre (x, y); None: (nx // 2, ny // 2)
    amp_range: tuple = (0.1, 0.5)  # "random": |psi_j| ~ Uniform[lo, hi]
    g_range: tuple | None = None   # per-site nonlinearity g_j ~ Uniform[lo, hi]
                                   # (stream 4) in place of g, if set
    extra: dict = field(default_factory=dict)

    @property
    def sites(self) -> int:
        return self.nx * self.ny

    def as_dict(self) -> dict:
        return asdict(self)


def make_potential(prob: LatticeProblem) -> np.ndarray:
    """On-site potential V (length nx*ny): disorder plus defect sites.

    Disorder is i.i.d. Uniform[-W/2, W/2] from stream 0.  Defects are
    ``defect_count`` distinct sites, chosen as the sites with the smallest
    stream-1 draws (ties, which need equal 64-bit draws, go to the lower
    site); a defect's value replaces the disorder value there.
    """
    s = prob.sites
    v = prob.disorder_w * (draw_uniform(prob.seed, STREAM_DISORDER, s) - 0.5)
    if prob.defect_count > 0:
        if prob.defect_count > s:
            raise ValueError("more defects than sites")
        keys = draw_u64(prob.seed, STREAM_DEFECTS, s)
        order = np.argsort(keys, kind="stable")
        v[order[: prob.defect_count]] = prob.defect_v
    if prob.origin_v is not None:
        v[0] = prob.origin_v
    return v


def make_wavepacket(prob: LatticeProblem) -> tuple[np.ndarray, np.ndarray]:
    """Normalised Gaussian wavepacket, returned as (p, q) = (Re psi, Im psi).

    psi_j = exp(-d_j^2 / (2 sigma^2) + i k.r_j) with d_j the minimum-image
    distance from site j to the centre (nx//2, ny//2 unless prob.centre
    names another site) and r_j = (x, y) the integer coordinates; then
    scaled so that sum |psi_j|^2 = 1.
    """
    x = np.arange(prob.nx, dtype=np.float64)
    y = np.arange(prob.ny, dtype=np.float64)
    cx, cy = (prob.nx // 2, prob.ny // 2) if prob.centre is None else prob.centre
    dx = np.abs(x - cx)
    dx = np.minimum(dx, prob.nx - dx)
    dy = np.abs(y - cy)
    dy = np.minimum(dy, prob.ny - dy)
    d2 = dy[:, None] ** 2 + dx[None, :] ** 2
    amp = np.exp(-d2 / (2.0 * prob.sigma ** 2))
    phase = prob.kx * x[None, :] + prob.ky * y[:, None]
    p = (amp * np.cos(phase)).reshape(-1)
    q = (amp * np.sin(phase)).reshape(-1)
    norm = math.sqrt(math.fsum((p * p).tolist()) + math.fsum((q * q).tolist()))
    return p / norm, q / norm


def make_cosine(prob: LatticeProblem) -> tuple[np.ndarray, np.ndarray]:
    """The initial condition of Sec. 3, u(x, y) = 1 + 2 cos x + 2 cos y, on the
    grid x_i = 2 pi i / nx, y_j = 2 pi j / ny of [0, 2 pi)^2 (real: q = 0);
    scaled to sum |u_j|^2 = 1 if prob.normalise."""
    x = 2.0 * math.pi * np.arange(prob.nx, dtype=np.float64) / prob.nx
    y = 2.0 * math.pi * np.arange(prob.ny, dtype=np.float64) / prob.ny
    p = (1.0 + 2.0 * np.cos(x)[None, :] + 2.0 * np.cos(y)[:, None]).reshape(-1)
    q = np.zeros_like(p)
    if prob.normalise:
        p = p / math.sqrt(math.fsum((p * p).tolist()))
    return p, q


def make_random_field(prob: LatticeProblem) -> tuple[np.ndarray, np.ndarray]:
    """A delocalised state with signal on every site: |psi_j| uniform in
    prob.amp_range (stream 2) and arg psi_j uniform in [0, 2 pi) (stream 3),
    independently per site; not normalised."""
    lo, hi = prob.amp_range
    amp = lo + (hi - lo) * draw_uniform(prob.seed, STREAM_AMPLITUDE, prob.sites)
    ph = 2.0 * math.pi * draw_uniform(prob.seed, STREAM_PHASE, prob.sites)
    return amp * np.cos(ph), amp * np.sin(ph)


def make_nonlinearity(prob: LatticeProblem) -> np.ndarray | None:
    """Per-site nonlinearity g_j (length nx*ny), i.i.d. Uniform[lo, hi] from
    stream 4, when the problem has a g_range; None for the uniform g."""
    if prob.g_range is None:
        return None
    lo, hi = prob.g_range
    return np.ascontiguousarray(lo + (hi - lo) * draw_uniform(prob.seed, STREAM_NONLINEARITY,
                                                               prob.sites))


def make_inputs(prob: LatticeProblem) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(V, p0, q0) for a problem; all float64 and C-contiguous."""
    v = make_potential(prob)
    if prob.initial == "cosine":
        p, q = make_cosine(prob)
    elif prob.initial == "random":
        p, q = make_random_field(prob)
    elif prob.initial == "wavepacket":
        p, q = make_wavepacket(prob)
    else:
        raise ValueError(f"unknown initial state {prob.initial!r}")
    return (np.ascontiguousarray(v), np.ascontiguousarray(p),
            np.ascontiguousarray(q))


def _defects(density: float, sites: int) -> int:
    return int(round(density * sites))


# The five workloads: plain runs at 32^2, 256^2 and 2048^2, the ensemble of
# 128^2 realisations and the serving mix.  Unstated parameters follow one
# fixed reading (listed with the input recipe in the design notes).
CONFIGS: dict[str, LatticeProblem] = {
    "lattice32": LatticeProblem(
        name="lattice32", nx=32, ny=32, disorder_w=1.0, defect_count=4,
        defect_v=50.0, g=1.0, sigma=3.0, kx=math.pi / 4, ky=0.0, h=0.01,
        steps=1000, seed=1),
    "lattice256": LatticeProblem(
        name="lattice256", nx=256, ny=256, disorder_w=1.0,
        defect_count=_defects(0.005, 256 * 256), defect_v=50.0, g=1.0,
        sigma=8.0, kx=math.pi / 4, ky=0.0, h=0.01, steps=10000, seed=2,
        energy_every=100),
    "lattice2048": LatticeProblem(
        name="lattice2048", nx=2048, ny=2048, disorder_w=2.0,
        defect_count=_defects(0.001, 2048 * 2048), defect_v=100.0, g=2.0,
        sigma=32.0, kx=math.pi / 2, ky=math.pi / 4, h=0.005, steps=2000,
        seed=3),
}
# The 2048^2 workload with its packet centred on the lattice corner: the
# packet wraps around all four edges, so the periodic wrap and the partial
# right and top tiles of a full-size run carry signal.
CONFIGS["lattice2048corner"] = replace(CONFIGS["lattice2048"], name="lattice2048corner",
                                       centre=(0, 0))


def continuum_hopping(n: int) -> float:
    """1 / h_x^2 for n points on [0, 2 pi): the hopping of K = -Delta_h
    (Eq. Kdefinition), whose diagonal is 4 / h_x^2 on a square grid."""
    return (n / (2.0 * math.pi)) ** 2


# The paper's own continuum runs (Sec. 3): K = -Delta_h on [0, 2 pi)^2 with
# periodic boundaries, u_0 = 1 + 2 cos x + 2 cos y, g = -gamma.
#   continuum70: the comparison runs, 70 x 70, V = 0, gamma = 0.1, h = 0.01,
#     u_0 as given (max 5).  Taken literally this focusing problem
#     concentrates (max |u| 5 -> 32 by t = 0.86) and the simplified Newton
#     iteration at h = 0.01 stops converging at t = 0.87, so the workload
#     runs t in [0, 0.5] rather than the paper's [0, 1].
#   delta100: the delta-function-like potential, 100 x 100, V = -50 at the
#     origin and 0 elsewhere, gamma = 0.05, h = 0.01 up to t = 20; u_0
#     normalised to sum |u|^2 = 1 (the paper's participation ratio 1/(Nx Ny)
#     of a uniform density implies that normalisation).
CONFIGS["continuum70"] = LatticeProblem(
    name="continuum70", nx=70, ny=70, t_hop=continuum_hopping(70),
    diag_shift=4.0 * continuum_hopping(70), disorder_w=0.0, defect_count=0, g=-0.1,
    initial="cosine", normalise=False, h=0.01, steps=50, seed=4, energy_every=5)
CONFIGS["delta100"] = LatticeProblem(
    name="delta100", nx=100, ny=100, t_hop=continuum_hopping(100),
    diag_shift=4.0 * continuum_hopping(100), disorder_w=0.0, defect_count=0, g=-0.05,
    initial="cosine", normalise=True, origin_v=-50.0, h=0.01, steps=2000, seed=5,
    energy_every=125)


def ensemble_member(r: int, side: int = 128, steps: int = 5000) -> LatticeProblem:
    """Realisation r of the 128^2 disorder ensemble (seed 1000 + r)."""
    return LatticeProblem(
        name=f"ensemble128_r{r}", nx=side, ny=side, disorder_w=1.0,
        defect_count=_defects(0.005, side * side), defect_v=50.0, g=1.0,
        sigma=8.0, kx=math.pi / 4, ky=0.0, h=0.01, steps=steps, seed=1000 + r)


# The disorder ensemble: ENSEMBLE_SIZE realisations of ensemble_member, each
# run for ENSEMBLE_STEPS steps.
ENSEMBLE_SIZE = 512
ENSEMBLE_STEPS = 5000


def ensemble(size: int = ENSEMBLE_SIZE) -> list[LatticeProblem]:
    return [ensemble_member(r) for r in range(size)]


# The serving mix: solve requests arriving as a Poisson process, each with
# its own lattice side, step count, nonlinearity and disorder realisation.
SERVING_SIDES = (64, 128, 256, 512, 1024)
SERVING_RATE = 200.0          # mean arrivals per second
SERVING_STEPS = (100, 5000)   # uniform, inclusive
SERVING_TRACE_SEED = 7000


def serving_request(rid: int) -> LatticeProblem:
    """Request rid of the serving mix (its disorder seed is rid): side drawn
    uniformly from SERVING_SIDES, steps uniform in SERVING_STEPS, g uniform in
    [0, 2]; W = 1 disorder with 0.5% defects at +50, sigma 8 (32 for the
    largest side), k = (pi/4, 0), h = 0.01."""
    u = draw_uniform(rid, 10, 3)
    side = SERVING_SIDES[min(int(u[0] * len(SERVING_SIDES)), len(SERVING_SIDES) - 1)]
    lo, hi = SERVING_STEPS
    steps = lo + min(int(u[1] * (hi - lo + 1)), hi - lo)
    return LatticeProblem(
        name=f"serving_r{rid}", nx=side, ny=side, disorder_w=1.0,
        defect_count=_defects(0.005, side * side), defect_v=50.0, g=2.0 * float(u[2]),
        sigma=32.0 if side >= 1024 else 8.0, kx=math.pi / 4, ky=0.0, h=0.01, steps=steps,
        seed=rid)


def serving_trace(n: int, rate: float = SERVING_RATE,
                  seed: int = SERVING_TRACE_SEED) -> list[tuple[float, LatticeProblem]]:
    """n requests (ids 1 .. n) with Poisson arrival times at `rate` per
    second: exponential gaps -ln(1 - u) / rate from the seeded generator."""
    u = draw_uniform(seed, 11, n)
    t = np.cumsum(-np.log1p(-u) / rate)
    return [(float(t[i]), serving_request(i + 1)) for i in range(n)]


def config(name: str, **overrides) -> LatticeProblem:
    """A copy of a named workload with some fields replaced."""
    base = CONFIGS[name].as_dict()
    base.update(overrides)
    return LatticeProblem(**base)
