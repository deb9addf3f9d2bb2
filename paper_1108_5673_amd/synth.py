"""Seeded synthetic partial-wave samples shaped like J/psi -> gamma X, X -> K+ K-.

The paper's benchmark analysis (Sec. 2 and Sec. 5) uses BES data and covariant
tensor amplitudes that are not available; these samples stand in for it with
the same structure: a coherent sum of resonances in the K+K- mass, each a
relativistic Breit-Wigner times a spin-dependent angular factor.

This module holds none of the likelihood arithmetic.  It draws kinematics,
evaluates the stand-in decay amplitudes, selects data events by accept-reject
from the coherent intensity at the generating parameters (the sampling density
only: no value it computes is passed on except the selected events' amplitudes)
and applies a random acceptance mask to flat Monte Carlo.  The lookup table,
the MC integral matrix, the likelihood and its gradient are computed separately
by the oracle and by the HIP library.

Recipe (all choices are stand-ins; the paper fixes none of them):
  * kinematics: m_KK ~ U[0.99, 2.8] GeV, cos(theta_gamma), cos(theta_K) ~ U[-1, 1]
    (flat in m, not phase-space weighted);
  * wave a: BW_a(m) = 1 / (M_a^2 - m^2 - i M_a Gamma_a), times the Legendre
    polynomial P_J(cos theta_K) for spin J, times sqrt((1 + cos^2 theta_gamma)/2);
  * wave list for W waves: masses linspace(1.0, 2.6, ceil(W/2))[a // 2],
    J = 0 for even a and 2 for odd a, Gamma = 0.15 GeV, unless given;
  * production amplitudes: Re and Im i.i.d. N(0, 1);
  * data: accept-reject from |sum_a V_a A_a|^2 at V_true with an envelope of 1.2x
    the maximum over a flat pre-sample; the whole draw restarts with a larger
    envelope if any candidate exceeds it;
  * MC: N_gen flat events, an exact-count random subset of N_acc is accepted;
  * seeds: numpy PCG64 from SeedSequence(SEED_BASE + workload index), spawned
    into independent streams for V_true, data, MC, the acceptance mask and the
    evaluation points.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 11085673
M_RANGE = (0.99, 2.8)


@dataclasses.dataclass(frozen=True)
class WaveSet:
    masses: tuple
    widths: tuple
    spins: tuple

    @property
    def n_waves(self) -> int:
        return len(self.masses)


def wave_set(n_waves: int, masses=None, widths=None, spins=None) -> WaveSet:
    """The wave list rule: resonance masses spread over 1.0-2.6 GeV, spins 0/2."""
    if masses is None:
        grid = np.linspace(1.0, 2.6, max(1, math.ceil(n_waves / 2)))
        masses = tuple(float(grid[a // 2]) for a in range(n_waves))
    if spins is None:
        spins = tuple(0 if a % 2 == 0 else 2 for a in range(n_waves))
    if widths is None:
        widths = tuple(0.15 for _ in range(n_waves))
    ws = WaveSet(tuple(map(float, masses)), tuple(map(float, widths)), tuple(map(int, spins)))
    assert len(ws.masses) == len(ws.widths) == len(ws.spins) == n_waves
    return ws


def legendre(j: int, x: np.ndarray) -> np.ndarray:
    """P_J(x) by the Bonnet recursion (P_J = d^J_00 for the K+K- decay angle)."""
    p0 = np.ones_like(x)
    if j == 0:
        return p0
    p1 = x.copy()
    for n in range(1, j):
        p0, p1 = p1, ((2 * n + 1) * x * p1 - n * p0) / (n + 1)
    return p1


def phase_space(rng: np.random.Generator, n: int):
    m = rng.uniform(M_RANGE[0], M_RANGE[1], n)
    cos_g = rng.uniform(-1.0, 1.0, n)
    cos_k = rng.uniform(-1.0, 1.0, n)
    return m, cos_g, cos_k


def amplitudes(kin, waves: WaveSet) -> np.ndarray:
    """Decay amplitudes A[i, a] (complex128) of the stand-in model."""
    m, cos_g, cos_k = kin
    photon = np.sqrt((1.0 + cos_g * cos_g) / 2.0)
    out = np.empty((m.shape[0], waves.n_waves), np.complex128)
    ang = {}
    for a, (mass, width, spin) in enumerate(zip(waves.masses, waves.widths, waves.spins)):
        if spin not in ang:
            ang[spin] = legendre(spin, cos_k) * photon
        bw = 1.0 / (mass * mass - m * m - 1j * mass * width)
        out[:, a] = bw * ang[spin]
    return out


def random_v(rng: np.random.Generator, n_waves: int, k: int | None = None) -> np.ndarray:
    """Complex production amplitudes with Re, Im i.i.d. N(0, 1)."""
    shape = (n_waves,) if k is None else (k, n_waves)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_walk(rng: np.random.Generator, v0: np.ndarray, steps: int, scale: float = 0.01):
    """V_0 = v0, V_{t+1} = V_t + scale * xi_t with Re, Im of xi i.i.d. N(0, 1)."""
    out = np.empty((steps, v0.shape[0]), np.complex128)
    v = np.array(v0, np.complex128)
    for t in range(steps):
        out[t] = v
        v = v + scale * random_v(rng, v0.shape[0])
    return out


def _density(A: np.ndarray, v: np.ndarray) -> np.ndarray:
    # sampling density for accept-reject: the coherent intensity at V_true
    s = A @ v
    return s.real * s.real + s.imag * s.imag


def draw_data(rng: np.random.Generator, waves: WaveSet, v_true: np.ndarray, n: int,
              presample: int = 2_000_000, batch: int = 500_000) -> np.ndarray:
    """Amplitudes of n data events drawn by accept-reject at v_true."""
    pre = _density(amplitudes(phase_space(rng, presample), waves), v_true)
    envelope = 1.2 * float(pre.max())
    while True:
        kept, count, ok = [], 0, True
        while count < n:
            A = amplitudes(phase_space(rng, batch), waves)
            dens = _density(A, v_true)
            if float(dens.max()) > envelope:
                envelope = 1.5 * float(dens.max())
                ok = False
                break
            sel = rng.uniform(0.0, envelope, batch) < dens
            kept.append(A[sel])
            count += int(sel.sum())
        if ok:
            return np.concatenate(kept)[:n]


def draw_mc(rng_events: np.random.Generator, rng_mask: np.random.Generator,
            waves: WaveSet, n_gen: int, n_acc: int, batch: int = 1_000_000) -> np.ndarray:
    """Amplitudes of the n_acc accepted events out of n_gen flat MC events."""
    assert 0 <= n_acc <= n_gen
    keep = np.zeros(n_gen, bool)
    keep[rng_mask.choice(n_gen, size=n_acc, replace=False)] = True
    out = np.empty((n_acc, waves.n_waves), np.complex128)
    pos = 0
    for start in range(0, n_gen, batch):
        size = min(batch, n_gen - start)
        A = amplitudes(phase_space(rng_events, size), waves)
        sel = keep[start:start + size]
        k = int(sel.sum())
        out[pos:pos + k] = A[sel]
        pos += k
    assert pos == n_acc
    return out


@dataclasses.dataclass
class Workload:
    name: str
    index: int
    n_waves: int
    n_data: int
    n_gen: int
    n_acc: int
    n_points: int
    points: str                      # "random" or "walk"
    waves: WaveSet
    walk_step: float = 0.01


def _workloads():
    c1 = wave_set(4, masses=(1.27, 1.52, 1.71, 2.0), widths=(0.18, 0.07, 0.14, 0.2),
                  spins=(2, 2, 0, 0))
    return {
        # correctness case: 10k events, 4 waves, FP64 complex table, 10 random points
        "w4_n10k": Workload("w4_n10k", 0, 4, 10_000, 100_000, 50_000, 10, "random", c1),
        # the metric workload: 1M events, 20 waves, 200 points on a random walk
        "w20_n1m": Workload("w20_n1m", 1, 20, 1_000_000, 4_000_000, 2_000_000, 200, "walk",
                            wave_set(20)),
        # differentiation case: 2M events, 32 waves, amplitude form, 20 random points
        "w32_n2m": Workload("w32_n2m", 2, 32, 2_000_000, 8_000_000, 4_000_000, 20, "random",
                            wave_set(32)),
        # batched starting points: 1M events, 20 waves, 256 random points
        "w20_n1m_k256": Workload("w20_n1m_k256", 3, 20, 1_000_000, 4_000_000, 2_000_000, 256,
                                 "random", wave_set(20)),
    }


WORKLOADS = _workloads()


@dataclasses.dataclass
class Sample:
    workload: Workload
    v_true: np.ndarray          # (W,) complex128
    data: np.ndarray            # (N, W) complex128 data amplitudes
    mc: np.ndarray              # (N_acc, W) complex128 accepted MC amplitudes
    n_gen: int
    points: np.ndarray          # (n_points, W) complex128 evaluation points


def make_sample(name: str, n_data: int | None = None, n_gen: int | None = None,
                n_acc: int | None = None, n_points: int | None = None,
                n_waves: int | None = None) -> Sample:
    """Regenerate a workload from its seed (sizes may be overridden for tests)."""
    wl = WORKLOADS[name]
    if n_waves is not None and n_waves != wl.n_waves:
        wl = dataclasses.replace(wl, n_waves=n_waves, waves=wave_set(n_waves))
    n_data = wl.n_data if n_data is None else n_data
    n_gen = wl.n_gen if n_gen is None else n_gen
    n_acc = (wl.n_acc if n_gen == wl.n_gen else n_gen // 2) if n_acc is None else n_acc
    n_points = wl.n_points if n_points is None else n_points
    ss = np.random.SeedSequence(SEED_BASE + wl.index)
    s_true, s_data, s_mc, s_mask, s_pts = [np.random.Generator(np.random.PCG64(s))
                                           for s in ss.spawn(5)]
    v_true = random_v(s_true, wl.n_waves)
    data = draw_data(s_data, wl.waves, v_true, n_data,
                     presample=min(2_000_000, max(100_000, 20 * n_data)))
    mc = draw_mc(s_mc, s_mask, wl.waves, n_gen, n_acc)
    if wl.points == "walk":
        pts = random_walk(s_pts, v_true, n_points, wl.walk_step)
    else:
        pts = random_v(s_pts, wl.n_waves, n_points)
    return Sample(wl, v_true, data, mc, n_gen, pts)


def small_sample(n_waves: int, n_data: int, n_mc: int, seed: int, n_points: int = 4) -> Sample:
    """A free-size sample for tests (flat data, no accept-reject): n_mc events
    generated, all accepted, n_points random V."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, seed])))
    ws = wave_set(n_waves)
    data = amplitudes(phase_space(rng, n_data), ws)
    mc = amplitudes(phase_space(rng, n_mc), ws)
    pts = random_v(rng, n_waves, n_points)
    wl = Workload("small", -1, n_waves, n_data, n_mc, n_mc, n_points, "random", ws)
    return Sample(wl, pts[0].copy(), data, mc, n_mc, pts)


# ---- the uneven multi-model batch ---------------------------------------------
@dataclasses.dataclass
class UnevenModel:
    n_waves: int
    n_data: int
    n_acc: int
    data: object               # (n_data, W) complex64, torch tensor on the device
    mc: object                 # (n_acc, W) complex64, torch tensor on the device
    v0: np.ndarray             # (W,) complex128 starting point


def uneven_sizes(n_models: int = 64, seed: int = 4, w_range=(8, 48), n_range=(100_000, 4_000_000)):
    """(W, N) of each model: W uniform on the integers of w_range, N
    log-uniform on n_range (seeded)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, seed])))
    ws = rng.integers(w_range[0], w_range[1] + 1, n_models)
    ns = np.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1]), n_models)).astype(np.int64)
    return [(int(w), int(n)) for w, n in zip(ws, ns)]


def amplitudes_torch(m, cos_g, cos_k, waves: WaveSet):
    """`amplitudes` for torch float64 kinematics (any device), complex64 out;
    spins 0 and 2."""
    import torch
    photon = torch.sqrt((1.0 + cos_g * cos_g) / 2.0)
    ang = {0: photon, 2: (1.5 * cos_k * cos_k - 0.5) * photon}
    out = torch.empty((m.shape[0], waves.n_waves), dtype=torch.complex64, device=m.device)
    for a, (mass, width, spin) in enumerate(zip(waves.masses, waves.widths, waves.spins)):
        den = torch.complex(mass * mass - m * m, torch.full_like(m, -mass * width))
        out[:, a] = (ang[spin] / den).to(torch.complex64)
    return out


def _amplitudes_torch(n: int, waves: WaveSet, gen, device):
    """Amplitudes of n flat events drawn with the torch generator `gen`."""
    import torch
    u = torch.rand((3, n), generator=gen, device=device, dtype=torch.float64)
    m = M_RANGE[0] + (M_RANGE[1] - M_RANGE[0]) * u[0]
    return amplitudes_torch(m, 2.0 * u[1] - 1.0, 2.0 * u[2] - 1.0, waves)


def uneven_models(sizes, mc_per_event: float = 2.0, seed: int = 4, device="cuda"):
    """Flat synthetic samples for the multi-model batch, one model at a time
    (a generator, so that only one model's MC is held at once): model k has W_k waves
    (the wave-list rule), N_k data events and mc_per_event * N_k accepted MC
    events, all drawn on the device with a seeded torch generator (the data
    are flat in phase space, not accept-reject: only their shape matters for a
    throughput measurement).  Spin factors are the Legendre P_0 = 1 and P_2."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(SEED_BASE + 1000 * seed)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, seed, 1])))
    for w, n in sizes:
        ws = wave_set(w)
        n_acc = int(mc_per_event * n)
        yield UnevenModel(w, n, n_acc, _amplitudes_torch(n, ws, gen, device),
                          _amplitudes_torch(n_acc, ws, gen, device), random_v(rng, w))
