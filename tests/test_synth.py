"""The seeded generator: reproducible, consistent with its recipe (CPU only)."""
import numpy as np

import oracle
from paper_1108_5673_amd import synth


def test_seed_reproduces_arrays():
    a = synth.make_sample("w4_n10k", n_data=2000, n_gen=20_000)
    b = synth.make_sample("w4_n10k", n_data=2000, n_gen=20_000)
    assert np.array_equal(a.data, b.data) and np.array_equal(a.mc, b.mc)
    assert np.array_equal(a.points, b.points) and np.array_equal(a.v_true, b.v_true)
    assert a.mc.shape == (10_000, 4) and a.data.shape == (2000, 4)


def test_workload_shapes():
    s = synth.make_sample("w4_n10k")
    assert s.data.shape == (10_000, 4) and s.mc.shape == (50_000, 4) and s.n_gen == 100_000
    assert s.points.shape == (10, 4)
    assert s.workload.waves.masses == (1.27, 1.52, 1.71, 2.0)


def test_wave_list_rule():
    ws = synth.wave_set(20)
    assert ws.masses[0] == 1.0 and ws.masses[-1] == 2.6 and ws.masses[0] == ws.masses[1]
    assert ws.spins[:4] == (0, 2, 0, 2) and set(ws.widths) == {0.15}


def test_legendre_and_breit_wigner():
    x = np.linspace(-1, 1, 11)
    assert np.allclose(synth.legendre(2, x), (3 * x * x - 1) / 2)
    assert np.allclose(synth.legendre(4, x), (35 * x ** 4 - 30 * x * x + 3) / 8)
    ws = synth.wave_set(1, masses=(1.5,), widths=(0.1,), spins=(0,))
    m = np.linspace(1.0, 2.0, 2001)
    amp = synth.amplitudes((m, np.zeros_like(m), np.zeros_like(m)), ws)[:, 0]
    # |BW|^2 peaks at the resonance mass; the phase passes 90 degrees there
    assert abs(m[np.argmax(np.abs(amp))] - 1.5) < 2e-3
    k = np.argmin(np.abs(m - 1.5))
    assert abs(np.angle(amp[k]) - np.pi / 2) < 1e-2


def test_accept_reject_follows_density():
    s = synth.make_sample("w4_n10k", n_data=5000, n_gen=20_000)
    dens_data = np.abs(s.data @ s.v_true) ** 2
    dens_mc = np.abs(s.mc @ s.v_true) ** 2
    # data are drawn from the density, flat MC is not: the mean density is larger
    assert dens_data.mean() > 1.5 * dens_mc.mean()


def test_mc_matrix_hermitian_psd():
    s = synth.make_sample("w4_n10k")
    M = oracle.get().mc_matrix(s.mc, s.n_gen)
    assert np.allclose(M, M.conj().T, rtol=0, atol=1e-14 * np.abs(M).max())
    ev = np.linalg.eigvalsh(M)
    assert ev.min() > 0
    assert np.isfinite(ev.max() / ev.min())


def test_random_walk_steps():
    rng = np.random.default_rng(0)
    v0 = synth.random_v(rng, 20)
    walk = synth.random_walk(rng, v0, 50, 0.01)
    assert np.array_equal(walk[0], v0)
    step = np.abs(np.diff(walk, axis=0))
    assert 0.003 < step.mean() < 0.03


def test_torch_amplitudes_match_numpy():
    import torch
    rng = np.random.default_rng(8)
    m, cg, ck = synth.phase_space(rng, 500)
    for w in (1, 8, 21):
        ws = synth.wave_set(w)
        a_np = synth.amplitudes((m, cg, ck), ws)
        a_t = synth.amplitudes_torch(torch.from_numpy(m), torch.from_numpy(cg),
                                     torch.from_numpy(ck), ws).numpy()
        np.testing.assert_allclose(a_t, a_np.astype(np.complex64), rtol=2e-7, atol=1e-7)


def test_uneven_sizes():
    sizes = synth.uneven_sizes()
    assert len(sizes) == 64
    ws = np.array([w for w, n in sizes])
    ns = np.array([n for w, n in sizes])
    assert ws.min() >= 8 and ws.max() <= 48 and ns.min() >= 100_000 and ns.max() <= 4_000_000
    assert sizes == synth.uneven_sizes()          # seeded
