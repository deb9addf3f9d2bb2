"""The 16-bit amplitude forms on the matrix cores (needs an MI355X).

Inputs both sides see: the amplitudes rounded to bfloat16 or float16 on the
host (torch's and numpy's round-to-nearest-even conversions from complex64;
float16 results below the smallest normal stored as zero), which the library
must store bit for bit; the oracle then evaluates Eq. 3 in
FP64 on those rounded amplitudes.

Tolerances, from the arithmetic of the kernel (u = 2^-24, the FP32 unit
roundoff).  S_i = sum_a A_ia V_a is accumulated in FP32 over n_t = 2W x 2 (the
parts of V) exact 16-bit products, so |dS_i| <= e_i = n_t u sum_a |A_ia||V_a|;
an event whose S_i nearly cancels has a large relative error, which enters
ln I_i as 2 e_i / |S_i| and the adjoint weight c_i = 1 / conj(S_i) as
e_i / |S_i|^2.  V is carried in two 16-bit parts, which leave out at most
v_i = 2^-15 sum_a |A_ia||V_a| of S_i (bf16; 2^-21 for fp16), the same for
every evaluation: its first-order share of the NLL is added back by the
assembly, so the NLL keeps the second-order part, 2 (v_i / |S_i|)^2 per event
(4 v_i / |S_i| where v_i / |S_i| >= 1/2), and the gradient takes v_i beside
e_i.  The kernel works on V / s (s the power
of two nearest ||V||), takes log2 of products of four I' = I / s^2 (three FP32
roundings, at most 3 u / ln 2 in log2 per product) with the FP32 hardware
logarithm (error below 2^-21 absolute plus 2 u |log2|, and |log2 of a
product| <= the sum of the four |log2 I'|), or of each I' where a product
leaves the normal range, and adds a lane's eight in FP32 before an FP64 lane
sum (8 u |log2 I'| more); per event at most 2^-21 + 10 u |log2 I'|.  The weights c are
split into two 16-bit parts (relative error 2^-16 for bfloat16, 2^-22 for
float16), and an FP32 adjoint accumulator adds at most kFoldTiles + 1 = 33
tiles (per tile four 32x32x16 MFMA steps of 16 products each, or for the
last 16 gradient rows two 16x16x32 steps of 32; at most four accumulator
roundings either way) before it is folded into FP64, plus one rounding each
for the fold and the FP32 record: gamma = (4 x 33 + 6) u per accumulated
term.  Per point, with
a_b = sum_i |A_ib| / |S_i| (the sum of |terms| of g_b):
  |dNLL|   <= 4 sum_i 2 e_i / |S_i| + sum_i 2 (v_i / |S_i|)^2
              + ln 2 sum_i (2^-21 + 10 u |log2 I'_i|) + 1e-9 |NLL|,
  ||dG||_2 <= 8 sqrt(2) || sum_i |A_i| (e_i + v_i) / |S_i|^2 ||_2
              + 4 (gamma + split) ||a||_2 + 1e-12 ||G||_2.
"""
import numpy as np
import pytest

import oracle
import paper_1108_5673_amd as pwa
from paper_1108_5673_amd import synth

pytestmark = pytest.mark.gpu

FORMS = ["amplitude_bf16", "amplitude_fp16"]
V_PARTS = {"amplitude_bf16": 2, "amplitude_fp16": 2}
V_REST = {"amplitude_bf16": 2.0 ** -15, "amplitude_fp16": 2.0 ** -21}
U32 = 2.0 ** -24
SPLIT = {"amplitude_bf16": 2.0 ** -16, "amplitude_fp16": 2.0 ** -22}
FOLD_TILES = 32


def _round16(a: np.ndarray, form: str) -> np.ndarray:
    """complex64 -> the stored 16-bit parts, widened back to complex128."""
    a = np.ascontiguousarray(a, np.complex64)
    re, im = a.real.astype(np.float32), a.imag.astype(np.float32)
    if form == "amplitude_fp16":
        # round to nearest even, then subnormal results stored as zero
        r, i = re.astype(np.float16).astype(np.float64), im.astype(np.float16).astype(np.float64)
        r[np.abs(r) < 2.0 ** -14] = 0.0
        i[np.abs(i) < 2.0 ** -14] = 0.0
    else:
        import torch
        r = torch.from_numpy(re).to(torch.bfloat16).to(torch.float64).numpy()
        i = torch.from_numpy(im).to(torch.bfloat16).to(torch.float64).numpy()
    return r + 1j * i


def _rel(g, ref):
    return float(np.linalg.norm(np.asarray(g) - ref) / np.linalg.norm(ref))


def _scale(V):
    """The power of two nearest ||V||_2 that the kernel divides V by."""
    nn = float(np.sum(np.abs(V) ** 2))
    return 1.0 if not nn > 0 else 2.0 ** np.rint(0.5 * np.log2(nn))


def _bounds(A, V, form, nll_ref, g_ref):
    """(|dNLL| bound, ||dG|| bound) of the derivation above."""
    n, w = A.shape
    S = A @ V
    aS = np.abs(S)
    e = 2 * w * V_PARTS[form] * U32 * (np.abs(A) @ np.abs(V))
    v = V_REST[form] * (np.abs(A) @ np.abs(V))
    r = v / aS
    second = np.where(r < 0.5, 2 * r ** 2, 4 * r)
    log2i = np.log2(aS ** 2 / _scale(V) ** 2)
    b_nll = (4 * np.sum(2 * e / aS) + np.sum(second)
             + np.log(2) * np.sum(2.0 ** -21 + 10 * U32 * np.abs(log2i)) + 1e-9 * abs(nll_ref))
    du = np.abs(A).T @ ((e + v) / aS ** 2)
    a = np.abs(A).T @ (1.0 / aS)
    gamma = (4 * (FOLD_TILES + 1) + 6) * U32
    b_g = (8 * np.sqrt(2) * np.linalg.norm(du) + 4 * (gamma + SPLIT[form]) * np.linalg.norm(a)
           + 1e-12 * np.linalg.norm(g_ref))
    return b_nll, b_g


def _check(form, w, n, n_mc, seed, k):
    o = oracle.get()
    s = synth.small_sample(w, n, n_mc, seed, n_points=k)
    d32 = s.data.astype(np.complex64)
    mc32 = s.mc.astype(np.complex64)
    model = pwa.Model(d32, mc32, n_mc, form=form)
    A = _round16(d32, form)
    assert np.array_equal(model.table().astype(np.complex128), A)
    M = o.mc_matrix(mc32.astype(np.complex128), n_mc)
    [(nll_b, g_b)] = pwa.nll_batched([model], [s.points])
    for j, V in enumerate(s.points):
        rn, rg, nbad = o.nll_amp(A, M, V)
        assert nbad == 0
        b_nll, b_g = _bounds(A, V, form, rn, rg)
        assert abs(nll_b[j] - rn) <= b_nll, (form, w, n, k, j, nll_b[j], rn, b_nll)
        dg = float(np.linalg.norm(g_b[j] - rg))
        assert dg <= b_g, (form, w, n, k, j, dg, b_g, _rel(g_b[j], rg))
    # a single call agrees with the oracle within the same bounds
    nll1, g1 = model.nll_grad(s.points[0])
    rn, rg, _ = o.nll_amp(A, M, s.points[0])
    b_nll, b_g = _bounds(A, s.points[0], form, rn, rg)
    assert abs(nll1 - rn) <= b_nll
    assert np.linalg.norm(g1 - rg) <= b_g
    model.close()


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("w,n,k", [(1, 1, 1), (2, 33, 3), (4, 1000, 16), (7, 4099, 17),
                                   (20, 5000, 37), (24, 777, 64), (33, 300, 5), (64, 2000, 20),
                                   # full 16-event tiles only; one and several full
                                   # column blocks of 32 vectors, and one more
                                   (20, 4096, 32), (3, 16, 33), (5, 17, 96), (16, 2048, 65)])
def test_matrix_parity(form, w, n, k):
    _check(form, w, n, 3 * n + 11, seed=1000 * w + n + k, k=k)


@pytest.mark.parametrize("form", FORMS)
def test_matrix_long_chunks(form):
    """1024 vectors over 10^5 events at 20 waves: 32 column blocks leave 64
    event chunks of about 98 tiles each, so the adjoint accumulators are folded
    into FP64 several times per chunk (every 32 tiles) before a record is
    written; three vectors against the oracle within the derived bounds."""
    o = oracle.get()
    s = synth.small_sample(20, 100_000, 4_000, seed=1024, n_points=1024)
    d32, mc32 = s.data.astype(np.complex64), s.mc.astype(np.complex64)
    model = pwa.Model(d32, mc32, 9_000, form=form)
    A = _round16(d32, form)
    M = o.mc_matrix(mc32.astype(np.complex128), 9_000)
    [(nll_b, g_b)] = pwa.nll_batched([model], [s.points])
    for j in (0, 511, 1023):
        rn, rg, nbad = o.nll_amp(A, M, s.points[j])
        assert nbad == 0
        b_nll, b_g = _bounds(A, s.points[j], form, rn, rg)
        assert abs(nll_b[j] - rn) <= b_nll, (form, j, nll_b[j], rn, b_nll)
        assert np.linalg.norm(g_b[j] - rg) <= b_g, (form, j, _rel(g_b[j], rg))
    model.close()


@pytest.mark.parametrize("form", FORMS)
def test_matrix_degenerate_event(form):
    s = synth.small_sample(6, 500, 800, seed=77, n_points=3)
    d = s.data.astype(np.complex64)
    d[123] = 0.0                          # I = 0 for every V
    model = pwa.Model(d, s.mc.astype(np.complex64), 800, form=form)
    with pytest.warns(UserWarning):
        [(nll, g)] = pwa.nll_batched([model], [s.points])
    assert np.all(np.isinf(nll)) and np.all(np.isnan(g))
    model.close()


@pytest.mark.parametrize("form", FORMS)
def test_matrix_degenerate_event_full_blocks(form):
    # 64 vectors (two full column blocks) over full 16-event tiles: the
    # degenerate event lies in the tiles taken by the software pipeline
    s = synth.small_sample(6, 4000, 5000, seed=78, n_points=64)
    d = s.data.astype(np.complex64)
    d[1234] = 0.0
    model = pwa.Model(d, s.mc.astype(np.complex64), 5000, form=form)
    with pytest.warns(UserWarning):
        [(nll, g)] = pwa.nll_batched([model], [s.points])
    assert np.all(np.isinf(nll)) and np.all(np.isnan(g))
    model.close()


def test_matrix_extreme_intensities():
    # bf16 keeps the FP32 exponent range: events scaled by 1e-15 and 1e+15 give
    # intensities near 1e-30 and 1e+30, whose products leave the FP32 range; the
    # result must still match the oracle within the arithmetic bounds
    form = "amplitude_bf16"
    o = oracle.get()
    s = synth.small_sample(10, 4096, 6000, seed=79, n_points=64)
    d32 = s.data.astype(np.complex64)
    d32[::97] *= np.float32(1e-15)
    d32[5::89] *= np.float32(1e15)
    mc32 = s.mc.astype(np.complex64)
    model = pwa.Model(d32, mc32, 6000, form=form)
    A = _round16(d32, form)
    M = o.mc_matrix(mc32.astype(np.complex128), 6000)
    [(nll_b, g_b)] = pwa.nll_batched([model], [s.points])
    for j in (0, 17, 40, 63):
        rn, rg, nbad = o.nll_amp(A, M, s.points[j])
        assert nbad == 0
        b_nll, b_g = _bounds(A, s.points[j], form, rn, rg)
        assert abs(nll_b[j] - rn) <= b_nll, (j, nll_b[j], rn, b_nll)
        assert np.linalg.norm(g_b[j] - rg) <= b_g, (j, _rel(g_b[j], rg))
    model.close()


@pytest.mark.parametrize("form", FORMS)
def test_matrix_repeatable(form):
    s = synth.small_sample(12, 3000, 4000, seed=5, n_points=40)
    model = pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), 4000, form=form)
    a = pwa.nll_batched([model], [s.points])[0]
    b = pwa.nll_batched([model], [s.points])[0]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    model.close()


@pytest.mark.parametrize("form", FORMS)
def test_matrix_buffer_reuse_and_growth(form):
    """One model, calls of different K in turn: a larger call grows the
    per-call buffers (the vector staging the kernels read, the per-vector
    values, the records), and a repeat of the first call afterwards gives the
    same results bit for bit (the same K, so the same event chunks); the
    larger call is held to the derived bounds against the oracle."""
    o = oracle.get()
    w, n, n_mc = 12, 3000, 4000
    s = synth.small_sample(w, n, n_mc, seed=6, n_points=300)
    d32, mc32 = s.data.astype(np.complex64), s.mc.astype(np.complex64)
    model = pwa.Model(d32, mc32, n_mc, form=form)
    P, Q = s.points[:40], s.points
    a1 = pwa.nll_batched([model], [P])[0]
    b = pwa.nll_batched([model], [Q])[0]
    a2 = pwa.nll_batched([model], [P])[0]
    assert np.array_equal(a1[0], a2[0]) and np.array_equal(a1[1], a2[1])
    A = _round16(d32, form)
    M = o.mc_matrix(mc32.astype(np.complex128), n_mc)
    for j in (0, 150, 299):
        rn, rg, nbad = o.nll_amp(A, M, Q[j])
        assert nbad == 0
        b_nll, b_g = _bounds(A, Q[j], form, rn, rg)
        assert abs(b[0][j] - rn) <= b_nll, (j, b[0][j], rn, b_nll)
        assert np.linalg.norm(b[1][j] - rg) <= b_g, (j, _rel(b[1][j], rg))
    model.close()
