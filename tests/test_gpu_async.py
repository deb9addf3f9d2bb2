"""Asynchronous entry points (needs an MI355X).

pwa_nll_async / pwa_nll_grad_async read V from device memory and write
[nll, n_bad, grad] to device memory without synchronising (include/pwa.h).
They run the same kernels as the synchronous calls, so the results must agree
bit for bit; captured in a HIP graph (torch.cuda.CUDAGraph), every replay must
read the V then in the buffer, with eager work and synchronisations between
the replays, and again agree with the synchronous calls.
"""
import numpy as np
import pytest
import torch

import paper_1108_5673_amd as pwa
from paper_1108_5673_amd import synth
from paper_1108_5673_amd._native import PWAError

pytestmark = pytest.mark.gpu

FORMS = ["table", "amplitude", "table_fp64", "table_fp64_plain"]


def _model(form, w=7, n=3001, seed=90):
    s = synth.small_sample(w, n, 2 * n, seed=seed, n_points=4)
    sp = form in ("table", "amplitude")
    d = s.data.astype(np.complex64) if sp else s.data
    mc = s.mc.astype(np.complex64) if sp else s.mc
    return pwa.Model(d, mc, 2 * n, form=form), s


@pytest.mark.parametrize("form", FORMS)
def test_async_equals_sync(form):
    model, s = _model(form)
    W = model.n_waves
    for V in s.points:
        nll, g = model.nll_grad(V)
        v_dev = torch.tensor(np.ascontiguousarray(V).view(np.float64), device="cuda")
        out = torch.full((2 + 2 * W,), -1.0, dtype=torch.float64, device="cuda")
        model.nll_grad_async(v_dev, out)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        assert o[0] == nll and o[1] == 0.0 and np.array_equal(o[2:], g)
        out2 = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
        model.nll_grad_async(v_dev, out2, grad=False)
        torch.cuda.synchronize()
        assert out2[0].item() == model.nll(V)
    model.close()


@pytest.mark.parametrize("form", ["table", "amplitude"])
def test_graph_replays(form):
    model, s = _model(form, w=20, n=20_000, seed=91)
    W = model.n_waves
    K = 3
    rng = np.random.default_rng(5)
    vbuf = torch.zeros((K, 2 * W), dtype=torch.float64, device="cuda")
    obuf = torch.zeros((K, 2 + 2 * W), dtype=torch.float64, device="cuda")
    vbuf.copy_(torch.tensor(rng.standard_normal((K, 2 * W))))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        model.nll_grad_async(vbuf[0], obuf[0])          # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for k in range(K):
            model.nll_grad_async(vbuf[k], obuf[k])
    for rep in range(4):
        V = rng.standard_normal((K, 2 * W))
        vbuf.copy_(torch.tensor(V))                      # eager work between replays
        obuf.fill_(-7.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        o = obuf.cpu().numpy()
        for k in range(K):
            nll, g = model.nll_grad(V[k])
            assert o[k, 0] == nll and o[k, 1] == 0.0 and np.array_equal(o[k, 2:], g), (rep, k)
    del graph
    model.close()


def test_async_degenerate_and_rejections():
    s = synth.small_sample(5, 400, 500, seed=92, n_points=1)
    d = s.data.astype(np.complex64)
    d[17] = 0.0
    model = pwa.Model(d, s.mc.astype(np.complex64), 500, form="amplitude")
    v_dev = torch.tensor(np.ascontiguousarray(s.points[0]).view(np.float64), device="cuda")
    out = torch.zeros(12, dtype=torch.float64, device="cuda")
    model.nll_grad_async(v_dev, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert o[0] == np.inf and o[1] == 1.0 and np.all(np.isnan(o[2:]))
    model.close()
    m16 = pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), 500,
                    form="amplitude_bf16")
    with pytest.raises(PWAError):
        m16.nll_grad_async(v_dev, out)
    with pytest.raises(ValueError):
        m16.nll_grad_async(v_dev.cpu(), out)
    m16.close()
