"""Energy and gradient inside a HIP graph.  The library only enqueues kernels on the caller's stream
(no allocation, memset, event or synchronisation on its path), so pp_energy and pp_field can be
captured with the caller's workspace and replayed.  Every replay is checked bitwise against the
eager results (the path is deterministic), with eager work and synchronisations between the
replays, and again after the inputs are changed in place."""
import sys

import numpy as np
import pytest

from workloads import make_random

torch = pytest.importorskip("torch")
pp = pytest.importorskip("paper_2307_12041_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_energy_and_gradient_replay_in_a_graph(prec):
    wl = make_random(5003, 300.0, 200.0, 96, 80, seed=81)
    x, y, w, h = (torch.as_tensor(np.ascontiguousarray(v), device=DEV) for v in wl.arrays())
    kw = dict(W=wl.W, H=wl.H, precision=prec)
    ws = torch.empty(pp.workspace_size(wl.W, wl.H, wl.n, wl.Mu, wl.Mp, precision=prec), dtype=torch.uint8,
                     device=DEV)

    def step():
        E, a = pp.energy(x, y, w, h, Mu=wl.Mu, Mp=wl.Mp, workspace=ws, **kw)
        gx, gy = pp.field(x, y, w, h, a, workspace=ws, **kw)
        return E, a, gx, gy

    def host(ts):
        torch.cuda.synchronize()
        return [t.cpu().numpy().copy() for t in ts]

    say(f"[graph] {prec}")
    ref = host(step())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()                                # warm-up on the capturing stream's side
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs = step()
    for rep in range(3):
        g.replay()
        got = host(outs)
        assert all(np.array_equal(u, v) for u, v in zip(got, ref)), (prec, rep)
        host(step())                          # eager work between the replays
    # new positions, written into the captured input buffers
    x.add_(0.75)
    y.sub_(0.5)
    ref2 = host(step())
    assert not np.array_equal(ref2[1], ref[1])
    for rep in range(2):
        g.replay()
        got = host(outs)
        assert all(np.array_equal(u, v) for u, v in zip(got, ref2)), (prec, "moved", rep)
