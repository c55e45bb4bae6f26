"""Restructure + evaluation recorded into a HIP graph and replayed: every
replay, with the program's own eager work and synchronisations between
replays, gives the eager result bit for bit (same kernels, same inputs); calls
that cannot be captured are refused with P2P_EUNSUPPORTED.  The eager results
themselves are checked against the oracle by the parity tests."""
import numpy as np
import pytest
import torch

from paper_2511_21535_amd import _lib as L
from paper_2511_21535_amd import api
from paper_2511_21535_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def _check_replays(step, outs, reps=3):
    step()
    torch.cuda.synchronize()
    want = [o.clone() for o in outs]
    g = api.Graph(step)
    torch.cuda.synchronize()
    for r in range(reps):
        for o in outs:
            o.fill_(float("nan"))          # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, w in zip(outs, want):
            assert torch.equal(o, w), f"replay {r}"
    return g


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_gravity_restructure_and_eval_replay(prec):
    x, y, z, m = W.plummer_mixture(20000, 71)
    print(f"case graph gravity prec={prec}", flush=True)
    g = [_t(v) for v in (x, y, z, m)]
    tree = api.Tree.build_particles(*g[:3], depth=20, leaf_cap=64)
    nbrs = tree.neighbors()
    assert nbrs.red_entries > 0
    red = api.restructure_gravity(tree, nbrs, *g, prec=prec)
    outs = [torch.empty(len(x), dtype=torch.float64, device=DEV) for _ in range(4)]
    outs_g = [torch.empty(len(x), dtype=torch.float64, device=DEV) for _ in range(4)]

    def step():
        api.restructure_gravity(tree, nbrs, *g, prec=prec, out=red)
        api.gravity(tree, nbrs, 1e-3, layout="redundant", prec=prec, red=red, out=outs)
        api.gravity(tree, nbrs, 1e-3, *g, layout="gather", prec=prec, out=outs_g)

    _check_replays(step, outs + outs_g)
    # new input values written into the captured arrays reach the replay
    gr = api.Graph(step)
    g[3].mul_(2.0)
    api.gravity(tree, nbrs, 1e-3, *g, layout="gather", prec=prec, out=outs)
    torch.cuda.synchronize()
    want = [o.clone() for o in outs]
    gr.replay()
    torch.cuda.synchronize()
    for o, w in zip(outs_g, want):
        assert torch.equal(o, w)


def test_helmholtz_single_rhs_replay():
    n = 32
    print("case graph helmholtz 32^3", flush=True)
    gq = _t(W.grid_rhs(n ** 3, 1, seed=72)[:, 0])
    grids = [api.Grid(n, *W.grid_geometry(n))]
    tree = api.Tree.build_grids(grids, device=torch.device(DEV))
    nbrs = tree.neighbors()
    red = api.restructure(tree, nbrs, [gq], prec="fp32", nrhs=1)
    out = torch.empty_like(gq)
    out_g = torch.empty_like(gq)

    def step():
        api.restructure(tree, nbrs, [gq], prec="fp32", nrhs=1, out=red)
        api.helmholtz(tree, nbrs, None, layout="redundant", prec="fp32", red=red, out=out)
        api.helmholtz(tree, nbrs, gq, layout="gather", prec="fp32", out=out_g)

    _check_replays(step, [torch.view_as_real(out), torch.view_as_real(out_g)])


def test_capture_refuses_host_steps():
    x, y, z, m = W.plummer_mixture(3000, 73)
    g = [_t(v) for v in (x, y, z, m)]
    tree = api.Tree.build_particles(*g[:3], depth=20, leaf_cap=64)
    print("case graph refusal", flush=True)
    for fn in (lambda: tree.neighbors(),
               lambda: api.Tree.build_particles(*g[:3], depth=20, leaf_cap=64)):
        graph = torch.cuda.CUDAGraph()
        with pytest.raises(L.P2PError) as err:
            with torch.cuda.graph(graph):
                fn()
        assert err.value.status == L.P2P_EUNSUPPORTED
    torch.cuda.synchronize()
    # the library still works eagerly afterwards
    assert tree.neighbors().count > 0
