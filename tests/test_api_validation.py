"""The Python binding refuses arrays the kernels cannot index safely -- host
tensors, the wrong dtype, non-contiguous views, the wrong length -- before any
call into the library (no GPU needed: nothing reaches a kernel)."""
import pytest
import torch

from paper_2511_21535_amd import _lib as L
from paper_2511_21535_amd import api


def _tree(n=10, kind=L.P2P_TREE_PARTICLES):
    z32 = torch.zeros(n, dtype=torch.int32)
    return api.Tree(n=n, n_leaves=1, kind=kind, key_bits=20, max_level=0, perm=z32,
                    leaf_start=torch.tensor([0, n], dtype=torch.int32), leaf_key=torch.zeros(1, dtype=torch.int64),
                    leaf_level=torch.zeros(1, dtype=torch.int8), iperm=z32)


def _nbrs():
    return api.Nbrs(count=1, nbr_start=torch.tensor([0, 1]), nbr_idx=torch.zeros(1, dtype=torch.int32),
                    red_entries=10)


def test_gravity_rejects_host_and_short_arrays():
    t, nb = _tree(), _nbrs()
    x = torch.zeros(10, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU tensor"):
        api.gravity(t, nb, 1e-3, x, x, x, x)
    with pytest.raises(ValueError, match="required"):
        api.gravity(t, nb, 1e-3, layout="gather")
    with pytest.raises(ValueError, match="GPU tensor"):
        api.restructure_gravity(t, nb, x, x, x, x)
    with pytest.raises(ValueError, match="GPU tensor"):
        api.restructure_interactions(t, nb, x, x, x, x)
    with pytest.raises(ValueError, match="GPU tensor"):
        api.gravity_adjoint(t, nb, 1e-3, x, x, x, x, x, x, x, x)


def test_remote_rejects_host_arrays():
    t, nb = _tree(), _nbrs()
    x = torch.zeros(10, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU tensor"):
        api.gravity_remote(t, _tree(7), nb, 1e-3, x, x, x, layout="redundant")
    with pytest.raises(ValueError, match="sx has 10 elements, expected 7"):
        api.restructure_remote(t, _tree(7), nb, x, x, x, x)
    s7 = torch.zeros(7, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU tensor"):
        api.restructure_remote(t, _tree(7), nb, s7, s7, s7, s7)


def test_helmholtz_rejects_wrong_dtype():
    t, nb = _tree(64, L.P2P_TREE_GRIDS), _nbrs()
    q = torch.zeros(64, dtype=torch.complex128)
    with pytest.raises(ValueError, match="complex64"):
        api.helmholtz(t, nb, q, prec="fp32")
    with pytest.raises(ValueError, match="GPU tensor"):
        api.helmholtz(t, nb, q, prec="fp64")
    with pytest.raises(ValueError, match="GPU tensor"):
        api.helmholtz_adjoint(t, nb, q)


def test_vec_checks_length_dtype_and_layout():
    ok = torch.zeros(10, dtype=torch.float64)
    assert api._vec(None, "m", 10, optional=True) is None
    with pytest.raises(ValueError, match="required"):
        api._vec(None, "m", 10)
    with pytest.raises(ValueError, match="9 elements, expected 10"):
        api._vec(ok[:9], "x", 10)
    with pytest.raises(ValueError, match="must be torch.float64"):
        api._vec(torch.zeros(10, dtype=torch.float32), "x", 10)
    with pytest.raises(ValueError, match="contiguous"):
        api._vec(torch.zeros(20, dtype=torch.float64)[::2], "x", 10)
    with pytest.raises(ValueError, match="GPU tensor"):
        api._vec(ok, "x", 10)
    with pytest.raises(ValueError, match="four arrays"):
        api._outs([ok, ok], 10, ok.device)
