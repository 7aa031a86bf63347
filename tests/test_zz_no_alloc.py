"""fo_initial_guess_learned_noalloc (the library's own device array as workspace) against
fo_initial_guess_learned (caller workspace): the same guess bit for bit, on two calls in a
row with a smaller mesh second, for both fallback rules; meshes beyond the array's size
are rejected before any device work."""
import ctypes

import numpy as np
import pytest
import torch

from fo_inputs import learned_mesh

from gpu_util import gpu_mesh

pytestmark = pytest.mark.gpu


def _network(seed):
    """Random parameters of the 10-128-128-128-22 network (Glorot-uniform weights, small
    biases), FP32 on the device."""
    from paper_2204_04321_amd.api import MLP
    rng = np.random.default_rng(seed)
    flat = []
    for i, j in zip(MLP.LAYERS[:-1], MLP.LAYERS[1:]):
        lim = np.sqrt(6.0 / (i + j))
        flat.append(rng.uniform(-lim, lim, i * j))
        flat.append(rng.normal(size=j) * 0.1)
    return torch.from_numpy(np.concatenate(flat).astype(np.float32)).cuda()


@pytest.mark.parametrize("fallback", [0, 1])
def test_noalloc_matches_workspace_entry_point(fallback):
    from paper_2204_04321_amd.api import MLP
    params = _network(7 + fallback)
    for seed, n_points in ((20011, 900), (20012, 400)):     # the second call has the smaller input
        M = gpu_mesh(learned_mesh(seed, n_points=n_points))
        norm = MLP.feature_stats(M.features())
        U_ref, used_ref = M.learned_guess(params, norm, fallback=fallback, smooth=3)
        U_na, used_na = M.learned_guess_noalloc(params, norm, fallback=fallback, smooth=3)
        torch.cuda.synchronize()
        print(f"\n[no-alloc] seed {seed}: {M.n_verts} columns, fallback {fallback}, network kept {used_na}")
        assert used_na == used_ref
        assert bool(torch.isfinite(U_na).all())
        assert torch.equal(U_na, U_ref)
        M.close()


def test_noalloc_rejects_meshes_beyond_its_array():
    from paper_2204_04321_amd import _lib
    from paper_2204_04321_amd.api import MLP
    M = gpu_mesh(learned_mesh(20013, n_points=16000))
    need = int(_lib.lib().fo_learned_workspace_bytes(M.handle))
    assert need > 32 << 20
    params = _network(9)
    norm = torch.zeros(20, dtype=torch.float32, device="cuda")
    U = torch.full((M.n_dofs,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.FoError) as e:
        M.learned_guess_noalloc(params, norm, out=U)
    assert e.value.status == _lib.FO_EINVAL
    torch.cuda.synchronize()
    assert bool((U == 7.0).all())          # nothing ran
    M.close()
