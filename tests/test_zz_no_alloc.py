"""The allocation-free material call (pa_energy_stress_tangent_noalloc)
against pa_energy_stress_tangent: the same kernels on the library's own
scratch array instead of a caller workspace, so the outputs must be
identical.  Two calls in a row, the second on a smaller batch (the array
keeps the first call's contents), then a batch at the stated limit, and a
batch one point beyond it, which is refused before any launch."""
import pytest
import torch

from paper_2510_00884_amd import synth
from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_workspace_call(prec):
    api = need_gpu()
    from paper_2510_00884_amd import _lib as L
    n_sv, h, Lh = 2, 32, 2
    p = synth.num_inputs(n_sv)
    gm = api.Model(synth.micnn_params(p, h, Lh, seed=1), n_sv, h, Lh, A=synth.structural_vectors(n_sv),
                   normalize=True, algorithm="adjoint")
    nmax = api.noalloc_max_points(gm)
    assert nmax == 131072
    for n in (40_003, 1_037, nmax):  # the second smaller than the first; the last at the limit
        say("noalloc", prec, n)
        F = torch.tensor(synth.sample_F(n, seed=n), device="cuda")
        ref = api.energy_stress_tangent(gm, F, prec=prec)
        nb_ref = torch.zeros(1, dtype=torch.int32, device="cuda")
        nb = torch.zeros(1, dtype=torch.int32, device="cuda")
        ref = api.energy_stress_tangent(gm, F, prec=prec, n_bad=nb_ref)
        got = api.energy_stress_tangent_noalloc(gm, F, prec=prec, n_bad=nb)
        torch.cuda.synchronize()
        for k in ("psi", "P", "A"):
            assert torch.isfinite(got[k]).all(), k
            assert torch.equal(got[k], ref[k]), (k, (got[k] - ref[k]).abs().max().item())
        assert nb.item() == nb_ref.item() == 0
    F = torch.tensor(synth.sample_F(nmax + 1, seed=5), device="cuda")
    with pytest.raises(L.PaError, match="131072"):
        api.energy_stress_tangent_noalloc(gm, F, prec=prec)
