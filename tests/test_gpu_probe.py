"""The pipe-overlap measurement probe (pa_pipe_probe) runs every kind of work
and every pairing to completion and writes one finite value per thread."""
import ctypes as C

import pytest
import torch

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def test_pipe_probe_runs_every_pairing():
    need_gpu()
    from paper_2510_00884_amd import _lib as L
    lib = L.load()
    blocks = 4
    out = torch.full((blocks * 512,), float("nan"), dtype=torch.float64, device="cuda")
    for lo in range(6):
        for hi in range(6):
            say("pipe probe", lo, hi)
            out.fill_(float("nan"))
            L.check(lib.pa_pipe_probe(lo, hi, 8, blocks, C.c_void_p(out.data_ptr()), None), "pa_pipe_probe")
            torch.cuda.synchronize()
            assert torch.isfinite(out).all()
