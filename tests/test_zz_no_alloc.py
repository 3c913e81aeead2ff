"""The allocation-free far-field entry point (sfmm_rcs_noalloc) against
sfmm_rcs on device vectors, through the C ABI: same kernel and inputs, so the
same RCS values, call after call (the second call smaller than the first, the
shared scratch keeping the first call's contents), and sizes beyond the
scratch refused before any GPU work."""

import numpy as np
import pytest

from workloads import random_complex_vector, sphere_body

pytestmark = pytest.mark.gpu

sfmm = pytest.importorskip("paper_1704_06862_amd.sfmm")
torch = pytest.importorskip("torch")


def test_noalloc_far_field_matches_sfmm_rcs():
    body = sphere_body(0.3, 4.0, 2)
    with sfmm.Context([body], precision=sfmm.PREC_FP64, finest_box=0.15, n_levels=3) as ctx:
        n = ctx.sfmm_num_unknowns()
        for n_rhs, n_dirs, seed in ((5, 181, 11), (2, 37, 12)):
            print("noalloc far field", n_rhs, n_dirs, flush=True)
            x = random_complex_vector(n, n_rhs, seed=seed)
            xd = torch.from_numpy(x).to("cuda")
            torch.cuda.synchronize()
            th = np.linspace(0.0, np.pi, n_dirs)
            tp = np.stack([th, 0.3 + 0 * th], 1)
            ref = ctx.sfmm_rcs(xd, tp)
            got = ctx.sfmm_rcs_noalloc(xd, tp)
            assert got.shape == (n_rhs, n_dirs, 2)
            assert np.all(ref > 0)
            assert np.max(np.abs(got - ref) / ref) <= 1e-13
        # n_dirs * (2 + 2 n_rhs) beyond the 262,144-double scratch
        xd = torch.zeros((200, n), dtype=torch.complex128, device="cuda")
        with pytest.raises(sfmm.SfmmError) as e:
            ctx.sfmm_rcs_noalloc(xd, np.zeros((1000, 2)))
        assert e.value.status == 1
        with pytest.raises(ValueError):
            ctx.sfmm_rcs_noalloc(np.zeros((1, n), dtype=complex), np.zeros((3, 2)))
