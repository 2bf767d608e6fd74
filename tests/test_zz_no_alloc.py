"""sw_step_noalloc (the time step without a context, for callers that cannot
allocate device memory) against sw_step through a context, to the parity bar:
bitwise, since both run the same kernels in the same launch shape.  Two calls
in a row on one device share the static scratch; the second is on a smaller
grid, so whatever the first left there must not leak into it.
"""
import numpy as np
import pytest
import torch

from paper_1107_2157_amd import ics, sw
from swtest import G, announce

pytestmark = pytest.mark.gpu


def _pair(nx, ny, dtype, scheme, bc, seed):
    h, hu, hv = ics.bumps_state(nx, ny, seed=seed, periodic=bc == sw.PERIODIC, count=3)
    out = []
    for _ in range(2):
        s = sw.Solver(nx, ny, g=G, dtype=dtype, bc_x=bc, bc_y=bc, scheme=scheme)
        s.set_state(h, hu, hv)
        out.append(s)
    return out


CASES = [  # (nx, ny, dtype, scheme, bc, steps): each second case is smaller than the first
    ((300, 200, "f32", sw.SCHEME_PAPER, sw.REFLECT, 23), (70, 33, "f32", sw.SCHEME_PAPER, sw.REFLECT, 9)),
    ((257, 130, "f64", sw.SCHEME_TRANSVERSE, sw.PERIODIC, 17), (64, 5, "f64", sw.SCHEME_PAPER, sw.PERIODIC, 12)),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_matches_step(first, second):
    for k, (nx, ny, dtype, scheme, bc, steps) in enumerate((first, second)):
        announce(f"step_noalloc call {k}: {dtype} {nx}x{ny} scheme={scheme} bc={bc} steps={steps}")
        ref, na = _pair(nx, ny, dtype, scheme, bc, seed=40 + k)
        ref.step(steps)
        t_ref, dt_ref, n_ref = ref.sync_status()
        status = torch.full((4,), -1.0, dtype=torch.float64, device="cuda")
        na.step_noalloc(steps, status)
        torch.cuda.synchronize()
        assert na.state.cur == ref.state.cur == steps % 2
        a, b = ref.get_state(halo=True), na.get_state(halo=True)
        for f in range(3):
            assert torch.equal(a[f], b[f]), f"field {f} differs (call {k})"
        st = status.cpu().numpy()
        assert st[0] == t_ref and st[1] == dt_ref and st[2] == n_ref == steps and st[3] == 0.0, (st, t_ref, n_ref)


def test_noalloc_rejects_bad_arguments():
    s = sw.Solver(32, 32, g=G)
    with pytest.raises(sw.SwError):
        s.step_noalloc(-1)
    saved = s.state.plane[1][0]
    s.state.plane[1][0] = s.state.plane[0][0]     # buffers sharing a plane
    with pytest.raises(sw.SwError):
        s.step_noalloc(2)
    s.state.plane[1][0] = saved
    s.step_noalloc(0)
    torch.cuda.synchronize()
    assert np.isfinite(s.get_state()[0].numpy()).all()
