"""The autotuner on the GPU (through the C ABI): its trials leave the
simulation where it was (state with halo, time and step counters, bitwise),
the choice is appended to the cache file under a key of arch, CUs, dtype,
scheme and size and read back by the next context of that size, and
malformed or unusable cache lines are skipped.  The batch tuner likewise."""
import torch

from paper_1107_2157_amd import ics, sw
from swtest import announce

import pytest

pytestmark = pytest.mark.gpu


def device_key_prefix():
    p = torch.cuda.get_device_properties(0)
    return f"{p.gcnArchName.split(':')[0]}:{p.multi_processor_count}"


def snapshot(s):
    return [x.numpy().tobytes() for x in s.get_state(halo=True)], s.sync_status()


def test_autotune_restores_state_and_caches(tmp_path):
    nx, ny = 300, 200
    announce("autotune single grid 300x200 f32")
    st = ics.random_state(nx, ny, seed=21)
    kw = dict(dtype="f32", bc_x=sw.PERIODIC, bc_y=sw.REFLECT)
    s = sw.Solver(nx, ny, **kw)
    s.set_state(*st)
    s.step(5)
    before = snapshot(s)
    key = f"{device_key_prefix()}:f32:0:{nx}x{ny}"
    cache = tmp_path / "tune.txt"
    cache.write_text(f"not a cache line\n{key} 2 8 3 0 1 0 1.0\n")   # vec 3 does not exist: trials run
    best = s.autotune(steps_per_trial=2, cache_path=str(cache))
    assert snapshot(s) == before
    assert s.get_tuning() == best
    lines = cache.read_text().splitlines()
    assert len(lines) == 3 and lines[-1].split()[0] == key
    assert [int(v) for v in lines[-1].split()[1:7]] == [best[k] for k in
                                                        ("variant", "rows", "vec", "occupancy", "prefetch", "order")]
    # tuning did not perturb the run: it continues exactly as one that never tuned
    ref = sw.Solver(nx, ny, **kw)
    ref.set_state(*st)
    ref.step(5)                      # default shape, as s before tuning
    ref.set_tuning(**best)
    s.step(7)
    ref.step(7)
    assert snapshot(s) == snapshot(ref)
    # the next context of this size reads the entry instead of timing again
    s2 = sw.Solver(nx, ny, **kw)
    s2.set_state(*st)
    assert s2.autotune(steps_per_trial=2, cache_path=str(cache)) == best
    assert cache.read_text().splitlines() == lines


def test_batch_autotune_restores_state_and_caches(tmp_path):
    sides = [64, 192, 130, 320]
    announce("autotune batch of 4 uneven grids f32")
    b = sw.Batch(sides, dtype="f32")
    for k, n in enumerate(sides):
        b.set_state(k, *ics.bumps_state(n, n, seed=300 + k, periodic=False, device="cuda"))
    b.step(4)
    before = ([[x.numpy().tobytes() for x in b.get_state(k)] for k in range(len(sides))], b.sync_status())
    cache = tmp_path / "batch_tune.txt"
    best = b.autotune(steps_per_trial=2, cache_path=str(cache))
    after = ([[x.numpy().tobytes() for x in b.get_state(k)] for k in range(len(sides))], b.sync_status())
    assert after == before
    assert b.get_tuning() == best
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and ":batch4:" in lines[0]
    assert b.autotune(steps_per_trial=2, cache_path=str(cache)) == best
    assert cache.read_text().splitlines() == lines
