"""abacus_nf_timestep_noalloc (the step-size criterion with the library's fixed scratch, for callers that
cannot allocate) against abacus_nf_timestep, which allocates its buffers: two calls in a row, the second on a
smaller batch, with gathered accelerations and with the force pass maxima (needs an MI355X)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle import SPLINE  # noqa: E402
from oracle import kdk as okdk  # noqa: E402
from workloads import gen  # noqa: E402


@pytest.fixture(scope="module")
def nf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_11398_amd as m
    m.library()
    return m


def _state(w, seed):
    pos = w.concat_positions()
    rng = np.random.default_rng(seed)
    vel = (1e-3 * rng.standard_normal(pos.shape)).astype(np.float32)
    return pos, vel


def _one_batch(nf, w, seed):
    boxes = [(b.n, b.box, b.K) for b in w.boxes]
    pos, vel = _state(w, seed)
    c = nf.build_cells(torch.from_numpy(pos).cuda(), boxes, 2)
    c.set_tuning(part_sources=1024)   # heavy cells split their source lists (finalized separately)
    acc = c.forces([b.eps for b in w.boxes], [b.gm for b in w.boxes], SPLINE, 1)
    v = torch.from_numpy(vel).cuda()
    want_gathered = c.timestep(v, acc, 0.25)
    got_gathered = c.timestep_noalloc(v, acc, 0.25)
    want_fused = c.timestep(v, None, 0.25)
    got_fused = c.timestep_noalloc(v, None, 0.25)
    nf.sync()
    print(f"N={w.n_total} boxes={len(w.boxes)}: noalloc {got_gathered} / {got_fused}, allocating "
          f"{want_gathered} / {want_fused}", flush=True)
    assert got_gathered == want_gathered and got_fused == want_fused
    a = acc.cpu().numpy()
    off = 0
    for b, g in zip(w.boxes, got_fused):
        ref = okdk.cell_timestep(b.pos, vel[off:off + b.n], a[off:off + b.n], b.box, b.K, 0.25)
        assert (np.isinf(ref) and np.isinf(g)) or abs(g - ref) <= 1e-9 * ref
        off += b.n
    c.free()


def test_noalloc_timestep_matches_the_allocating_entry_twice(nf):
    big = gen.workload("batched", n_boxes=4, lo=32 ** 3, hi=48 ** 3, seed=41)
    small = gen.workload("batched", n_boxes=1, lo=12 ** 3, hi=14 ** 3, seed=43)
    assert small.n_total < big.n_total
    _one_batch(nf, big, 1)
    _one_batch(nf, small, 2)


def test_noalloc_timestep_rejects_batches_beyond_its_scratch(nf):
    n_boxes = 4097
    pos = torch.full((n_boxes, 3), 0.5, dtype=torch.float32, device="cuda")
    c = nf.build_cells(pos, [(1, 1.0, 5)] * n_boxes, 2)
    v = torch.zeros((n_boxes, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(nf.NearFieldError) as e:
        c.timestep_noalloc(v, v, 0.25)
    assert e.value.code == -7   # ABACUS_NF_ELIMIT
    assert np.isinf(c.timestep(v, v, 0.25)).all()   # the allocating entry takes the same batch
    c.free()
