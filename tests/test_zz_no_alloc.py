"""The allocation-free entry point (tpcca_run_batch_noalloc) against
tpcca_run_batch on the same device-resident units: two calls in a row, the
second with fewer clusters, every output byte for byte; the second call also
against the FP32 oracle, and a batch beyond the fixed work array rejected."""
import types

import numpy as np
import pytest

import oracle
import tpcgen
from tests import _parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def event():
    return tpcgen.central_event(seed=0, keep_truth=False)


def _noalloc(tpcca, torch, row_x, dcl, drow, units):
    n_cl = int(units[:, 1].sum())
    n_trk = int(sum(int(n) // 3 + 1 for n in units[:, 1]))
    # outputs filled with a pattern, so that stale or unwritten entries show
    tracks = torch.full((n_trk * tpcca.TRACK_DTYPE.itemsize,), 0xAB, dtype=torch.uint8, device="cuda")
    hits = torch.full((n_cl,), -7, dtype=torch.int32, device="cuda")
    asg = torch.full((n_cl,), -7, dtype=torch.int32, device="cuda")
    ures = torch.full((units.shape[0] * tpcca.UNIT_RESULT_DTYPE.itemsize,), 0xCD, dtype=torch.uint8,
                      device="cuda")
    torch.cuda.synchronize()
    nt, nh = tpcca.run_batch_noalloc(row_x, dcl, drow, units, tracks, hits, asg, ures)
    tr = tracks.cpu().numpy().view(tpcca.TRACK_DTYPE)[:nt]
    return (ures.cpu().numpy().view(tpcca.UNIT_RESULT_DTYPE), tr, hits.cpu().numpy()[:nh],
            asg.cpu().numpy())


def test_noalloc_equals_run_batch_on_two_calls(torch_cuda, event, row_x):
    from paper_1709_00618_amd import tpcca
    torch = torch_cuda
    b = event
    dcl = torch.from_numpy(np.ascontiguousarray(b.cl)).cuda()
    drow = torch.from_numpy(np.ascontiguousarray(b.row)).cuda()
    torch.cuda.synchronize()
    # four sectors (about 1.2e5 clusters), then one sector
    for call, sel in enumerate(([0, 1, 2, 3], [5])):
        units = np.ascontiguousarray(b.units[sel])
        print(f"no-alloc call {call}: units {sel}, {int(units[:, 1].sum())} clusters", flush=True)
        got = _noalloc(tpcca, torch, row_x, dcl, drow, units)
        with tpcca.Context(row_x) as ctx:
            ctx.run_batch(dcl, drow, units, device=True)
            want = ctx.get_batch_results()
        names = ("unit results", "tracks", "hits", "assignment")
        for name, g, w in zip(names, got, want):
            assert g.shape == w.shape, (name, g.shape, w.shape)
            assert g.tobytes() == w.tobytes(), f"call {call}: {name} differ"
        assert got[1].shape[0] > 100
        if call == 1:
            sub = types.SimpleNamespace(units=units)
            cl, row, _, _, _ = b.unit(5)
            refs = [oracle.run_sector(cl, row, row_x, precision=32)]
            _parity.compare_batch(got[0], got[1], got[2], got[3], sub, refs)


def test_noalloc_rejects_more_than_its_work_array(torch_cuda, event, row_x):
    """All 36 sectors of a central event need about 0.4 GB: refused on the
    host before any work is queued, with the limit in the message."""
    from paper_1709_00618_amd import tpcca
    torch = torch_cuda
    b = event
    dcl = torch.from_numpy(np.ascontiguousarray(b.cl)).cuda()
    drow = torch.from_numpy(np.ascontiguousarray(b.row)).cuda()
    n_cl = b.n_clusters
    n_trk = int(sum(int(n) // 3 + 1 for n in b.units[:, 1]))
    tracks = torch.empty(n_trk * tpcca.TRACK_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    hits = torch.empty(n_cl, dtype=torch.int32, device="cuda")
    asg = torch.empty(n_cl, dtype=torch.int32, device="cuda")
    ures = torch.empty(b.units.shape[0] * tpcca.UNIT_RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(tpcca.TpccaError) as e:
        tpcca.run_batch_noalloc(row_x, dcl, drow, b.units, tracks, hits, asg, ures)
    assert e.value.status == tpcca.ENOMEM and "MiB" in str(e.value)
    # a too small output is refused the same way
    with pytest.raises(tpcca.TpccaError) as e:
        tpcca.run_batch_noalloc(row_x, dcl, drow, b.units[:1], tracks[:108], hits, asg, ures)
    assert e.value.status == tpcca.ECAPACITY
