"""gres_compute_noalloc (the entry point for callers that cannot allocate) against gres_compute
with a caller workspace: bit-identical g_exit and gres on two calls in a row, the second one
smaller, so the second runs over what the first left in the library's fixed workspace."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2412_02274_amd import _lib, api, datagen

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _skyline(x):
    xs = api.ingest(torch.from_numpy(x).to(DEV))
    plan = api.build(xs, "none", 1)
    plan.local_skylines()
    idx = plan.merge()
    plan.close()
    return xs, idx


def _bits(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("mapping", ["auto", "tiles", "levels"])
def test_noalloc_equals_gres_compute_twice(mapping):
    print(f"noalloc mapping={mapping}", flush=True)
    # first call: 200,000 x 6 anticorrelated (a skyline of thousands of tuples), g_max 25
    x1 = datagen.ant(200_000, 6, 11)
    xs1, idx1 = _skyline(x1)
    ge_ref, gr_ref = api.gres(xs1, idx1, 25, mapping)
    ge_na, gr_na = api.gres_noalloc(xs1, idx1, 25, mapping)
    torch.cuda.synchronize()
    assert idx1.numel() > 2000
    assert torch.equal(ge_na, ge_ref)
    assert (_bits(gr_na) == _bits(gr_ref)).all()
    # second call, smaller: 5,003 x 4 uniform (ragged tile tail), g_max 130, every row as a
    # candidate (a superset of the skyline gives the same answer)
    x2 = datagen.uni(5003, 4, 12)
    xs2 = api.ingest(torch.from_numpy(x2).to(DEV))
    idx2 = torch.arange(5003, dtype=torch.int64, device=DEV)
    ge_ref2, gr_ref2 = api.gres(xs2, idx2, 130, mapping)
    ge_na2, gr_na2 = api.gres_noalloc(xs2, idx2, 130, mapping)
    torch.cuda.synchronize()
    assert torch.equal(ge_na2, ge_ref2)
    assert (_bits(gr_na2) == _bits(gr_ref2)).all()
    want_ge, _ = oracle.gres(x2, np.arange(5003), 130)
    assert (ge_na2.cpu().numpy() == want_ge).all()


def test_noalloc_on_a_side_stream_and_empty():
    print("noalloc side stream", flush=True)
    x = datagen.ties(20_000, 5, 3)
    xs, idx = _skyline(x)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ge, gr = api.gres_noalloc(xs, idx, 25, stream=side)
    side.synchronize()
    ge_ref, _ = api.gres(xs, idx, 25)
    torch.cuda.synchronize()
    assert torch.equal(ge, ge_ref)
    want, _ = oracle.gres(x, idx.cpu().numpy(), 25)
    assert (ge.cpu().numpy() == want).all()
    # s = 0: nothing to do, SKY_OK
    empty = torch.empty(0, dtype=torch.int64, device=DEV)
    ge0, gr0 = api.gres_noalloc(xs, empty, 25)
    assert ge0.numel() == 0 and gr0.numel() == 0


def test_noalloc_refuses_beyond_its_workspace():
    lib = _lib.load()
    s = 1 << 21  # far beyond 64 MiB of workspace at d = 8
    assert lib.gres_workspace_bytes(s, 8, 25) > _lib.SKY_NOALLOC_SCRATCH_BYTES
    xs = torch.zeros((8, 16), dtype=torch.float32, device=DEV)
    idx = torch.zeros(s, dtype=torch.int64, device=DEV)
    with pytest.raises(_lib.SkyError) as e:
        api.gres_noalloc(xs, idx, 25)
    assert e.value.code == _lib.SKY_ERR_UNSUPPORTED
