"""Block reuse in the split FP32-map gather.

With many short work items (more than about 64 per workgroup) the gather takes
its items in runs of consecutive anchors and stages only the map column that
enters the 8 x 8 block (k_gather.hip).  Every item's block is still split with
the scale of its own maximum, so the result must equal the per-item path bit for
bit (the batch gather, which never reuses a block), repeat exactly from run to
run, and match the oracle, the direct sum of Eq. 2 (Galloway et al. 2022,
Sec. 2.1), to the FP32-form bar.
"""
import numpy as np
import pytest

import workloads as W
from parity import assert_parity

pytestmark = pytest.mark.gpu

# lmax 128: about 1.5e5 anchors, all hit by 4e6 uniform pointings (one item each),
# i.e. a few hundred items per workgroup of the persistent gather: runs of several.
L, K, N = 128, 8, 4_000_000


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2201_03478_amd import api
    api.N.load()
    dev = torch.device("cuda", 0)
    sky = W.sky_alm(L, 910)
    blm = W.beam_alm(L, K, 911)
    ptg = W.uniform_pointings(N, 912)
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    return torch, api, sky, blm, ptg, to(sky), to(blm), to(ptg.reshape(-1, 3))


def test_reuse_equals_per_item_path_and_repeats(env):
    torch, api, _, _, _, sky, blm, ptg = env
    plan = api.Plan(L, K)
    assert plan.info()["precision"] == 1  # the FP32-map form
    plan.set_sky_beam(sky, blm)
    first = plan.interpolate(ptg).clone()
    second = plan.interpolate(ptg).clone()
    torch.cuda.synchronize()
    assert torch.equal(first, second), "gather with block reuse is not repeatable"
    batch = api.Batch([dict(lmax=L, kmax=K, blm=blm, ptg=ptg)], L)
    (per_item,) = batch.run(sky, use_graph=False)
    torch.cuda.synchronize()
    diff = int((first != per_item).sum())
    assert diff == 0, "%d of %d samples differ from the per-item gather" % (diff, N)


def test_reuse_matches_oracle(env, oracle_lib):
    torch, api, sky_np, blm_np, ptg_np, sky, blm, ptg = env
    plan = api.Plan(L, K)
    plan.set_sky_beam(sky, blm)
    tod = plan.interpolate(ptg).double().cpu().numpy()
    idx = np.sort(np.random.default_rng(913).choice(N, 300, replace=False))
    ref = oracle_lib.convolve(sky_np, blm_np, L, K, ptg_np.reshape(-1, 3)[idx])
    assert_parity(tod[idx], ref, 1e-6, "gather with block reuse, lmax %d kmax %d" % (L, K))
