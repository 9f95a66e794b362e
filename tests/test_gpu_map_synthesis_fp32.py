"""The FP32-map synthesis against the FP64 one, stage by stage.

The FP32-map form computes the ring sums, the theta upsampling and the phi
synthesis in FP64 but stores F, G and the maps as FP32 (complex64), and its
compile-time transforms keep their LDS buffers in complex64 (one rounding per
radix pass).  Its component maps, the spin maps of Eq. 9 (Galloway et al. 2022,
Sec. 2.1) on the oversampled grid, must then equal the FP64 form's maps to a few
FP32 roundings.  The cases cover the three compile-time transform lengths
(lmax 256, 512, 1024) and a runtime-planned one (lmax 300).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2201_03478_amd import api
    api.N.load()
    return torch, api, torch.device("cuda", 0)


@pytest.mark.parametrize("L,K", [(256, 32), (512, 100), (1024, 16), (300, 8)])
def test_fp32_maps_match_fp64_maps(env, L, K):
    torch, api, dev = env
    sky = torch.from_numpy(W.sky_alm(L, 1200 + L)).to(dev)
    blm = torch.from_numpy(W.beam_alm(L, K, 1300 + K)).to(dev)
    maps = {}
    for prec in ("f64maps_f32gather", "fp64"):
        plan = api.Plan(L, K, prec, kernel_width=8)
        plan.set_sky_beam(sky, blm)
        inf = plan.info()
        maps[prec] = plan.debug_stage(1)[:, :, :inf["n_comp"]].double()
        torch.cuda.synchronize()
        plan.close()
    m32, m64 = maps["f64maps_f32gather"], maps["fp64"]
    assert m32.shape == m64.shape
    d = m32 - m64
    rel = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(m64))
    mx = float(d.abs().max() / m64.abs().max())
    print("lmax %d kmax %d: FP32 maps vs FP64 maps rel-L2 %.3e, max %.3e" % (L, K, rel, mx))
    # a few FP32 roundings: measured 5e-8 to 8e-8 (rel-L2) and 8e-8 to 1.8e-7 (max)
    assert rel <= 4e-7, rel
    assert mx <= 2e-6, mx
