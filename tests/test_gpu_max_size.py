"""The largest lattices: above 4 GiB per population buffer the byte offsets of the bounce-back fast
path no longer fit in 32 bits, so the step takes the general kernel (64-bit addressing) and the
overlapped step is unavailable. 400 x 384 x 384 FP32 (59 M sites, 4.5 GB per population buffer),
one bubble, two method steps, against the oracle on the whole lattice (about 21 GB of host
memory), and the lattice-size limit of the descriptor."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_common import gpu_sim, oracle_state, rel_l2
from paper_1710_07073_amd import lbm as L

BB = O.BC_BOUNCE_BACK


@pytest.mark.gpu
def test_lattice_above_4gib_takes_the_general_step_and_matches_the_oracle():
    shape = (400, 384, 384)
    n = int(np.prod(shape))
    assert 19 * n * 4 > 2 ** 32
    w = W.Workload("max_fp32_400x384x384", shape, 1.6, (BB,) * 6, np.array([[199.5], [191.5], [8.0]]),
                   np.array([4.0]), W.params(g=1e-4, sigma=W.sigma_for(1e-4, 4.0)), 2, "f32")
    print(f"[case] {w.name}: {n} sites, {19 * n * 4 / 1e9:.2f} GB per population buffer", flush=True)
    sim = gpu_sim(w)
    assert L.lbm_get_overlap(sim.ctx) == (True, False)  # on by default, not available at this size
    sim.step(w.steps)
    _, u, sums = sim.moments()
    u = u.double().cpu().numpy()
    x = sim.bubbles.positions()
    rng = np.random.default_rng(3)
    idx = torch.from_numpy(rng.integers(0, 19 * n, 2_000_000))
    g = sim.populations().reshape(-1)[idx.to(sim.device)].double().cpu().numpy()
    sim.check()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    lat, bub, P = oracle_state(w)
    for _ in range(w.steps):
        O.method_step(lat, P, bub)
    _, u_o, sums_o = lat.moments()
    eu = rel_l2(u, u_o)
    eg = np.abs(g - lat.g.reshape(-1)[idx.numpy()]).max()
    print(f"rel-L2 u {eu:.2e}, max |dg| over 2e6 sampled populations {eg:.2e}, "
          f"|dx_b| {np.abs(x - bub.pos).max():.2e}", flush=True)
    assert eu <= 2e-5
    assert eg <= 1e-6  # FP32 shifted populations of order 1e-3 after two steps
    assert np.abs(x - bub.pos).max() <= 1e-6
    assert abs(sums[0] - sums_o[0]) <= 1e-6 * n


def test_lattice_size_limit():
    """19 N must stay below 2^31 (element indices in 31 bits): 113.0 M sites at most."""
    ok = L.make_desc((512, 512, 431), 1.0, L.LBM_FP32_SHIFTED)  # 19 N = 2146697216
    L.lbm_bytes_required(ok)
    too_big = L.make_desc((512, 512, 432), 1.0, L.LBM_FP32_SHIFTED)  # 19 N = 2151677952
    with pytest.raises(L.LbmError) as e:
        L.lbm_bytes_required(too_big)
    assert e.value.code == L.LBM_EINVAL
