"""Full-size workloads in the benchmark's launch configuration, checked on
sampled outputs the oracle can compute one by one (particles are independent)
and through properties that hold at any size.

Long runs (1e5 turns): particles near the separatrix are chaotic, so besides
per-particle bounds for the core, the distributions of the Hamiltonian error
dH/|H_sep| are compared in logarithmic bins from 1e-10 to 1e-2: GPU and oracle
may disagree on at most 0.5% of the sampled particles.
"""
import numpy as np
import pytest

import oracle
from synth import (SPS_RING, SIGMA_DP, SIGMA_Z, SEEDS, batched_specs, gaussian_bunch,
                   join_f32c, ring_for, split_f32c)
from tests._parity import bucket_error, moment_error, near_separatrix

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    m.ltrk_set_plan()
    yield m
    m.ltrk_set_plan()


def dh_histogram(z, dp, z0, dp0, ring):
    c = oracle.derive(ring)
    dh = np.abs(oracle.hamiltonian(z, dp, ring) - oracle.hamiltonian(z0, dp0, ring)) / abs(c["H_sep"])
    edges = np.concatenate([[0.0], np.logspace(-10, -2, 17), [np.inf]])
    return np.histogram(dh, bins=edges)[0]


def test_precision_workload_fp64_and_f32c(ltrk):
    """1e7 particles x 1e5 turns, leap-frog: FP64 against the oracle on a
    strided sample of 300 particles; F32C moments against FP64 moments of the
    full population; the last moment rows against two-pass moments of the
    final states."""
    n, T = 10_000_000, 100_000
    z_in, dp_in = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, SEEDS["precision"])
    zh, zc = split_f32c(z_in)
    dh, dc = split_f32c(dp_in)
    z0, dp0 = join_f32c(zh, zc), join_f32c(dh, dc)
    stream = torch.cuda.Stream()
    z, dp = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    m64 = torch.empty((T, 5), dtype=torch.float64, device="cuda")
    f32 = [torch.as_tensor(a).cuda() for a in (zh, dh, zc, dc)]
    m32 = torch.empty((T, 5), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        ltrk.ltrk_track_f64(z, dp, T, SPS_RING, "leapfrog", m64, stream=stream)
        ltrk.ltrk_track_f32c(*f32, T, SPS_RING, "leapfrog", m32, stream=stream)
    torch.cuda.synchronize()
    zg, dg, mg = z.cpu().numpy(), dp.cpu().numpy(), m64.cpu().numpy()
    idx = np.arange(0, n, n // 300)
    zr, dr, _ = oracle.track(z0[idx], dp0[idx], T, SPS_RING, "leapfrog", with_moments=False,
                             threads=1)
    e = bucket_error(zg[idx], dg[idx], zr, dr, SPS_RING)
    near = near_separatrix(z0[idx], dp0[idx], SPS_RING)
    assert np.median(e[~near]) <= 1e-10 and e[~near].max() <= 1e-8
    hg = dh_histogram(zg[idx], dg[idx], z0[idx], dp0[idx], SPS_RING)
    hr = dh_histogram(zr, dr, z0[idx], dp0[idx], SPS_RING)
    assert np.abs(hg - hr).sum() <= max(2, int(0.005 * idx.size))
    assert moment_error(mg[-1:], oracle.moments(zg, dg)[None, :]).max() <= 1e-12
    a = [x.cpu().numpy() for x in f32]
    z32, d32 = join_f32c(a[0], a[2]), join_f32c(a[1], a[3])
    mf = m32.cpu().numpy()
    assert moment_error(mf[-1:], oracle.moments(z32, d32)[None, :]).max() <= 1e-12
    # F32C against FP64: the bound the measured 1e-5 level of the moments sits under
    assert moment_error(mf, mg).max() <= 5e-5


def test_batched_workload_full_size(ltrk):
    """256 bunches (sizes log-uniform 1e3-1e6, own V and h), 1e4 turns, FP64,
    the benchmark's launch plan: 16 particles of every bunch against the
    oracle and every bunch's last moment row against the two-pass moments of
    its final state."""
    T = 10_000
    specs = batched_specs()
    bunches, inits = [], []
    for s in specs:
        r = ring_for(s)
        c = oracle.derive(r)
        z0, dp0 = gaussian_bunch(s.n, s.sigma_dp * c["D"] / c["omega"], s.sigma_dp, s.seed)
        inits.append((z0, dp0))
        bunches.append(dict(z=torch.as_tensor(z0).cuda(), dp=torch.as_tensor(dp0).cuda(), ring=r,
                            moments=torch.empty((T, 5), dtype=torch.float64, device="cuda")))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ltrk.ltrk_track_batched(bunches, T, "leapfrog", "f64", stream=stream)
    torch.cuda.synchronize()
    worst_core = 0.0
    for s, b, (z0, dp0) in zip(specs, bunches, inits):
        r = ring_for(s)
        zg, dg = b["z"].cpu().numpy(), b["dp"].cpu().numpy()
        idx = np.linspace(0, s.n - 1, 16).astype(np.int64)
        zr, dr, _ = oracle.track(z0[idx], dp0[idx], T, r, "leapfrog", with_moments=False,
                                 threads=1)
        e = bucket_error(zg[idx], dg[idx], zr, dr, r)
        near = near_separatrix(z0[idx], dp0[idx], r)
        if (~near).any():
            worst_core = max(worst_core, e[~near].max())
        mom = b["moments"][-1:].cpu().numpy()
        assert moment_error(mom, oracle.moments(zg, dg)[None, :]).max() <= 1e-12
    assert worst_core <= 1e-9
