"""The allocation-free statistics entry point, hmc_texture_stats_static,
against hmc_texture_stats on the same spins and against the oracle (integer
counts, bit-exact; ratios formed the same way on the host): two calls in a
row on one device, the second with a smaller input (fewer sites, grains and
bins, and values outside [0, Q)), so that nothing of the first call's
scratch contents leaks into the second.  Oversized requests are refused on
the host before any device work."""
import numpy as np
import pytest

import oracle
import paper_1007_3509_amd as hmc
import synth

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def test_static_limits_are_checked_on_the_host():
    fake = 1 << 20            # never dereferenced: the sizes are refused first
    for kw in (dict(n_grains=hmc.HMC_STATIC_MAX_GRAINS + 1), dict(n_grains=0),
               dict(n_bins=hmc.HMC_STATIC_MAX_BINS + 1, grain_bin=np.zeros(10, np.int32)),
               dict(n_sites=0), dict(n_sites=1 << 32), dict(spin=7),
               dict(n_bins=2, grain_bin=np.array([0, 1, 2] + [0] * 7, np.int32))):
        args = dict(dev_spins=fake, spin=hmc.HMC_I16, n_sites=100, n_grains=10)
        args.update(kw)
        with pytest.raises(hmc.HmcError) as e:
            hmc.hmc_texture_stats_static(**args)
        assert e.value.status == hmc.HMC_E_INVAL


@pytest.mark.gpu
def test_static_stats_equal_lattice_stats_on_two_calls():
    cases = [
        # (dims, nbr, spin, Q, n_bins, sweeps, inert)
        ((96, 64, 32), hmc.HMC_VN6, hmc.HMC_I16, 5000, 23, 5, False),
        ((48, 40), hmc.HMC_VN4, hmc.HMC_I32, 300, 7, 9, True),
    ]
    stream = torch.cuda.current_stream()
    for dims, nbr, spin, Q, n_bins, sweeps, inert in cases:
        say(f"[gpu] static texture stats dims={dims} Q={Q} bins={n_bins} inert={inert}")
        rng = np.random.default_rng(Q)
        B = synth.quantise(0.2 * (0.27 + 0.23 * rng.random(Q)))
        gb = rng.integers(-1, n_bins, size=Q).astype(np.int32)
        with hmc.Lattice(dims, nbr, Q, voronoi_seed=Q + 1, spin=spin) as lat:
            lat.set_grain_energy(B)
            lat.sweep(0.7, sweeps, 3)
            spins = lat.spins().astype(np.int32)
            if inert:
                spins.reshape(-1)[::17] = -1
                spins.reshape(-1)[5] = Q + 3
                t = torch.from_numpy(spins).to(device="cuda:0", dtype=torch.int32)
            else:
                t = torch.from_numpy(spins.astype(np.int16)).to("cuda:0")
            want = lat.texture_stats(gb, n_bins) if not inert else None
        N = spins.size
        torch.cuda.synchronize()
        got = hmc.hmc_texture_stats_static(t.data_ptr(), spin, N, Q, gb, n_bins, stream=stream.cuda_stream)
        _, ng_o, mean_o, frac_o = oracle.texture(spins, Q, gb, n_bins)
        assert got[0] == ng_o and got[1] == mean_o and np.array_equal(got[2], frac_o)
        if want is not None:
            assert got[0] == want[0] and got[1] == want[1] and np.array_equal(got[2], want[2])
        # no bins: the grain count and mean area alone
        n0, m0, f0 = hmc.hmc_texture_stats_static(t.data_ptr(), spin, N, Q, None, 0, stream=stream.cuda_stream)
        assert (n0, m0) == (ng_o, mean_o) and f0.size == 0
    with pytest.raises(hmc.HmcError):   # host memory is refused
        host = np.zeros(64, np.int16)
        hmc.hmc_texture_stats_static(host.ctypes.data, hmc.HMC_I16, 64, 4)
