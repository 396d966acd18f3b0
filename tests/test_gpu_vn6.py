"""GPU: the six-neighbour 16-bit sweep kernel with compile-time tiles
against the general tile kernel and the oracle, element by element (Sec. 3
trials, Sec. 4 Red/Black passes).

* every compiled tile, two and one colour passes per launch, grains in LDS
  (Q <= 4096) and in global memory (also with an energy spread beyond
  2^16), on lattices of several tiles along every axis, with more tiles than
  workgroups (each walks several, prefetching the next): spins equal to the
  oracle's and to the general kernel's;
* both kernels queue the same trials (profiling counter);
* a caller's buffer (launch counts of either parity, so single-pass
  launches starting on either colour) and values outside [0, Q) that stay
  inert;
* the default tiling of the 256^3 workload (32x16x16, two workgroups per
  CU) takes this kernel.
"""
import numpy as np
import pytest

import oracle
import paper_1007_3509_amd as hmc
import synth

pytestmark = pytest.mark.gpu

# torch before the library: the process then holds one HIP runtime, torch's
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def _run(dims, Q, B, kT, chunks, seed, tiling, kernel, vseed=5, init=None):
    with hmc.Lattice(dims, hmc.HMC_VN6, Q, voronoi_seed=None if init is not None else vseed) as lat:
        if init is not None:
            lat.set_spins(init)
        lat.set_grain_energy(B)
        lat.set_tiling(*tiling)
        hmc.hmc_set_sweep_kernel(lat.h, kernel)
        start = lat.spins().astype(np.int32)
        hmc.hmc_profile(lat.h, True)
        hmc.hmc_profile_trials(lat.h)
        for n in chunks:
            lat.sweep(kT, n, seed)
        trials = hmc.hmc_profile_trials(lat.h)
        hmc.hmc_profile(lat.h, False)
        return start, lat.spins().astype(np.int32), trials


@pytest.mark.parametrize("tiling", [(64, 16, 16, 1), (32, 32, 16, 1), (32, 16, 16, 1), (16, 16, 16, 1),
                                    (64, 16, 8, 1), (64, 16, 16, -1), (32, 16, 16, -2)])
@pytest.mark.parametrize("Q", [300, 6000])
def test_compiled_tiles_equal_general_kernel_and_oracle(tiling, Q):
    dims, kT, seed = (128, 64, 48), 0.6, 11
    rng = np.random.default_rng(Q)
    B = synth.quantise(0.15 * (0.27 + 0.23 * rng.random(Q)))
    say(f"[gpu] vn6 tiling={tiling} Q={Q}")
    start, got, tr_a = _run(dims, Q, B, kT, [3, 4], seed, tiling, hmc.HMC_KERNEL_AUTO)
    _, gen, tr_g = _run(dims, Q, B, kT, [3, 4], seed, tiling, hmc.HMC_KERNEL_GENERIC)
    want = oracle.sweep(start, hmc.HMC_VN6, dims, B, kT, 7, seed, threads=8)
    assert np.array_equal(got, want), f"{int(np.sum(got != want))} sites differ from the oracle"
    assert np.array_equal(gen, want)
    assert tr_a == tr_g and tr_a > 0


@pytest.mark.parametrize("tiling", [(64, 16, 16, 1), (32, 16, 16, -1)])
def test_wide_energy_spread_reads_grains_from_global_memory(tiling):
    """Grain energies spread over more than 2^16 fixed-point units cannot be
    staged as 16-bit offsets; the kernel reads them from global memory."""
    dims, Q, kT, seed = (128, 64, 48), 6000, 1.5, 13
    B = synth.quantise(np.random.default_rng(2).uniform(-1.2, 1.2, Q))
    assert int(B.max()) - int(B.min()) >= 65536
    say(f"[gpu] vn6 wide spread tiling={tiling}")
    start, got, tr_a = _run(dims, Q, B, kT, [5], seed, tiling, hmc.HMC_KERNEL_AUTO)
    _, gen, tr_g = _run(dims, Q, B, kT, [5], seed, tiling, hmc.HMC_KERNEL_GENERIC)
    want = oracle.sweep(start, hmc.HMC_VN6, dims, B, kT, 5, seed, threads=8)
    assert np.array_equal(got, want) and np.array_equal(gen, want)
    assert tr_a == tr_g


@pytest.mark.parametrize("dims,tiling", [((256, 128, 128), (16, 16, 16, 1)), ((144, 128, 128), (16, 16, 16, 1)),
                                         ((144, 128, 128), (16, 16, 16, -1)), ((256, 256, 128), (32, 16, 16, 1)),
                                         ((320, 128, 128), (64, 16, 16, 1)), ((320, 128, 128), (64, 16, 16, -1))])
def test_workgroups_walk_several_tiles(dims, tiling):
    """More tiles than workgroups: with two workgroups per CU (16^3 and
    32x16x16 tiles) each walks several tiles, loading the next box after
    storing one; with one per CU (64x16x16) each walks several, prefetching
    the next box during the passes.  576 and 320 tiles do not split evenly."""
    Q, kT, seed = 6000, 0.6, 17
    B = synth.quantise(0.15 * (0.27 + 0.23 * np.random.default_rng(4).random(Q)))
    say(f"[gpu] vn6 several tiles per workgroup dims={dims} tiling={tiling}")
    start, got, tr_a = _run(dims, Q, B, kT, [2, 1], seed, tiling, hmc.HMC_KERNEL_AUTO)
    _, gen, tr_g = _run(dims, Q, B, kT, [2, 1], seed, tiling, hmc.HMC_KERNEL_GENERIC)
    want = oracle.sweep(start, hmc.HMC_VN6, dims, B, kT, 3, seed, threads=8)
    assert np.array_equal(got, want), f"{int(np.sum(got != want))} sites differ from the oracle"
    assert np.array_equal(gen, want) and tr_a == tr_g


def test_wrapped_buffer_parities_and_inert_values():
    dims, Q, kT, seed = (64, 32, 32), 40, 0.8, 3
    s = oracle.voronoi(dims, Q, 9).reshape(dims[2], dims[1], dims[0]).astype(np.int16)
    s[10:12, 3:20, 5:40] = -1
    s[0, 0, 0] = 300
    B = synth.quantise(np.linspace(0.0, 0.2, Q))
    t = torch.from_numpy(s.copy()).to("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    say("[gpu] vn6 wrapped int16 buffer")
    with hmc.Lattice(dims, hmc.HMC_VN6, Q, stream=stream, dev_ptr=t.data_ptr()) as lat:
        lat.set_grain_energy(B)
        lat.set_tiling(32, 16, 16, 1)
        want = s.astype(np.int32)
        done = 0
        for n in (1, 2, 3):          # odd and even launch counts: the last launch is split into single passes
            lat.sweep(kT, n, seed)
            want = oracle.sweep(want, hmc.HMC_VN6, dims, B, kT, n, seed, mcs0=done)
            done += n
            torch.cuda.synchronize()
            got = t.cpu().numpy().astype(np.int32)
            assert np.array_equal(got, want), f"after {done} steps {int(np.sum(got != want))} sites differ"
        assert np.all(got[10:12, 3:20, 5:40] == -1) and got[0, 0, 0] == 300


def test_default_3d_tiling_takes_the_compiled_kernel():
    w = synth.schmid_3d_256()
    with hmc.Lattice(w.dims, w.nbr, w.n_grains, spin=w.spin) as lat:
        assert tuple(hmc.hmc_get_tiling(lat.h)) == (32, 16, 16, 1)
        assert hmc.hmc_get_sweep_kernel(lat.h) == hmc.HMC_KERNEL_COMPILED
