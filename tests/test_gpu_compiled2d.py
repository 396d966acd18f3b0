"""GPU: the sweep kernels with compile-time tiles for 16-bit lattices other
than the six-neighbour one (VN4 in 128x128 tiles with 6 MC steps per launch
and 256x128 with 4, Moore8 in 128x128 and 256x128 tiles with 3, Moore26 in
32x16x16 tiles with 2 or 4 colour passes) against the general tile kernel and the
oracle, element by element (Sec. 3 trials, Sec. 4 Red/Black passes).

* single lattices of several tiles along both axes, grains in LDS (Q <=
  4096) and in global memory, MC step counts that end in a shorter launch
  (run by the general kernel): spins equal to the oracle's and to the
  general kernel's, and both queue the same trials;
* a caller's buffer (the last launch split in two) and values outside
  [0, Q) that stay inert;
* the default tilings of 2048^2 and 4096^2 VN4 and Moore8 lattices take
  this kernel (Moore8 ensembles in it: the ensemble tests).
"""
import os

import numpy as np
import pytest

import oracle
import paper_1007_3509_amd as hmc
import synth

pytestmark = pytest.mark.gpu
THREADS = max(1, min(16, os.cpu_count() or 1))

# torch before the library: the process then holds one HIP runtime, torch's
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def _energies(Q, seed):
    return synth.quantise(0.2 * (0.27 + 0.23 * np.random.default_rng(seed).random(Q)))


def _run(dims, nbr, Q, B, kT, chunks, seed, tiling, kernel, vseed=5):
    with hmc.Lattice(dims, nbr, Q, voronoi_seed=vseed, spin=hmc.HMC_I16) as lat:
        lat.set_grain_energy(B)
        lat.set_tiling(*tiling)
        hmc.hmc_set_sweep_kernel(lat.h, kernel)
        which = hmc.hmc_get_sweep_kernel(lat.h)
        start = lat.spins().astype(np.int32)
        hmc.hmc_profile(lat.h, True)
        hmc.hmc_profile_trials(lat.h)
        for n in chunks:
            lat.sweep(kT, n, seed)
        trials = hmc.hmc_profile_trials(lat.h)
        hmc.hmc_profile(lat.h, False)
        return start, lat.spins().astype(np.int32), trials, which


CASES = [(hmc.HMC_VN4, (384, 256), (128, 128, 1, 6), [6, 9]),
         (hmc.HMC_VN4, (256, 512), (128, 128, 1, 6), [6, 4]),
         (hmc.HMC_VN4, (512, 384), (256, 128, 1, 4), [4, 5]),
         (hmc.HMC_MOORE8, (384, 256), (128, 128, 1, 3), [3, 4]),
         (hmc.HMC_MOORE8, (768, 256), (256, 128, 1, 3), [6, 2]),
         (hmc.HMC_MOORE26, (64, 32, 48), (32, 16, 16, -4), [1, 2]),
         (hmc.HMC_MOORE26, (64, 32, 48), (32, 16, 16, -2), [2, 1]),
         (hmc.HMC_MOORE26, (32, 16, 16), (32, 16, 16, -2), [3])]


@pytest.mark.parametrize("nbr,dims,tiling,chunks", CASES)
@pytest.mark.parametrize("Q", [300, 6000])
def test_compiled_tiles_equal_general_kernel_and_oracle(nbr, dims, tiling, chunks, Q):
    kT, seed = 0.6, 31
    B = _energies(Q, Q + nbr)
    say(f"[gpu] compiled 2D nbr={nbr} dims={dims} tiling={tiling} Q={Q}")
    start, got, tr_a, which = _run(dims, nbr, Q, B, kT, chunks, seed, tiling, hmc.HMC_KERNEL_AUTO)
    _, gen, tr_g, which_g = _run(dims, nbr, Q, B, kT, chunks, seed, tiling, hmc.HMC_KERNEL_GENERIC)
    assert which == hmc.HMC_KERNEL_COMPILED and which_g == hmc.HMC_KERNEL_GENERIC
    want = oracle.sweep(start, nbr, dims, B, kT, sum(chunks), seed, threads=THREADS)
    assert not np.array_equal(want, start)
    assert np.array_equal(got, want), f"{int(np.sum(got != want))} sites differ from the oracle"
    assert np.array_equal(gen, want)
    assert tr_a == tr_g and tr_a > 0


@pytest.mark.parametrize("kT", [1e-3, 40.0])
def test_degenerate_temperatures(kT):
    dims, Q, seed = (256, 256), 500, 9
    B = _energies(Q, 3)
    say(f"[gpu] compiled 2D VN4 kT={kT}")
    start, got, tr_a, _ = _run(dims, hmc.HMC_VN4, Q, B, kT, [12], seed, (128, 128, 1, 6), hmc.HMC_KERNEL_AUTO)
    want = oracle.sweep(start, hmc.HMC_VN4, dims, B, kT, 12, seed, threads=THREADS)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("nbr,tiling", [(hmc.HMC_VN4, (128, 128, 1, 6)), (hmc.HMC_MOORE8, (128, 128, 1, 3))])
def test_wrapped_buffer_and_inert_values(nbr, tiling):
    dims, Q, kT, seed = (256, 256), 40, 0.8, 3
    s = oracle.voronoi(dims, Q, 9).reshape(dims[1], dims[0]).astype(np.int16)
    s[100:104, 20:90] = -1
    s[0, 0] = 300
    B = synth.quantise(np.linspace(0.0, 0.2, Q))
    t = torch.from_numpy(s.copy()).to("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    k = tiling[3]
    say(f"[gpu] compiled 2D wrapped int16 buffer nbr={nbr}")
    with hmc.Lattice(dims, nbr, Q, stream=stream, dev_ptr=t.data_ptr(), spin=hmc.HMC_I16) as lat:
        lat.set_grain_energy(B)
        lat.set_tiling(*tiling)
        assert hmc.hmc_get_sweep_kernel(lat.h) == hmc.HMC_KERNEL_COMPILED
        want = s.astype(np.int32)
        done = 0
        # one full launch (odd count: split in two), two, then a full and a short one
        for n in (k, 2 * k, k + 1):
            lat.sweep(kT, n, seed)
            want = oracle.sweep(want, nbr, dims, B, kT, n, seed, mcs0=done, threads=THREADS)
            done += n
            torch.cuda.synchronize()
            got = t.cpu().numpy().astype(np.int32)
            assert np.array_equal(got, want), f"after {done} steps {int(np.sum(got != want))} sites differ"
        assert np.all(got[100:104, 20:90] == -1) and got[0, 0] == 300


@pytest.mark.parametrize("passes", [2, 4])
def test_moore26_wrapped_buffer_and_inert_values(passes):
    """Moore26 launches of two or four colour passes start on any colour
    they divide."""
    dims, Q, kT, seed = (64, 32, 32), 40, 0.8, 3
    s = oracle.voronoi(dims, Q, 9).reshape(dims[2], dims[1], dims[0]).astype(np.int16)
    s[10:12, 3:20, 5:40] = -1
    s[0, 0, 0] = 300
    B = synth.quantise(np.linspace(0.0, 0.2, Q))
    t = torch.from_numpy(s.copy()).to("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    say(f"[gpu] compiled Moore26 wrapped int16 buffer, {passes} passes per launch")
    with hmc.Lattice(dims, hmc.HMC_MOORE26, Q, stream=stream, dev_ptr=t.data_ptr(), spin=hmc.HMC_I16) as lat:
        lat.set_grain_energy(B)
        lat.set_tiling(32, 16, 16, -passes)
        assert hmc.hmc_get_sweep_kernel(lat.h) == hmc.HMC_KERNEL_COMPILED
        want = s.astype(np.int32)
        done = 0
        for n in (1, 2):
            lat.sweep(kT, n, seed)
            want = oracle.sweep(want, hmc.HMC_MOORE26, dims, B, kT, n, seed, mcs0=done, threads=THREADS)
            done += n
            torch.cuda.synchronize()
            got = t.cpu().numpy().astype(np.int32)
            assert np.array_equal(got, want), f"after {done} steps {int(np.sum(got != want))} sites differ"
        assert np.all(got[10:12, 3:20, 5:40] == -1) and got[0, 0, 0] == 300


@pytest.mark.parametrize("nbr,side,tiling", [(hmc.HMC_VN4, 2048, (128, 128, 1, 6)),
                                             (hmc.HMC_MOORE8, 2048, (128, 128, 1, 3)),
                                             (hmc.HMC_VN4, 4096, (256, 128, 1, 4)),
                                             (hmc.HMC_MOORE8, 4096, (256, 128, 1, 3))])
def test_default_tiling_of_large_lattices_takes_the_compiled_kernel(nbr, side, tiling):
    with hmc.Lattice((side, side), nbr, 4000, spin=hmc.HMC_I16) as lat:
        assert tuple(hmc.hmc_get_tiling(lat.h)) == tiling
        assert hmc.hmc_get_sweep_kernel(lat.h) == hmc.HMC_KERNEL_COMPILED
    with hmc.Lattice((1024, 1024), hmc.HMC_VN4, 4000, spin=hmc.HMC_I16) as lat:
        assert hmc.hmc_get_sweep_kernel(lat.h) == hmc.HMC_KERNEL_GENERIC


def test_moore26_default_tiling_takes_the_compiled_kernel():
    w = synth.moore26_3d_128()
    with hmc.Lattice(w.dims, w.nbr, w.n_grains, spin=w.spin) as lat:
        assert tuple(hmc.hmc_get_tiling(lat.h)) == (32, 16, 16, -2)
        assert hmc.hmc_get_sweep_kernel(lat.h) == hmc.HMC_KERNEL_COMPILED
