"""GPU: lattices over caller-owned device memory (a torch tensor's storage)
and network inference on device memory, through the C ABI.

* a wrapped tensor holds the oracle's spins after every sweep call, whatever
  the parity of the launch count (bit-exact);
* a wrapped lattice and a library-owned one give the same spins;
* values outside [0, Q) follow the oracle's inert rule site for site and are
  left out of the statistics;
* bad buffers are rejected before any device work;
* hmc_mlp_infer on device arrays and a side stream equals hmc_mlp_forward
  and follows the oracle's double-precision network within float32 error.
"""
import numpy as np
import pytest

import oracle
import paper_1007_3509_amd as hmc
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def _tensor_from(arr, dtype):
    return torch.from_numpy(np.ascontiguousarray(arr)).to(device="cuda:0", dtype=dtype)


@pytest.mark.parametrize("spin,tdtype", [(hmc.HMC_I16, torch.int16), (hmc.HMC_I32, torch.int32)])
@pytest.mark.parametrize("k,chunks", [(2, [5]), (4, [3]), (4, [6, 1]), (1, [1, 1, 2]), (-3, [1, 2]), (-1, [3])])
def test_wrapped_tensor_follows_oracle(spin, tdtype, k, chunks):
    dims, Q, vseed, seed, kT = (64, 48), 30, 11, 21, 0.7
    say(f"[gpu] wrap spin={spin} k={k} chunks={chunks}")
    start = oracle.voronoi(dims, Q, vseed).reshape(dims[1], dims[0])
    B = synth.quantise(np.linspace(0.05, 0.2, Q))
    t = _tensor_from(start, tdtype)
    stream = torch.cuda.current_stream().cuda_stream
    with hmc.Lattice(dims, hmc.HMC_VN4, Q, spin=spin, stream=stream, dev_ptr=t.data_ptr()) as lat:
        lat.set_grain_energy(B)
        lat.set_tiling(16, 16, 0, k)
        want = start.astype(np.int32)
        done = 0
        for n in chunks:
            lat.sweep(kT, n, seed)
            want = oracle.sweep(want, hmc.HMC_VN4, dims, B, kT, n, seed, mcs0=done)
            done += n
            torch.cuda.synchronize()
            got = t.cpu().numpy().astype(np.int32)
            assert np.array_equal(got, want), f"after {done} MCS: {int(np.sum(got != want))} sites differ"
        assert np.array_equal(lat.spins().astype(np.int32), want)
        # snapshot / restore and set_spins act on the caller's buffer too
        lat.set_spins(start)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy().astype(np.int32), start)


def test_wrapped_equals_owned_moore8():
    dims, Q, vseed, seed, kT = (64, 64), 60, 5, 8, 0.9
    say("[gpu] wrap vs owned moore8")
    start = oracle.voronoi(dims, Q, vseed).reshape(64, 64)
    B = synth.quantise(np.linspace(0.0, 0.3, Q))
    t = _tensor_from(start, torch.int16)
    stream = torch.cuda.current_stream().cuda_stream
    with hmc.Lattice(dims, hmc.HMC_MOORE8, Q, voronoi_seed=vseed) as own, \
            hmc.Lattice(dims, hmc.HMC_MOORE8, Q, stream=stream, dev_ptr=t.data_ptr()) as wr:
        for lat in (own, wr):
            lat.set_grain_energy(B)
            lat.sweep(kT, 7, seed)
        a, b = own.spins(), wr.spins()
        torch.cuda.synchronize()
        assert np.array_equal(a, b)
        assert np.array_equal(t.cpu().numpy(), a)


@pytest.mark.parametrize("pair", [False, True])
def test_out_of_range_values_are_inert(pair):
    """Values outside [0, Q) in a caller's buffer: the GPU follows the
    oracle's inert rule site for site (such a site never changes, such a
    neighbour is never proposed; with a pair table it bonds with nothing),
    and the statistics leave them out."""
    dims, Q, seed, kT = (32, 32), 4, 3, 1.0
    say(f"[gpu] wrap out-of-range values, pair={pair}")
    rng = np.random.default_rng(1)
    s = rng.integers(0, Q, size=(32, 32)).astype(np.int32)
    s[10:14, 6:20] = -1
    s[0, 0] = 99
    s[20, 5] = 1 << 20
    B = np.array([0, 3000, -2000, 1000], np.int32)
    t = _tensor_from(s, torch.int32)
    stream = torch.cuda.current_stream().cuda_stream
    with hmc.Lattice(dims, hmc.HMC_VN4, Q, spin=hmc.HMC_I32, stream=stream, dev_ptr=t.data_ptr()) as lat:
        lat.set_grain_energy(B)
        if pair:
            A = np.triu(rng.integers(20000, 90000, size=(Q, Q)), 1)
            Jp = (A + A.T).astype(np.int32)
            lat.set_pair_energy(Jp)
            want = oracle.sweep_pair(s, hmc.HMC_VN4, dims, Jp, B, kT, 20, seed)
        else:
            want = oracle.sweep(s, hmc.HMC_VN4, dims, B, kT, 20, seed)
        lat.sweep(kT, 20, seed)
        got = lat.spins()
        assert np.array_equal(got, want), f"{int(np.sum(got != want))} sites differ from the oracle"
        assert np.all(got[10:14, 6:20] == -1) and got[0, 0] == 99 and got[20, 5] == 1 << 20
        assert not np.array_equal(got, s)
        areas_o, n_o, mean_o, _ = oracle.texture(want, Q)
        assert np.array_equal(lat.grain_areas(), areas_o)
        n, mean, _ = lat.texture_stats()
        assert n == n_o and mean == mean_o
        assert lat.boundary_sites() == oracle.boundary_sites(want, hmc.HMC_VN4, dims, Q)


def test_wrap_rejects_bad_buffers():
    desc = hmc.make_desc((4096, 4096), hmc.HMC_VN4)
    small = torch.zeros(16, dtype=torch.int16, device="cuda:0")
    with pytest.raises(hmc.HmcError):
        hmc.hmc_lattice_wrap(desc, small.data_ptr(), 10)
    host = np.zeros(64 * 64, dtype=np.int16)
    with pytest.raises(hmc.HmcError):
        hmc.hmc_lattice_wrap(hmc.make_desc((64, 64), hmc.HMC_VN4), host.ctypes.data, 10)
    big = torch.zeros(64 * 64 + 1, dtype=torch.int16, device="cuda:0")
    with pytest.raises(hmc.HmcError):   # odd byte offset
        hmc.hmc_lattice_wrap(hmc.make_desc((64, 64), hmc.HMC_VN4), big.data_ptr() + 1, 10)
    with pytest.raises(hmc.HmcError):
        hmc.hmc_lattice_wrap(hmc.make_desc((64, 64), hmc.HMC_VN4), 0, 10)


def test_mlp_infer_on_device_and_side_stream():
    say("[gpu] mlp infer")
    M = hmc.hmc_mlp_create(seed=17)
    try:
        theta, _ = hmc.hmc_mlp_get_params(M)
        rng = np.random.default_rng(6)
        X = rng.uniform(-1, 1, size=(1000, 9)).astype(np.float32)
        Xd = torch.from_numpy(X).to("cuda:0")
        yd = torch.empty(1000, dtype=torch.float32, device="cuda:0")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            hmc.hmc_mlp_infer(M, Xd.data_ptr(), yd.data_ptr(), 1000, side.cuda_stream)
        side.synchronize()
        got = yd.cpu().numpy()
        assert np.array_equal(got, hmc.hmc_mlp_forward(M, X))
        want = oracle.mlp_forward(theta.astype(np.float64), X.astype(np.float64))
        assert np.max(np.abs(got - want)) <= 1e-5 * max(1.0, float(np.max(np.abs(want))))
        hmc.hmc_mlp_infer(M, Xd.data_ptr(), yd.data_ptr(), 0, None)   # n = 0 is a no-op
        with pytest.raises(hmc.HmcError):
            hmc.hmc_mlp_infer(M, 0, yd.data_ptr(), 10, None)
    finally:
        hmc.hmc_mlp_free(M)


@pytest.mark.parametrize("pair", [False, True])
def test_nfold_on_wrapped_tensor_keeps_out_of_range_values(pair):
    """The n-fold way on a caller's buffer that holds values outside [0, Q):
    spins, event count and clock equal the oracle's under the same inert
    rule as the sweep."""
    dims, Q = (32, 32), 4
    say(f"[gpu] nfold on a wrapped tensor with out-of-range values, pair={pair}")
    rng = np.random.default_rng(2)
    s = rng.integers(0, Q, size=(32, 32)).astype(np.int32)
    s[10:14, 6:20] = -1
    s[0, 0] = 99
    B = np.array([0, 3000, -2000, 1000], np.int32)
    Jp = None
    t = _tensor_from(s, torch.int32)
    stream = torch.cuda.current_stream().cuda_stream
    with hmc.Lattice(dims, hmc.HMC_VN4, Q, spin=hmc.HMC_I32, stream=stream, dev_ptr=t.data_ptr()) as lat:
        lat.set_grain_energy(B)
        if pair:
            A = np.triu(rng.integers(20000, 90000, size=(Q, Q)), 1)
            Jp = (A + A.T).astype(np.int32)
            lat.set_pair_energy(Jp)
        lat.nfold(0.8, 3.0, 5)
        torch.cuda.synchronize()
        got = t.cpu().numpy()
        assert np.array_equal(got, lat.spins())
        want, t_last, n_ev, _ = oracle.nfold(s, hmc.HMC_VN4, dims, B, 0.8, 5, 3.0, Jp=Jp)
        assert np.array_equal(got, want), f"{int(np.sum(got != want))} sites differ from the oracle"
        assert lat.nfold_clock()[1:] == (t_last, n_ev)
        assert np.all(got[10:14, 6:20] == -1) and got[0, 0] == 99
        assert n_ev > 50
