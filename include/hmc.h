/*
 * hmc.h -- C ABI of libhmc, the MI355X (gfx950) implementation of the
 * red/black Q-state Potts sweep with a per-grain bulk energy.
 *
 * The method: Zhang, Dingreville, Bartel, Lusk, "Hybrid Monte Carlo
 * simulation of stress-induced texture evolution with inelastic effects"
 * (arXiv:1007.3509).
 *   Sec. 3, Eq. (7): H = sum over sites and their M neighbours of the bond
 *     energy plus a bulk energy b_i per site.  Bonds cost J between unlike
 *     spins (J(1-delta), each bond once); b_i = b(q_i) is a property of the
 *     grain (Sec. 6: a swept site inherits the overtaking grain's stored
 *     dislocation energy).
 *   Sec. 3: a trial flip is accepted with a probability that depends on the
 *     change of H (Metropolis, min(1, exp(-dE/kT))).
 *   Sec. 4: Red/Black updating -- one colour class per half step, no state
 *     changes until the half step is over.
 *
 * Conventions shared by every call
 *   - Every call returns an hmc_status; nothing throws across the ABI.
 *     On failure hmc_last_error() gives a message (thread-local, valid until
 *     the next hmc_* call on the same thread).
 *   - Arguments are validated on the host before any device work, so invalid
 *     input never reaches a kernel.
 *   - Spins: x fastest, row-major, periodic, values 0..Q-1 (Q = n_grains),
 *     int16 (Q <= 32767) or int32.  Every side even and >= 4; N < 2^32.
 *   - Energies: int32 in units of 2^-16 (J_fx = 65536*J; B[q] = b(q)*65536).
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with
 *     key = (lo32(seed), hi32(seed)), counter = (site, mcs, colour, 0).
 *     Word 0 picks the trial spin, word 1 decides acceptance.
 *   - Acceptance is integer: d = J_fx*(c(q) - c(q')) + B[q'] - B[q]
 *     (c(s) = number of neighbours holding s); accept iff d <= 0 or
 *     r1 < T(d) = min(2^32-1, floor(2^32 exp(-d / (65536 kT)))), T built on
 *     the host in double precision with the C library exp.
 *   - Neighbour order: VN4 +x,-x,+y,-y; VN6 adds +z,-z; Moore8 adds
 *     (+1,+1),(-1,-1),(+1,-1),(-1,+1); Moore26 (dx,dy,dz) in {-1,0,1}^3\{0}
 *     lexicographic in (dz,dy,dx).  Colours: VN4 (x+y)&1, VN6 (x+y+z)&1,
 *     Moore8 (x&1)|(y&1)<<1, Moore26 (x&1)|(y&1)<<1|(z&1)<<2, passes
 *     c = 0..C-1 every MC step.
 *   - Determinism: final spins are a function of (initial spins, B, kT, seed,
 *     starting MC step, neighbourhood, trial mode, J_fx) only -- not of the
 *     tiling, the launch split, or how n_mcs is divided between calls.
 *   - Streams: a lattice is bound to one HIP stream (NULL: the library makes
 *     its own).  hmc_sweep is asynchronous; calls that return data to the host
 *     synchronise that stream.  A handle is not thread-safe; distinct handles
 *     are independent.
 *   - Ownership: *_create / *_init allocate, *_free releases.  Host arrays
 *     passed in are copied before return.  Output buffers belong to the caller.
 */
#ifndef HMC_H
#define HMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hmc_status;
enum {
    HMC_OK = 0,
    HMC_E_INVAL = -1,    /* bad argument (null pointer, size, enum, range) */
    HMC_E_NOMEM = -2,    /* device allocation failed or HMC_MAX_BYTES exceeded */
    HMC_E_DEVICE = -3,   /* a HIP call failed (message carries hipGetErrorString) */
    HMC_E_RANGE = -4,    /* an energy change could leave int32, or a table is too large */
    HMC_E_STATE = -5,    /* handle in the wrong state (e.g. ensemble member changed) */
    HMC_E_INTERNAL = -6
};

enum { HMC_VN4 = 0, HMC_MOORE8 = 1, HMC_VN6 = 2, HMC_MOORE26 = 3 };   /* C = 2, 4, 2, 8 */
enum { HMC_I16 = 0, HMC_I32 = 1 };
/* Trial spin.  NEIGHBOUR (production): the spin of a neighbour picked by
 * word 0.  UNIFORM (test mode): q' = (q + 1 + floor(r0*(Q-1)/2^32)) mod Q,
 * a symmetric proposal under which the Boltzmann distribution of Eq. (7)
 * is invariant.  The paper does not name the trial rule (Sec. 3). */
enum { HMC_PROP_NEIGHBOUR = 0, HMC_PROP_UNIFORM = 1 };

typedef struct {
    int32_t ndim;       /* 2 (VN4, Moore8) or 3 (VN6, Moore26) */
    int32_t dims[3];    /* Lx, Ly, Lz (Lz ignored for ndim 2); even, >= 4 */
    int32_t nbr;        /* HMC_VN4 .. HMC_MOORE26 */
    int32_t spin;       /* HMC_I16 or HMC_I32 */
    int32_t proposal;   /* HMC_PROP_NEIGHBOUR or HMC_PROP_UNIFORM */
    int32_t J_fx;       /* 65536 * J, in [1, 2^24] */
} hmc_lattice_desc;

typedef struct hmc_lattice_s hmc_lattice;

/* Library version of this header's ABI (incremented on any change). */
int32_t hmc_abi_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *hmc_last_error(void);

/* Number of HIP devices visible (0 without a GPU); never fails. */
int32_t hmc_device_count(void);

/* Allocate a lattice with all spins 0, bulk energies 0 and MC step 0.
 * n_grains = Q, the number of spin values (1..32767 for int16, 1..2^31-1
 * for int32).  stream: a hipStream_t, or NULL for a library-owned stream.
 * Errors: INVAL (desc, sizes, Q), NOMEM, DEVICE. */
hmc_status hmc_lattice_create(const hmc_lattice_desc *desc, int32_t n_grains, void *stream,
                              hmc_lattice **out);

/* As hmc_lattice_create, then the initial microstructure (the paper does not
 * specify one; a seeded Voronoi tessellation is used): point g has fixed-point
 * coordinates X_k = floor(r_k * 256 L_k / 2^32) from Philox(counter =
 * (g, 0, 0, 0x564F524E), key = voronoi_seed); site x sits at 256 x; every
 * site takes the index of the nearest point under periodic squared distance
 * (integers), ties to the lower index.  Grains may be empty. */
hmc_status hmc_lattice_init(const hmc_lattice_desc *desc, int32_t n_grains, uint64_t voronoi_seed,
                            void *stream, hmc_lattice **out);

/* As hmc_lattice_create, but over the caller's device buffer dev_spins
 * (N spins of the descriptor's type, e.g. a torch tensor's storage), which
 * the lattice borrows: it is neither cleared nor freed, the caller keeps it
 * alive until hmc_lattice_free, and after every call that changes the spins
 * the current state is back in it once the lattice's stream reaches that
 * point (the library keeps a second buffer of its own for the sweep).
 * Values outside [0, Q) are never changed, never proposed and not counted
 * by the statistics.  Errors: INVAL (NULL, not device memory, allocation
 * smaller than the lattice, misaligned, and as hmc_lattice_create), NOMEM,
 * DEVICE. */
hmc_status hmc_lattice_wrap(const hmc_lattice_desc *desc, void *dev_spins, int32_t n_grains, void *stream,
                            hmc_lattice **out);

/* Release a lattice (synchronises its stream first).  NULL is a no-op. */
hmc_status hmc_lattice_free(hmc_lattice *L);

/* Per-grain bulk energy b(q) of Eq. (7) in 2^-16 units (Sec. 6: carried by
 * the grain).  B_fx: int32[n_grains], host memory (on_device = 0) or device
 * memory (on_device = 1, read after the work queued on the lattice's stream);
 * copied, so the caller may reuse it on return.  The upload is queued on the
 * lattice's stream: sweeps queued before the call use the old energies, later
 * ones the new, and a host array is not held up by the sweeps still running.
 * n_grains must equal the lattice's Q.
 * Errors: INVAL; RANGE if |J_fx|*M + 2 max|B| >= 2^31. */
hmc_status hmc_set_grain_energy(hmc_lattice *L, const int32_t *B_fx, int32_t n_grains, int32_t on_device);

/* Bond energy per pair of spin values (Eq. (7) writes J for each pair
 * q_i, q_n; the closing section names misorientation-dependent boundary
 * energy as the use of that freedom).  Jp: int32[Q*Q], row-major, Jp[a*Q+b]
 * the energy of an unlike bond between spins a and b in 2^-16 units;
 * symmetric, zero diagonal, entries in [0, 2^24]; host (on_device = 0) or
 * device memory (on_device = 1); copied (4 Q^2 bytes on the device).
 * While set, hmc_sweep uses dE = sum over the M neighbours s_k of
 * (Jp[q'][s_k] - Jp[q][s_k]) + B[q'] - B[q] with the same trials, the same
 * random numbers and the threshold T(d) of every d > 0; the descriptor's
 * J_fx is not used.  Jp = NULL restores the uniform bond energy J_fx.
 * Ensembles do not take lattices in this mode.  Synchronous.
 * Errors: INVAL (NULL lattice, n_grains != Q, table not symmetric, nonzero
 * diagonal, entries out of range), RANGE (M max Jp + 2 max|B| >= 2^31),
 * NOMEM, DEVICE. */
hmc_status hmc_set_pair_energy(hmc_lattice *L, const int32_t *Jp, int32_t n_grains, int32_t on_device);

/* Read-Shockley pair energies of Q grain orientations, computed on the GPU:
 * theta = misorientation angle of grains a and b (smallest rotation angle of
 * g_b g_a^T over the 24 proper rotations of the cube; euler: Q x 3 Bunge
 * angles, passive sample -> crystal), J = J_max (theta/theta_m)
 * (1 - ln(theta/theta_m)) below theta_m (degrees) and J_max above, written
 * as round-half-even(J * 65536) into Jp_out int32[Q*Q] (symmetric, zero
 * diagonal).  The paper gives no law for J; Read and Shockley, Phys. Rev. 78
 * (1950) 275.  euler and Jp_out are both host (on_device = 0) or both device
 * arrays.  Synchronous.  Errors: INVAL (NULL, Q outside [1, 46340], J_max
 * outside [0, 256], theta_m <= 0), NOMEM, DEVICE. */
hmc_status hmc_misorientation_energy(const double *euler, int32_t Q, double J_max, double theta_m_deg,
                                     int32_t on_device, int32_t *Jp_out);

/* Per-site bulk field: Eq. (7) gives each site its own bulk energy b_i;
 * E_site int32[N] (2^-16 units, |E| <= 2^24, host or device per on_device,
 * copied) adds to the grain energies B[q_i].  When a trial at site i is
 * accepted the site's field becomes e_new: with HMC_FIELD_CARRY the field of
 * the neighbour whose spin it adopts (the overtaking grain's dislocation
 * content moves with the boundary, the reading the paper's closing section
 * adopts), with HMC_FIELD_RECRYSTALLISE zero (the swept site is
 * dislocation-free, the alternative it describes).  dE gains
 * e_new - E_site[i]; acceptance uses T(d) for every d > 0.  Needs neighbour
 * trials; not combined with pair bond energies; ensembles do not take such
 * lattices.  The field is checkpointed by hmc_snapshot / hmc_restore.
 * E_site = NULL removes the field.  Synchronous.  Errors: INVAL (sizes,
 * rule, trial mode, pair mode, values), RANGE (J_fx M + 2 max|B| +
 * 2 max|E| >= 2^31), NOMEM, DEVICE. */
enum { HMC_FIELD_CARRY = 0, HMC_FIELD_RECRYSTALLISE = 1 };
hmc_status hmc_set_site_energy(hmc_lattice *L, const int32_t *E_site, uint64_t n_sites, int32_t on_device,
                               int32_t rule);

/* Copy the current per-site field to host int32[N].  Synchronous.
 * Errors: INVAL, STATE (no field set), DEVICE. */
hmc_status hmc_get_site_energy(hmc_lattice *L, int32_t *out, uint64_t n_sites);

/* n_mcs Monte Carlo steps of red/black Metropolis (Sec. 4) at temperature
 * kT (the paper's effective temperature alpha_mc with J = 1), drawing from
 * the Philox stream of `seed`.  Steps are numbered from the lattice's MC
 * counter, which advances by n_mcs.  Asynchronous on the lattice's stream.
 * Errors: INVAL (kT <= 0 or not finite, n_mcs < 0), RANGE (table cap),
 * NOMEM, DEVICE. */
hmc_status hmc_sweep(hmc_lattice *L, float kT, int32_t n_mcs, uint64_t seed);

/* Grain statistics of the current spins (the texture the paper follows over
 * time, Sec. 5): n_grains = number of spin values present; mean area =
 * N / n_grains; frac[b] = sum of the areas of grains with grain_bin[q] == b,
 * divided by N.  grain_bin: int32[Q] host array with values in [-1, n_bins)
 * (-1 = leave the grain out); may be NULL when n_bins == 0.  frac_out:
 * double[n_bins].  Synchronous.  Errors: INVAL, DEVICE. */
hmc_status hmc_texture_stats(hmc_lattice *L, const int32_t *grain_bin, int32_t n_bins,
                             int32_t *n_grains_out, double *mean_area_out, double *frac_out);

/* Area (site count) of every spin value 0..Q-1 into int64[Q].  Synchronous. */
hmc_status hmc_grain_areas(hmc_lattice *L, int64_t *areas_out);

/* For callers that cannot allocate (code under graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the statistics of
 * hmc_texture_stats for n_sites spins in the caller's device buffer
 * dev_spins (spin = HMC_I16 or HMC_I32, values outside [0, n_grains) not
 * counted), with no device or host allocation.  The working memory is a
 * fixed array inside the library, one per device (about 0.5 MiB, held until
 * the process ends), which bounds n_grains <= HMC_STATIC_MAX_GRAINS and
 * n_bins <= HMC_STATIC_MAX_BINS; larger requests fail with HMC_E_INVAL
 * before any device work.  Runs on the current device, on `stream` (NULL:
 * the default stream), which must belong to that device.  grain_bin: host
 * int32[n_grains] in [-1, n_bins) (NULL when n_bins == 0); outputs as
 * hmc_texture_stats.  Synchronous.  Every call on a device uses that
 * device's one array: calls that overlap in time on one device (other
 * threads, other streams) race and must be serialised by the caller.
 * Errors: INVAL (NULL, sizes, not device memory, misaligned), DEVICE. */
#define HMC_STATIC_MAX_GRAINS 65536
#define HMC_STATIC_MAX_BINS 1024
hmc_status hmc_texture_stats_static(const void *dev_spins, int32_t spin, uint64_t n_sites, int32_t n_grains,
                                    const int32_t *grain_bin, int32_t n_bins, void *stream,
                                    int32_t *n_grains_out, double *mean_area_out, double *frac_out);

/* Copy the spins to / from host memory (bytes must equal N * spin size).
 * set_spins rejects values outside [0, Q).  Synchronous. */
hmc_status hmc_get_spins(hmc_lattice *L, void *host_dst, uint64_t bytes);
hmc_status hmc_set_spins(hmc_lattice *L, const void *host_src, uint64_t bytes);

/* Device-side checkpoint: snapshot copies spins and the MC counter into a
 * buffer the lattice owns; restore copies them back.  Asynchronous.
 * restore without a snapshot: STATE. */
hmc_status hmc_snapshot(hmc_lattice *L);
hmc_status hmc_restore(hmc_lattice *L);

/* MC step counter (the second Philox counter word); checkpoint / resume. */
hmc_status hmc_get_mcs(const hmc_lattice *L, uint64_t *mcs);
hmc_status hmc_set_mcs(hmc_lattice *L, uint64_t mcs);

/* Tiling of the sweep kernel: interior tile (tx, ty, tz) and the work fused
 * per launch: mcs_per_launch > 0 MC steps, or mcs_per_launch < 0 for
 * -mcs_per_launch colour passes (launches that cover part of an MC step,
 * useful with 4 or 8 colours).  Zero means "choose automatically".  Each
 * tile side must be an even divisor of the lattice side; the LDS box (tile +
 * a halo of one site per fused colour pass) must fit the kernel's LDS
 * budget; at most 64 passes per launch.  Results do not depend on the
 * tiling.  get_tiling returns the tiling in force as int32[4] with the same
 * sign convention. */
hmc_status hmc_set_tiling(hmc_lattice *L, int32_t tx, int32_t ty, int32_t tz, int32_t mcs_per_launch);
hmc_status hmc_get_tiling(const hmc_lattice *L, int32_t *out4);

/* Which sweep kernel runs the Red/Black passes (Sec. 4).  HMC_KERNEL_AUTO
 * (the default): 16-bit lattices with neighbour trials, one bond energy and
 * grain energies (lattice x side a multiple of 4) run a kernel compiled for
 * their tile where there is one: six-neighbour 64x16x16, 32x32x16,
 * 32x16x16, 16x16x16 or 64x16x8 with one or two colour passes per launch
 * (32x16x16, the default tile of such lattices, 16x16x16 and 64x16x8 run two
 * workgroups per CU); four-neighbour 128x128 with 6 MC steps per launch
 * and 256x128 with 4; eight-neighbour 128x128 and 256x128 with 3 (launches
 * of fewer passes, at the end of a call, take the general kernel);
 * 26-neighbour 32x16x16 with two or four colour passes per launch (two, the
 * default of such lattices when their sides allow the tile); everything else
 * the general tile kernel.  HMC_KERNEL_GENERIC: always the
 * general kernel.  The spins do not depend on the choice.  Errors: INVAL. */
enum { HMC_KERNEL_AUTO = 0, HMC_KERNEL_GENERIC = 1, HMC_KERNEL_COMPILED = 2 };
hmc_status hmc_set_sweep_kernel(hmc_lattice *L, int32_t which);
/* The kernel the next full sweep launch of L will run: HMC_KERNEL_COMPILED
 * (the compiled-tile kernel) or HMC_KERNEL_GENERIC.  Errors: INVAL. */
hmc_status hmc_get_sweep_kernel(const hmc_lattice *L, int32_t *which);

/* Kernel timing with HIP events recorded around every sweep launch on the
 * lattice's stream.  profile_read synchronises, returns the summed kernel
 * time, the number of launches and the site updates they performed since
 * profiling was enabled (or last read), and resets the sums. */
hmc_status hmc_profile(hmc_lattice *L, int32_t enable);
hmc_status hmc_profile_read(hmc_lattice *L, double *kernel_ms, int64_t *launches, int64_t *site_updates);

/* Trials drawn (Philox calls: queued sites, including the redundant halo
 * work of fused steps) by sweep launches made while profiling was enabled,
 * since enabling or the last call; resets the count.  0 if profiling was
 * never enabled.  Synchronous. */
hmc_status hmc_profile_trials(hmc_lattice *L, int64_t *trials);

/* Number of grain-boundary sites of the current spins: sites whose spin is
 * in [0, Q) and differs from at least one of their M neighbours (the sites
 * whose trials can change the state, Sec. 3).  Synchronous. */
hmc_status hmc_boundary_sites(hmc_lattice *L, int64_t *n_out);

/* Wait for all work queued on the lattice's stream. */
hmc_status hmc_synchronize(hmc_lattice *L);

/* The uint32 threshold table of the Metropolis rule (Sec. 3; Red/Black
 * passes of Sec. 4 read it) as the host builds it, without a device:
 * T(d) = min(2^32-1, floor(2^32 exp(-d / (65536 kT)))) for
 * d = J_fx*dn + dB, rows dn = dn_lo..M (dn_lo the smallest dn with a
 * positive d), columns dB = -R..R (R = Bmax - Bmin), entry
 * [(dn - dn_lo) * TW + dB + R], TW = 2R + 1; entries with d <= 0 hold
 * 2^32 - 1 and are never read.  Each row is cut into nb buckets of bw
 * columns; bounds[2k] = T at the bucket's largest d, bounds[2k+1] = T at
 * its smallest positive d, so T over the bucket lies between them (T is
 * non-increasing in d) and a trial whose r1 is outside [lower, upper) needs
 * no table read.  layout6 receives (dn_lo, rows, R, TW, nb, bw); table
 * (rows*TW entries) and bounds (2*rows*nb) may be NULL to query the layout.
 * Errors: INVAL (NULL layout, kT <= 0 or not finite, M not 4/6/8/26,
 * J_fx outside [1, 2^24], Bmin > Bmax, a buffer below its cap), RANGE. */
hmc_status hmc_threshold_table_host(float kT, int32_t M, int32_t J_fx, int32_t Bmin, int32_t Bmax, int32_t *layout6,
                                    uint32_t *table, uint64_t table_cap, uint32_t *bounds, uint64_t bounds_cap);

/* The threshold table a sweep of L at temperature kT reads, copied back
 * from device memory after it is built (or reused) exactly as hmc_sweep
 * builds it.  layout8 receives (kind, dn_lo, rows, R, TW, nb, bw, Dmax):
 * kind 0 is the bucketed table of hmc_threshold_table_host (Dmax = -1);
 * kind 1, used with pair bond energies or a per-site field, holds T(d) for
 * d = 0..Dmax in TW = Dmax + 1 entries (T(0) = 2^32 - 1, d <= 0 accepted
 * before any read) and no bounds.  table and bounds may be NULL.
 * Synchronous.  Errors: INVAL (NULL lattice or layout, kT, a buffer below
 * its cap), RANGE, NOMEM, DEVICE. */
hmc_status hmc_threshold_table(hmc_lattice *L, float kT, int32_t *layout8, uint32_t *table, uint64_t table_cap,
                               uint32_t *bounds, uint64_t bounds_cap);

/* ------------------------------------------------------------ ensembles
 * Many independent lattices (uneven sizes, temperatures and seeds) advanced
 * together: one persistent kernel walks a ragged table of every member's
 * tiles, each launch moves every member k MC steps, and the launch sequence
 * of a call is captured once into a HIP graph and replayed.  Each member's
 * result is exactly what hmc_sweep on that member alone would give (same
 * Philox streams, same table), whatever the ensemble's tiling. */
typedef struct hmc_ensemble_s hmc_ensemble;

/* Borrow n >= 1 lattices that share neighbourhood, spin type and trial mode
 * (sizes, Q, J_fx, energies may differ).  The lattices stay owned by the
 * caller and must outlive the ensemble; free the ensemble first.  Errors:
 * INVAL (NULL, n, mixed kinds, duplicate member), NOMEM, DEVICE. */
hmc_status hmc_ensemble_create(hmc_lattice *const *lats, int32_t n, hmc_ensemble **out);

/* Tile shape and MC steps per launch shared by all members (0 = automatic:
 * autotuned entry if one is loaded, else a default).  Each tile side must
 * divide the matching side of every member. */
hmc_status hmc_ensemble_set_tiling(hmc_ensemble *E, int32_t tx, int32_t ty, int32_t tz, int32_t mcs_per_launch);
hmc_status hmc_ensemble_get_tiling(hmc_ensemble *E, int32_t *out4);

/* n_mcs MC steps on every member; kT[i], seed[i] as in hmc_sweep for member
 * i (host arrays of n entries).  Ordered after all work pending on the
 * members' streams; members' later work waits for it.  Advances every
 * member's MC counter by n_mcs.  Asynchronous. */
hmc_status hmc_ensemble_sweep(hmc_ensemble *E, const float *kT, const uint64_t *seed, int32_t n_mcs);

/* Wait for the ensemble's stream. */
hmc_status hmc_ensemble_synchronize(hmc_ensemble *E);

/* Kernel timing of ensemble sweeps: while enabled, HIP events are recorded
 * on the ensemble's stream around each graph replay (outside the graph), so
 * the time covers the replay's kernels and the gaps between them.
 * profile_read synchronises, returns the summed time, the kernel launches
 * and the site updates (sum over members of N * n_mcs) since enabling or the
 * last read, and resets the sums.  Errors: INVAL (NULL). */
hmc_status hmc_ensemble_profile(hmc_ensemble *E, int32_t enable);
hmc_status hmc_ensemble_profile_read(hmc_ensemble *E, double *kernel_ms, int64_t *launches, int64_t *site_updates);

/* Time candidate tilings on the ensemble's own members (their spins and MC
 * counters are restored afterwards), keep the fastest and return it in
 * best_out4 (tx, ty, tz, k).  n_mcs per candidate; kT/seed as in
 * hmc_ensemble_sweep.  Synchronous. */
hmc_status hmc_ensemble_autotune(hmc_ensemble *E, const float *kT, const uint64_t *seed, int32_t n_mcs,
                                 int32_t *best_out4);

/* Release the ensemble (not its members).  NULL is a no-op. */
hmc_status hmc_ensemble_free(hmc_ensemble *E);

/* ---------------------------------------------------------- n-fold way
 * The rejection-free alternative to red/black updating named in Sec. 1 and
 * Sec. 4 (Bortz, Kalos, Lebowitz 1975; Hassold and Holm 1993): the single-
 * site Metropolis process of Sec. 3 in continuous time.  Every site attempts
 * at rate one per MC step; an attempt proposes one of S slots (NEIGHBOUR:
 * the M neighbour spins, S = M; UNIFORM: q+1..q+Q-1 mod Q, S = Q-1) and is
 * accepted with the sweep's rule.  Slot k of site i fires at rate
 * w_ik / (S 2^32) per MC step, w_ik = 2^32 if d <= 0, T(d) if d > 0 (T and d
 * as above; a neighbour slot holding the site's own spin has weight 0), W is
 * the sum of all weights, and events happen one at a time:
 *   - event n draws Philox4x32-10 blocks with key (lo32(seed), hi32(seed))
 *     and counter (lo32(n), hi32(n), 0x4E464F57, j), j = 0, 1, ..., read
 *     word by word;
 *   - words 0, 1 give u = w0 + 2^32 w1 and the rank r = floor(u W / 2^64);
 *     the event is the site whose cumulative weight (sites in index order)
 *     first exceeds r, then, with r reduced by the sites before it, the slot
 *     whose cumulative weight first exceeds the rest;
 *   - the following words give E, an Exp(1) variate in 32.32 fixed point by
 *     von Neumann's comparison method (a trial takes u0 and the length n of
 *     the strictly decreasing run u0 > u1 > ... it starts, the word ending
 *     the run used up; odd n returns K + u0/2^32, even n adds one to K;
 *     runs cut at 64 words, K at 64);
 *   - the event happens at t_last + (E S) / W (double, one rounding per
 *     operation); if that is beyond the end of the call it is not executed
 *     and the next call draws it again from the same counter, so splitting
 *     a run between calls changes nothing.  A lattice with W = 0 has no event.
 * Each lattice carries its own clock (t_now, t_last, n_events), starting at
 * zero, separate from the MC-step counter of hmc_sweep; snapshots include it.
 * Spin values outside [0, Q) (a wrapped buffer may hold them) are inert, as
 * in the sweep: such a site has weight 0 and such a neighbour is never
 * proposed and, with a pair table, bonds with nothing.
 * The lattice's spins live in LDS during a call (N * spin size + N/8 + 4 Q
 * bytes must fit the device's LDS, 160 KiB on MI355X: up to about 75 000
 * int16 or 38 000 int32 sites, else HMC_E_RANGE); per-site fields are not
 * supported (HMC_E_STATE); the UNIFORM mode needs uniform bonds and Q <= 65.
 * Calls are synchronous. */

/* Advance one lattice by mcs MC steps of continuous time. */
hmc_status hmc_nfold(hmc_lattice *L, float kT, double mcs, uint64_t seed);

/* Advance n distinct lattices by mcs MC steps each in one launch per event
 * budget, one wave per lattice; kT[n], seed[n] per lattice.  The lattices
 * share device, neighbourhood, spin type, trial mode and bond model (uniform
 * or pair table); sizes, grain counts and energies may differ.  The result
 * of each lattice equals its own hmc_nfold run. */
hmc_status hmc_nfold_batch(hmc_lattice *const *lats, int32_t n, const float *kT, double mcs,
                           const uint64_t *seed);

/* Clock of the n-fold way: the time the lattice has been advanced to, the
 * time of its last event and the number of events so far. */
hmc_status hmc_nfold_clock(const hmc_lattice *L, double *t_now, double *t_last, uint64_t *n_events);
/* Set the clock (a restart from saved spins); t_last <= t_now, both finite. */
hmc_status hmc_nfold_set_clock(hmc_lattice *L, double t_now, double t_last, uint64_t n_events);

/* Self-test of the event loop's waiting-time variate: out[c] = E of event
 * n0 + c under `seed` (drawn after its two selection words, 32.32 fixed
 * point), computed on the current device with the event kernel's own code.
 * The kernel measures a decreasing run in one step when it ends inside the
 * first `window` words of the event's stream and walks it word by word
 * otherwise; window 64 is the event loop's, 4, 7 and 16 send more runs down
 * the word-by-word path.  Every window gives the same values.  out: host,
 * count entries (count <= 2^26, else HMC_E_RANGE); any other window is
 * HMC_E_INVAL.  Synchronous. */
hmc_status hmc_nfold_exponentials(uint64_t seed, uint64_t n0, int64_t count, int32_t window, uint64_t *out);

/* ------------------------------------------------------------ autotuner
 * Time candidate tilings (tile sides x MC steps per launch) of hmc_sweep on
 * a scratch lattice with this descriptor, n_grains Voronoi grains and zero
 * bulk energy at temperature kT, n_mcs steps per candidate.  The fastest is
 * returned (best_out4 = tx, ty, tz, k; us_per_mcs_out its time per MC step),
 * registered for lattices of this shape created afterwards in this process,
 * and appended as one JSON line to cache_path when it is not NULL.
 * Synchronous.  Errors: INVAL, NOMEM, DEVICE, and file errors as INVAL. */
hmc_status hmc_autotune(const hmc_lattice_desc *desc, int32_t n_grains, float kT, int32_t n_mcs,
                        const char *cache_path, int32_t *best_out4, double *us_per_mcs_out);

/* Load tilings from a cache written by hmc_autotune (later lines win).
 * Returns the number of entries read in *n_loaded. */
hmc_status hmc_tuning_load(const char *cache_path, int32_t *n_loaded);

/* ------------------------------------------- stored energy: solver and network
 * The bulk energy of a grain is its stored dislocation energy (Sec. 3, Eq. (4):
 * E_rho = rho G b^2 / 2 with rho = (2 sigma_f / (G b))^2 = 2 sigma_f^2 / G),
 * produced by the Monte Carlo crystal-plasticity update of Sec. 2.  A small
 * network trained on the solver's output can stand in for it. */

/* Monte Carlo crystal plasticity (Sec. 2, Eqs. (1)-(2), Table 1 nickel
 * constants) for n crystals, FP64 on the GPU, one thread per crystal.
 * euler: n x 3 Bunge angles (phi1, Phi, phi2) of the passive sample->crystal
 * rotation; eps: n x 6 total strain from the virgin crystal in the sample
 * frame (e11, e22, e33, e23, e13, e12; tensor shear components), applied in
 * K = ceil(max|e_ij| / 1e-5) <= 200 sub-steps.  One slip system per
 * sub-step among those with |tau| > tau_c, chosen by Eq. (2) with
 * p ~ exp(-1000/MPa * E_a) and R from Philox(key = seed,
 * counter = (sample0 + i, step, 0, 0x4D435053)); Voce hardening
 * (tau0 8, tau_s 122, h0 440 MPa).  Outputs E_out[i] = 2 tau_c^2 / G in MPa
 * (G = (C11 - C12 + 3 C44) / 5) and optionally tau_c.  on_device: 1 if all
 * four arrays are device pointers, 0 for host arrays.  Synchronous.
 * Errors: INVAL (NULL, n < 0, n >= 2^31, non-finite strain), NOMEM, DEVICE. */
hmc_status hmc_mcp_solve(const double *euler, const double *eps, int64_t n, uint64_t seed, uint64_t sample0,
                         int32_t on_device, double *E_out, double *tauc_out);

/* 9-64-64-1 tanh network predicting E_rho from (Bunge angles, strain).
 * Features: the Rodrigues vector of the orientation's equivalent under the
 * 24 cubic crystal rotations with the smallest rotation angle (the cubic
 * fundamental zone), over sqrt 2 - 1, then e_ij / 2e-3; so orientations
 * that differ by a crystal symmetry get the same prediction.  Target
 * standardised by the training mean and standard deviation (kept in the
 * handle).  Parameters (4865 floats): W1[64][9], b1[64], W2[64][64], b2[64],
 * w3[64], b3.  create: Xavier-uniform weights from Philox(seed), zero
 * biases. */
typedef struct hmc_mlp_s hmc_mlp;
hmc_status hmc_mlp_create(uint64_t seed, hmc_mlp **out);
hmc_status hmc_mlp_free(hmc_mlp *M);

/* Host copies of the parameters (float[4865]) and of the target
 * normalisation (double[2] = mean, std; may be NULL).  set_params resets
 * Adam's moments and step. */
hmc_status hmc_mlp_get_params(hmc_mlp *M, float *host_dst, double *norm_out);
hmc_status hmc_mlp_set_params(hmc_mlp *M, const float *host_src, const double *norm);

/* Train on n samples (euler n x 3, eps n x 6, E n in MPa; host or device
 * per on_device) for `epochs` passes in mini-batches of `batch` (a multiple
 * of 32), shuffled each epoch with Philox(seed); mean squared error on the
 * standardised target; Adam with learning rate lr decaying on a cosine to
 * lr/10.  final_loss (may be NULL): mean batch loss of the last epoch.
 * Synchronous.  Errors: INVAL, NOMEM, DEVICE. */
hmc_status hmc_mlp_train(hmc_mlp *M, const double *euler, const double *eps, const double *E, int64_t n,
                         int32_t on_device, int32_t epochs, int32_t batch, float lr, uint64_t seed,
                         float *final_loss);

/* Predicted E_rho (MPa) for n crystals; arrays host or device per
 * on_device.  Synchronous. */
hmc_status hmc_mlp_predict(hmc_mlp *M, const double *euler, const double *eps, int64_t n, int32_t on_device,
                           double *E_out);

/* Inference on device memory, asynchronous on `stream` (NULL: the
 * handle's own stream; another stream is first ordered after the handle's
 * pending work).  X_dev: n x 9 scaled features (float, row-major); y_dev:
 * n standardised outputs (float; E_rho = y * std + mean with the handle's
 * normalisation).  Synchronise `stream` before freeing the handle.
 * Errors: INVAL, DEVICE. */
hmc_status hmc_mlp_infer(hmc_mlp *M, const float *X_dev, float *y_dev, int64_t n, void *stream);

/* Standardised outputs for already-scaled features X (n x 9, host). */
hmc_status hmc_mlp_forward(hmc_mlp *M, const float *X, int32_t n, float *y_out);

/* Mean squared error over n samples (n a multiple of 32) of scaled features
 * X (n x 9) and standardised targets t, and its gradient (float[4865]), by
 * the training kernels; parameters unchanged.  Host arrays.  Synchronous. */
hmc_status hmc_mlp_loss_grad(hmc_mlp *M, const float *X, const float *t, int32_t n, float *loss_out,
                             float *grad_out);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with a host gradient. */
hmc_status hmc_mlp_adam_step(hmc_mlp *M, const float *grad, float lr);

/* Bulk energies of a lattice's grains from their stored energy under one
 * macroscopic strain eps6 (6 components, sample frame): B[q] =
 * round-half-even(E_rho[q] * E_scale * 65536), then as hmc_set_grain_energy.
 * euler: host Q x 3 orientations of the grains.  mode 0: the network, with
 * an audit of n_audit grains (drawn with Philox(seed)) against the solver,
 * each solved with its own random stream (the value the fallback would give
 * it); if the strain leaves the training box (|e_ij| > 2e-3), any prediction
 * is not finite, or the largest relative audit error exceeds audit_tol,
 * every grain is solved instead (*used_solver = 1).  The solver keys grain q
 * by sample index q (hmc_mcp_solve with sample0 = 0).  mode 1: the solver for every
 * grain (the method without the network; M may be NULL).  *audit_err gets
 * the largest relative audit error (0 if no audit ran); B_out (may be NULL)
 * receives the int32[Q] energies set.  Synchronous.
 * Errors: INVAL, RANGE (energy range), NOMEM, DEVICE. */
hmc_status hmc_surrogate_update(hmc_lattice *L, hmc_mlp *M, const double *euler, const double *eps6, double E_scale,
                                int32_t mode, int32_t n_audit, double audit_tol, uint64_t seed,
                                int32_t *used_solver, double *audit_err, int32_t *B_out);

#ifdef __cplusplus
}
#endif

#endif /* HMC_H */
