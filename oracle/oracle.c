/*
 * oracle.c -- plain, slow, single-purpose CPU reference for the red/black
 * Q-state Potts sweep with a per-grain bulk energy.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file.  Only the test-suite, the package smoke check and
 * the CPU-baseline leg of the benchmark load the shared object built from it.
 * It shares no source with the HIP library: its own Philox, its own
 * neighbour tables, its own acceptance rule written out from the definitions.
 *
 * Paper: L. Zhang, R. Dingreville, T. Bartel, M. T. Lusk, "Hybrid Monte
 * Carlo simulation of stress-induced texture evolution with inelastic
 * effects" (arXiv:1007.3509).
 *
 *   Sec. 3, Eq. (7)  Potts Hamiltonian: bond term over the M neighbours of
 *                    every site plus a bulk term b_i.
 *   Sec. 3           acceptance of a trial flip from the change of H.
 *   Sec. 4           Red/Black updating: the lattice is a checkerboard, each
 *                    MC step is split into half steps and no state changes
 *                    until a half step has finished.
 *   Sec. 6           the swept site takes the overtaking grain's dislocation
 *                    energy, so the bulk term is a property of the spin:
 *                    b_i = b(q_i).
 *
 * Readings where the paper is silent or garbled (each is listed in the
 * design notes of the repository):
 *   - Eq. (7) prints J*delta(q_i,q_n); grain growth needs the unlike-bond
 *     count, so the bond energy is J*(1 - delta), each bond counted once.
 *   - Metropolis acceptance min(1, exp(-dE/kT)), dE <= 0 always accepted.
 *   - fixed point: J_fx = 65536*J, B[q] = b(q)*65536 as int32.
 *   - acceptance is integer: accept iff d <= 0 or r1 < T(d), with
 *     T(d) = min(2^32-1, floor(2^32 * exp(-d / (65536 kT)))) evaluated in
 *     double with the C library exp.
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *     key = (lo32(seed), hi32(seed)), counter = (site, mcs, colour, 0);
 *     word 0 picks the trial spin, word 1 decides acceptance.
 *   - trial spin: the spin of neighbour k = floor(r0*M / 2^32) (production),
 *     or, in a symmetric test mode, q' = (q + 1 + floor(r0*(Q-1)/2^32)) mod Q.
 *   - colours: VN4 (x+y)&1, VN6 (x+y+z)&1, Moore8 (x&1)|(y&1)<<1,
 *     Moore26 (x&1)|(y&1)<<1|(z&1)<<2; passes run c = 0..C-1 every MC step.
 *   - spins are numbered 0..Q-1; the lattice is periodic, x fastest.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

enum { ORC_VN4 = 0, ORC_MOORE8 = 1, ORC_VN6 = 2, ORC_MOORE26 = 3 };
enum { ORC_PROP_NEIGHBOUR = 0, ORC_PROP_UNIFORM = 1 };

/* ---------------------------------------------------------------- Philox */

/* Philox4x32 with 10 rounds, written from the description in Salmon et al.
 * (SC'11, Sec. 3): each round multiplies counter words 0 and 2 by two fixed
 * odd constants, keeps the 64-bit products, and recombines high halves with
 * the other two words and the round key; the key is bumped by two Weyl
 * constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi_a = (uint32_t)(prod_a >> 32), lo_a = (uint32_t)prod_a;
        uint32_t hi_b = (uint32_t)(prod_b >> 32), lo_b = (uint32_t)prod_b;
        uint32_t y0 = hi_b ^ x1 ^ k0;
        uint32_t y1 = lo_b;
        uint32_t y2 = hi_a ^ x3 ^ k1;
        uint32_t y3 = lo_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Vectorised helper for the tests: n counters (4 words each) -> n outputs. */
void orc_philox_many(const uint32_t *ctrs, int64_t n, const uint32_t key[2], uint32_t *outs)
{
    int64_t i;
    for (i = 0; i < n; ++i) orc_philox4x32_10(ctrs + 4 * i, key, outs + 4 * i);
}

/* ------------------------------------------------------------- geometry */

int orc_num_neighbours(int nbr)
{
    switch (nbr) {
    case ORC_VN4: return 4;
    case ORC_MOORE8: return 8;
    case ORC_VN6: return 6;
    case ORC_MOORE26: return 26;
    default: return -1;
    }
}

int orc_num_colours(int nbr)
{
    switch (nbr) {
    case ORC_VN4: return 2;
    case ORC_MOORE8: return 4;
    case ORC_VN6: return 2;
    case ORC_MOORE26: return 8;
    default: return -1;
    }
}

/* Neighbour offsets in the fixed order used to pick the trial spin. */
static int orc_offsets(int nbr, int off[26][3])
{
    int n = 0, dx, dy, dz;
    switch (nbr) {
    case ORC_VN4: {
        static const int t[4][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}};
        memcpy(off, t, sizeof t);
        return 4;
    }
    case ORC_MOORE8: {
        static const int t[8][3] = {{1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
        memcpy(off, t, sizeof t);
        return 8;
    }
    case ORC_VN6: {
        static const int t[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                                    {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
        memcpy(off, t, sizeof t);
        return 6;
    }
    case ORC_MOORE26:
        for (dz = -1; dz <= 1; ++dz)
            for (dy = -1; dy <= 1; ++dy)
                for (dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0 && dz == 0) continue;
                    off[n][0] = dx; off[n][1] = dy; off[n][2] = dz;
                    ++n;
                }
        return 26;
    default:
        return -1;
    }
}

static int orc_colour(int nbr, int64_t x, int64_t y, int64_t z)
{
    switch (nbr) {
    case ORC_VN4: return (int)((x + y) & 1);
    case ORC_VN6: return (int)((x + y + z) & 1);
    case ORC_MOORE8: return (int)((x & 1) | ((y & 1) << 1));
    case ORC_MOORE26: return (int)((x & 1) | ((y & 1) << 1) | ((z & 1) << 2));
    default: return -1;
    }
}

static int64_t orc_wrap(int64_t a, int64_t L)
{
    a %= L;
    if (a < 0) a += L;
    return a;
}

/* Linear index of the k-th neighbour of site (x,y,z) on the periodic box. */
static int64_t orc_neighbour_index(const int64_t dims[3], int off[26][3], int k,
                                   int64_t x, int64_t y, int64_t z)
{
    int64_t nx = orc_wrap(x + off[k][0], dims[0]);
    int64_t ny = orc_wrap(y + off[k][1], dims[1]);
    int64_t nz = orc_wrap(z + off[k][2], dims[2]);
    return nx + dims[0] * (ny + dims[1] * nz);
}

/* Exposed for tests: the n-th neighbour index of every neighbour of site i. */
int orc_neighbours_of(int nbr, const int32_t dims_in[3], int64_t i, int64_t *out)
{
    int off[26][3];
    int64_t dims[3] = {dims_in[0], dims_in[1], dims_in[2]};
    int M = orc_offsets(nbr, off), k;
    int64_t x = i % dims[0], y = (i / dims[0]) % dims[1], z = i / (dims[0] * dims[1]);
    for (k = 0; k < M; ++k) out[k] = orc_neighbour_index(dims, off, k, x, y, z);
    return M;
}

int orc_colour_of(int nbr, const int32_t dims_in[3], int64_t i)
{
    int64_t x = i % dims_in[0], y = (i / dims_in[0]) % dims_in[1];
    int64_t z = i / ((int64_t)dims_in[0] * dims_in[1]);
    return orc_colour(nbr, x, y, z);
}

/* ------------------------------------------------------ energy / accept */

/* T(d) for d > 0: the acceptance probability exp(-dE/kT) scaled to 2^32 and
 * floored, with dE = d / 65536 (fixed point) and the Metropolis rule. */
uint32_t orc_threshold(int64_t d, float kT)
{
    double x = (double)d / (65536.0 * (double)kT);
    double p = exp(-x);
    double v = ldexp(p, 32);
    if (v >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)floor(v);
}

/* T(d) for many d (d <= 0 gives 2^32 - 1: always accepted). */
void orc_threshold_many(const int64_t *d, int64_t n, float kT, uint32_t *out)
{
    int64_t i;
    for (i = 0; i < n; ++i) out[i] = d[i] > 0 ? orc_threshold(d[i], kT) : 0xFFFFFFFFu;
}

/* Change of Eq. (7) (read with J*(1-delta), each bond once) when site i
 * goes from its spin q to q_new, in 2^-16 units:
 *   dE = J * (#unlike bonds after - #unlike bonds before) + b(q_new) - b(q)
 *      = J * (c(q) - c(q_new)) + B[q_new] - B[q],
 * where c(s) is the number of the M neighbours of i holding spin s. */
int64_t orc_delta_energy(const int32_t *spins, int nbr, const int32_t dims_in[3],
                         int32_t J_fx, const int32_t *B, int64_t i, int32_t q_new)
{
    int off[26][3];
    int64_t dims[3] = {dims_in[0], dims_in[1], dims_in[2]};
    int M = orc_offsets(nbr, off), k;
    int64_t x = i % dims[0], y = (i / dims[0]) % dims[1], z = i / (dims[0] * dims[1]);
    int32_t q = spins[i];
    int64_t unlike_before = 0, unlike_after = 0;
    for (k = 0; k < M; ++k) {
        int32_t s = spins[orc_neighbour_index(dims, off, k, x, y, z)];
        if (s != q) unlike_before += 1;
        if (s != q_new) unlike_after += 1;
    }
    return (int64_t)J_fx * (unlike_after - unlike_before) + (int64_t)B[q_new] - (int64_t)B[q];
}

/* The same change when every bond carries its own energy (the paper's
 * J_{q_i,q_n} of Eq. (7)): with Jp[a*Q + b] the energy of an unlike bond
 * between spins a and b (symmetric, zero diagonal, 2^-16 units),
 *   dE = sum over the M neighbours s_k of (Jp[q_new][s_k] - Jp[q][s_k])
 *        + B[q_new] - B[q];
 * a like bond costs nothing, which the zero diagonal expresses. */
int64_t orc_delta_energy_pair(const int32_t *spins, int nbr, const int32_t dims_in[3],
                              const int32_t *Jp, int32_t Q, const int32_t *B, int64_t i, int32_t q_new)
{
    int off[26][3];
    int64_t dims[3] = {dims_in[0], dims_in[1], dims_in[2]};
    int M = orc_offsets(nbr, off), k;
    int64_t x = i % dims[0], y = (i / dims[0]) % dims[1], z = i / (dims[0] * dims[1]);
    int32_t q = spins[i];
    int64_t after = 0, before = 0;
    for (k = 0; k < M; ++k) {
        int32_t s = spins[orc_neighbour_index(dims, off, k, x, y, z)];
        if (s < 0 || s >= Q) continue;   /* a value outside [0, Q) bonds with nothing */
        after += Jp[(int64_t)q_new * Q + s];
        before += Jp[(int64_t)q * Q + s];
    }
    return after - before + (int64_t)B[q_new] - (int64_t)B[q];
}

/* ----------------------------------------------------------------- sweep */

/* n_mcs Monte Carlo steps of red/black Metropolis on a periodic lattice.
 *
 * spins   : int32[N], x fastest, values in [0, Q) (others are inert, below);
 *           updated in place.
 * dims    : (Lx, Ly, Lz); Lz = 1 for the 2D neighbourhoods.  Every side even.
 * B       : int32[Q], bulk energy per spin value in 2^-16 units.
 * mcs0    : absolute index of the first step (part of the RNG counter).
 * threads : OpenMP threads over the sites of one half step (any value gives
 *           the same result: sites of one colour share no bond and every
 *           trial reads the state as it was when the half step began).
 *
 * A value outside [0, Q) (a caller's buffer may hold one; it names no grain)
 * is inert: such a site never changes, a neighbour holding one is never
 * proposed, and its bond contributes the same before and after a trial --
 * unlike both q and q' under J(1 - delta), nothing with a pair table -- so
 * it drops out of the energy change.
 *
 * Returns 0, or -1 on bad arguments, -2 if an energy change leaves int32. */
/* Per-site bulk field (Eq. (7)'s b_i varying inside a grain): E_site[i] in
 * 2^-16 units adds to the grain's B[q_i].  When site i is swept, its field
 * becomes e_new: with ORC_FIELD_CARRY the value of the neighbour whose spin
 * it adopts (the overtaking grain's dislocation content is carried into the
 * swept site, the paper's closing discussion), with ORC_FIELD_RECRYSTALLISE
 * zero (a dislocation-free, recrystallised site). */
enum { ORC_FIELD_CARRY = 0, ORC_FIELD_RECRYSTALLISE = 1 };

static int sweep_impl(int32_t *spins, int nbr, int proposal, const int32_t dims_in[3],
                      int32_t J_fx, const int32_t *Jp, const int32_t *B, int32_t Q, float kT,
                      uint64_t mcs0, int32_t n_mcs, uint64_t seed, int threads,
                      int32_t *E_site, int rule)
{
    int off[26][3];
    int M = orc_offsets(nbr, off);
    int C = orc_num_colours(nbr);
    int64_t dims[3] = {dims_in[0], dims_in[1], dims_in[2]};
    int64_t N = dims[0] * dims[1] * dims[2];
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    int32_t *before, *before_e = NULL;
    int overflow = 0;
    int32_t step;
    int colour;
    if (M < 0 || n_mcs < 0 || Q < 1 || !(kT > 0.0f)) return -1;
    if (N <= 0) return -1;
    if (n_mcs == 0) return 0;
    if (E_site && proposal != ORC_PROP_NEIGHBOUR) return -1;   /* the carry rule needs a proposing neighbour */
    before = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    if (!before) return -1;
    if (E_site) {
        before_e = (int32_t *)malloc((size_t)N * sizeof(int32_t));
        if (!before_e) { free(before); return -1; }
    }
    if (threads < 1) threads = 1;

    for (step = 0; step < n_mcs; ++step) {
        uint32_t t = (uint32_t)(mcs0 + (uint64_t)step);
        for (colour = 0; colour < C; ++colour) {
            int64_t i;
            /* Half step: every trial sees the state at the start of the
             * half step; accepted flips land in `spins` only. */
            memcpy(before, spins, (size_t)N * sizeof(int32_t));
            if (E_site) memcpy(before_e, E_site, (size_t)N * sizeof(int32_t));
#pragma omp parallel for num_threads(threads) schedule(static) reduction(| : overflow)
            for (i = 0; i < N; ++i) {
                int64_t x = i % dims[0], y = (i / dims[0]) % dims[1];
                int64_t z = i / (dims[0] * dims[1]);
                uint32_t ctr[4], r[4];
                int32_t q, q_new, e_new = 0;
                int64_t d;
                if (orc_colour(nbr, x, y, z) != colour) continue;
                q = before[i];
                if (q < 0 || q >= Q) continue;   /* inert: never changes */
                ctr[0] = (uint32_t)i; ctr[1] = t; ctr[2] = (uint32_t)colour; ctr[3] = 0u;
                orc_philox4x32_10(ctr, key, r);
                if (proposal == ORC_PROP_NEIGHBOUR) {
                    int k = (int)(((uint64_t)r[0] * (uint64_t)M) >> 32);
                    int64_t j = orc_neighbour_index(dims, off, k, x, y, z);
                    q_new = before[j];
                    if (E_site) e_new = rule == ORC_FIELD_CARRY ? before_e[j] : 0;
                } else {
                    uint32_t s = (uint32_t)(((uint64_t)r[0] * (uint64_t)(Q - 1)) >> 32);
                    q_new = (int32_t)(((int64_t)q + 1 + (int64_t)s) % Q);
                }
                if (q_new == q || q_new < 0 || q_new >= Q) continue;   /* no change, or an inert value */
                d = Jp ? orc_delta_energy_pair(before, nbr, dims_in, Jp, Q, B, i, q_new)
                       : orc_delta_energy(before, nbr, dims_in, J_fx, B, i, q_new);
                if (E_site) d += (int64_t)e_new - (int64_t)before_e[i];
                if (d > INT32_MAX || d < INT32_MIN) { overflow = 1; continue; }
                if (d <= 0 || r[1] < orc_threshold(d, kT)) {
                    spins[i] = q_new;
                    if (E_site) E_site[i] = e_new;
                }
            }
        }
    }
    free(before);
    free(before_e);
    return overflow ? -2 : 0;
}

int orc_sweep(int32_t *spins, int nbr, int proposal, const int32_t dims_in[3],
              int32_t J_fx, const int32_t *B, int32_t Q, float kT,
              uint64_t mcs0, int32_t n_mcs, uint64_t seed, int threads)
{
    return sweep_impl(spins, nbr, proposal, dims_in, J_fx, NULL, B, Q, kT, mcs0, n_mcs, seed, threads, NULL, 0);
}

/* As orc_sweep with a per-site bulk field E_site int32[N] (updated in place)
 * and the rule that sets the field of a swept site (ORC_FIELD_CARRY or
 * ORC_FIELD_RECRYSTALLISE); neighbour trials only. */
int orc_sweep_field(int32_t *spins, int32_t *E_site, int rule, int nbr, const int32_t dims_in[3],
                    int32_t J_fx, const int32_t *B, int32_t Q, float kT,
                    uint64_t mcs0, int32_t n_mcs, uint64_t seed, int threads)
{
    if (!E_site || (rule != ORC_FIELD_CARRY && rule != ORC_FIELD_RECRYSTALLISE)) return -1;
    return sweep_impl(spins, nbr, ORC_PROP_NEIGHBOUR, dims_in, J_fx, NULL, B, Q, kT, mcs0, n_mcs, seed, threads,
                      E_site, rule);
}

/* As orc_sweep with a bond energy per pair of spins: Jp int32[Q*Q],
 * symmetric, zero diagonal, 2^-16 units. */
int orc_sweep_pair(int32_t *spins, int nbr, int proposal, const int32_t dims_in[3],
                   const int32_t *Jp, const int32_t *B, int32_t Q, float kT,
                   uint64_t mcs0, int32_t n_mcs, uint64_t seed, int threads)
{
    if (!Jp) return -1;
    return sweep_impl(spins, nbr, proposal, dims_in, 0, Jp, B, Q, kT, mcs0, n_mcs, seed, threads, NULL, 0);
}

/* -------------------------------------------------------------- Voronoi */

/* Seed point g of the initial microstructure: Philox with
 * counter (g, 0, 0, 0x564F524E) under key = voronoi seed; word k gives the
 * fixed-point coordinate floor(r_k * (256*L_k) / 2^32), a site sitting at
 * 256*x.  The paper does not state the initial microstructure; a seeded
 * Voronoi tessellation is the reading used. */
void orc_voronoi_points(int ndim, const int32_t dims[3], int32_t G, uint64_t vseed,
                        int64_t *pts /* G*3 */)
{
    uint32_t key[2] = {(uint32_t)(vseed & 0xFFFFFFFFu), (uint32_t)(vseed >> 32)};
    int32_t g;
    int k;
    for (g = 0; g < G; ++g) {
        uint32_t ctr[4] = {(uint32_t)g, 0u, 0u, 0x564F524Eu}, r[4];
        orc_philox4x32_10(ctr, key, r);
        for (k = 0; k < 3; ++k) {
            if (k < ndim)
                pts[3 * g + k] = (int64_t)(((uint64_t)r[k] * (uint64_t)((int64_t)dims[k] * 256)) >> 32);
            else
                pts[3 * g + k] = 0;
        }
    }
}

/* Periodic squared distance between a site and a point, 1/256-site units. */
static int64_t orc_pdist2(int ndim, const int64_t pos[3], const int64_t *pt, const int32_t dims[3])
{
    int64_t s = 0;
    int k;
    for (k = 0; k < ndim; ++k) {
        int64_t span = (int64_t)dims[k] * 256;
        int64_t a = pos[k] - pt[k];
        if (a < 0) a = -a;
        if (span - a < a) a = span - a;
        s += a * a;
    }
    return s;
}

/* Brute force: every site takes the index of its nearest seed point,
 * ties going to the lower index.  O(N*G); for small lattices. */
int orc_voronoi_brute(int ndim, const int32_t dims[3], int32_t G, uint64_t vseed, int32_t *spins)
{
    int64_t N = (int64_t)dims[0] * dims[1] * (ndim == 3 ? dims[2] : 1), i;
    int64_t *pts = (int64_t *)malloc((size_t)G * 3 * sizeof(int64_t));
    if (!pts || G < 1) { free(pts); return -1; }
    orc_voronoi_points(ndim, dims, G, vseed, pts);
    for (i = 0; i < N; ++i) {
        int64_t pos[3] = {256 * (i % dims[0]), 256 * ((i / dims[0]) % dims[1]),
                          256 * (i / ((int64_t)dims[0] * dims[1]))};
        int64_t best = INT64_MAX;
        int32_t bg = 0, g;
        for (g = 0; g < G; ++g) {
            int64_t d2 = orc_pdist2(ndim, pos, pts + 3 * g, dims);
            if (d2 < best) { best = d2; bg = g; }
        }
        spins[i] = bg;
    }
    free(pts);
    return 0;
}

/* The same labelling through a uniform bucket grid: cells are searched in
 * growing Chebyshev rings around the site's cell until no unvisited cell can
 * hold a point as close as the best one found.  A point in ring r+1 or
 * further lies at least r cell widths away along one axis, so the search
 * stops once best < (r * w_min)^2.  Equal distances keep the lower index, and
 * a cell visited twice (small grids, wrap-around) cannot change the winner. */
int orc_voronoi_grid(int ndim, const int32_t dims[3], int32_t G, uint64_t vseed, int32_t *spins,
                     int threads)
{
    int64_t N = (int64_t)dims[0] * dims[1] * (ndim == 3 ? dims[2] : 1);
    int64_t *pts, i;
    int64_t nc[3] = {1, 1, 1}, ncell, c;
    int64_t *cell_start, *cell_items, *fill;
    double w_min = 1e300;
    int k;
    if (G < 1 || (ndim != 2 && ndim != 3)) return -1;
    pts = (int64_t *)malloc((size_t)G * 3 * sizeof(int64_t));
    if (!pts) return -1;
    orc_voronoi_points(ndim, dims, G, vseed, pts);
    {
        /* about one point per cell */
        double per_axis = pow((double)G, 1.0 / ndim);
        for (k = 0; k < ndim; ++k) {
            double frac = (double)dims[k] / pow((double)N, 1.0 / ndim);
            int64_t n = (int64_t)floor(per_axis * frac);
            if (n < 1) n = 1;
            if (n > dims[k]) n = dims[k];
            nc[k] = n;
            if ((double)dims[k] * 256.0 / (double)n < w_min) w_min = (double)dims[k] * 256.0 / (double)n;
        }
    }
    ncell = nc[0] * nc[1] * nc[2];
    cell_start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    cell_items = (int64_t *)malloc((size_t)G * sizeof(int64_t));
    fill = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
    if (!cell_start || !cell_items || !fill) { free(pts); free(cell_start); free(cell_items); free(fill); return -1; }
    {
        int32_t g;
        int64_t *cell_of = (int64_t *)malloc((size_t)G * sizeof(int64_t));
        for (g = 0; g < G; ++g) {
            int64_t cc[3] = {0, 0, 0};
            for (k = 0; k < ndim; ++k) cc[k] = pts[3 * g + k] * nc[k] / ((int64_t)dims[k] * 256);
            cell_of[g] = cc[0] + nc[0] * (cc[1] + nc[1] * cc[2]);
            cell_start[cell_of[g] + 1] += 1;
        }
        for (c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
        for (g = 0; g < G; ++g) {   /* ascending g inside each cell */
            int64_t cc = cell_of[g];
            cell_items[cell_start[cc] + fill[cc]++] = g;
        }
        free(cell_of);
    }
#pragma omp parallel for num_threads(threads < 1 ? 1 : threads) schedule(dynamic, 1024)
    for (i = 0; i < N; ++i) {
        int64_t pos[3] = {256 * (i % dims[0]), 256 * ((i / dims[0]) % dims[1]),
                          256 * (i / ((int64_t)dims[0] * dims[1]))};
        int64_t home[3] = {0, 0, 0};
        int64_t best = INT64_MAX;
        int32_t bg = -1;
        int64_t r;
        int kk;
        for (kk = 0; kk < ndim; ++kk) home[kk] = (pos[kk] / 256) * nc[kk] / dims[kk];
        for (r = 0;; ++r) {
            int64_t a, b, e;
            int64_t rz = (ndim == 3) ? r : 0;
            int covered = 1;
            for (e = -rz; e <= rz; ++e)
                for (b = -r; b <= r; ++b)
                    for (a = -r; a <= r; ++a) {
                        int64_t m = a < 0 ? -a : a, cx, cy, cz, cell, j;
                        if ((b < 0 ? -b : b) > m) m = b < 0 ? -b : b;
                        if ((e < 0 ? -e : e) > m) m = e < 0 ? -e : e;
                        if (m != r) continue;      /* shell of ring r only */
                        cx = orc_wrap(home[0] + a, nc[0]);
                        cy = orc_wrap(home[1] + b, nc[1]);
                        cz = orc_wrap(home[2] + e, nc[2]);
                        cell = cx + nc[0] * (cy + nc[1] * cz);
                        for (j = cell_start[cell]; j < cell_start[cell + 1]; ++j) {
                            int32_t g = (int32_t)cell_items[j];
                            int64_t d2 = orc_pdist2(ndim, pos, pts + 3 * g, dims);
                            if (d2 < best || (d2 == best && g < bg)) { best = d2; bg = g; }
                        }
                    }
            for (kk = 0; kk < ndim; ++kk)
                if (2 * r + 1 < nc[kk]) covered = 0;
            if (covered) break;
            if (bg >= 0) {
                double bound = floor((double)r * w_min);
                if ((double)best < bound * bound) break;
            }
        }
        spins[i] = bg;
    }
    free(pts); free(cell_start); free(cell_items); free(fill);
    return 0;
}

/* -------------------------------------------------------------- texture */

/* Grain statistics of a spin field: area of every spin value, number of
 * spin values present, mean area N / n_grains, and the area fraction of
 * every bin (grain_bin[q] in [0, n_bins), -1 leaves grain q out).  Counts
 * are integers; ratios are taken in double.  These are the quantities the
 * paper follows over time (orientation distributions, Sec. 5). */
int orc_texture(const int32_t *spins, int64_t N, int32_t Q, const int32_t *grain_bin, int32_t n_bins,
                int64_t *areas /* Q */, int32_t *n_grains, double *mean_area, double *frac /* n_bins */)
{
    int64_t i;
    int32_t q, b, count = 0;
    int64_t *bin_area;
    for (q = 0; q < Q; ++q) areas[q] = 0;
    for (i = 0; i < N; ++i) {
        if (spins[i] < 0 || spins[i] >= Q) continue;   /* inert values belong to no grain */
        areas[spins[i]] += 1;
    }
    for (q = 0; q < Q; ++q) if (areas[q] > 0) ++count;
    *n_grains = count;
    *mean_area = count > 0 ? (double)N / (double)count : 0.0;
    if (n_bins > 0) {
        bin_area = (int64_t *)calloc((size_t)n_bins, sizeof(int64_t));
        if (!bin_area) return -1;
        for (q = 0; q < Q; ++q) {
            b = grain_bin ? grain_bin[q] : -1;
            if (b >= 0 && b < n_bins) bin_area[b] += areas[q];
        }
        for (b = 0; b < n_bins; ++b) frac[b] = (double)bin_area[b] / (double)N;
        free(bin_area);
    }
    return 0;
}

/* Grain-boundary sites (Sec. 3: with neighbour-spin trials only a site with
 * a neighbour of another spin can change): sites whose spin is in [0, Q)
 * and differs from at least one of its M neighbours. */
int64_t orc_boundary_sites(const int32_t *spins, int nbr, const int32_t dims_in[3], int32_t Q)
{
    int off[26][3];
    int64_t dims[3] = {dims_in[0], dims_in[1], dims_in[2]};
    int M = orc_offsets(nbr, off), k;
    int64_t x, y, z, count = 0;
    for (z = 0; z < dims[2]; ++z)
        for (y = 0; y < dims[1]; ++y)
            for (x = 0; x < dims[0]; ++x) {
                int32_t q = spins[x + dims[0] * (y + dims[1] * z)];
                if (q < 0 || q >= Q) continue;
                for (k = 0; k < M; ++k)
                    if (spins[orc_neighbour_index(dims, off, k, x, y, z)] != q) {
                        ++count;
                        break;
                    }
            }
    return count;
}
