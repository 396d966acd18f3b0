/*
 * nfold.c -- CPU reference for the rejection-free (n-fold way) counterpart
 * of the Metropolis Potts dynamics.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the test-suite, the package smoke check and
 * the CPU-baseline leg of the benchmark load the shared object built from
 * it.  It shares no source with the HIP library.
 *
 * Paper: Zhang, Dingreville, Bartel, Lusk, arXiv:1007.3509.  Sec. 1 and
 * Sec. 4 name the n-fold way (Bortz, Kalos, Lebowitz 1975; Hassold and Holm
 * 1993 for the Potts model) as the alternative to red/black updating.  The
 * n-fold way simulates the same single-site Metropolis process of Sec. 3,
 * read in continuous time, without rejected trials:
 *
 *   - every site attempts a flip at rate one per MC step; an attempt picks
 *     one of S candidate slots uniformly (S = M neighbour slots whose spin
 *     is proposed, or in the symmetric test mode S = Q-1 other spin values
 *     q+1..q+Q-1 mod Q) and is accepted with min(1, exp(-dE/kT)), dE the
 *     change of Eq. (7) as in the sweep;
 *   - so slot k of site i fires at rate w_ik / (S 2^32) per MC step, with
 *     the integer weight w_ik = 2^32 if d <= 0, T(d) if d > 0 (the sweep's
 *     threshold, floor(2^32 exp(-d / (65536 kT))) capped at 2^32-1), and 0
 *     for a neighbour slot holding the site's own spin;
 *   - with W_i = sum_k w_ik and W = sum_i W_i, the next event comes after an
 *     exponential waiting time of rate W / (S 2^32) and is slot k of site i
 *     with probability w_ik / W (Bortz et al.: pick the class of the event in
 *     proportion to its total rate, then the member).
 *
 * Choices made where the method leaves them open (listed in the design
 * notes of the repository):
 *   - random numbers: Philox4x32-10, key = (lo32(seed), hi32(seed)), for
 *     event number n counter = (lo32(n), hi32(n), 0x4E464F57, j), blocks
 *     j = 0, 1, ... read word by word in order.  Words 0 and 1 form
 *     u = w0 + 2^32 w1; the rank of the event is r = floor(u W / 2^64).
 *     The event is the site i whose cumulative weight (sites in index order)
 *     first exceeds r, and inside it the slot whose cumulative weight first
 *     exceeds the rest of r.
 *   - the waiting time uses the remaining words: an Exp(1) variate E from
 *     von Neumann's comparison method (1951), in 32.32 fixed point: a trial
 *     takes u0 and counts the length n of the strictly decreasing run
 *     u0 > u1 > ... it starts (the word that ends the run is used up); odd n
 *     accepts E = K + u0 / 2^32, even n adds one to K and starts a new trial.
 *     Runs are cut at 64 words and K at 64 (probabilities below 1e-27).
 *   - time is a double in MC steps: dt = (E_fx * S) / W with both operands
 *     converted exactly (E_fx * S < 2^53) or rounded once (W), one correctly
 *     rounded division and one correctly rounded addition t = t_last + dt.
 *   - a run to t_end executes events while t_last + dt <= t_end; the event
 *     that would land beyond t_end is not executed and its counter is not
 *     used up, so the next run redraws the same event from t_last: a run
 *     split into several gives the same state and clock as one run.  A
 *     lattice with W = 0 has no event.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t orc_threshold(int64_t d, float kT);
int orc_neighbours_of(int nbr, const int32_t dims_in[3], int64_t i, int64_t *out);
int orc_num_neighbours(int nbr);

enum { NF_PROP_NEIGHBOUR = 0, NF_PROP_UNIFORM = 1 };
enum { NF_TAG = 0x4E464F57 };
enum { NF_BLOCK = 64 };

/* ----------------------------------------------------- random words */

typedef struct {
    uint32_t key[2];
    uint64_t n;        /* event number */
    uint32_t j;        /* next Philox block */
    uint32_t buf[4];
    int used;          /* words of buf already read */
} nf_stream;

static void nf_stream_init(nf_stream *st, uint64_t seed, uint64_t n)
{
    st->key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    st->key[1] = (uint32_t)(seed >> 32);
    st->n = n;
    st->j = 0;
    st->used = 4;
}

static uint32_t nf_word(nf_stream *st)
{
    if (st->used == 4) {
        uint32_t ctr[4];
        ctr[0] = (uint32_t)(st->n & 0xFFFFFFFFu);
        ctr[1] = (uint32_t)(st->n >> 32);
        ctr[2] = (uint32_t)NF_TAG;
        ctr[3] = st->j++;
        orc_philox4x32_10(ctr, st->key, st->buf);
        st->used = 0;
    }
    return st->buf[st->used++];
}

/* von Neumann's exponential: E in 32.32 fixed point. */
static uint64_t nf_exponential(nf_stream *st)
{
    uint64_t K = 0;
    for (;;) {
        uint32_t u0 = nf_word(st), prev = u0;
        int n = 1;
        while (n < 64) {
            uint32_t v = nf_word(st);
            if (v < prev) { prev = v; ++n; }
            else break;
        }
        if (n & 1) return (K << 32) | (uint64_t)u0;
        if (++K == 64) return K << 32;
    }
}

/* Exposed for the tests: the first `count` exponentials of event streams
 * n0, n0+1, ... (one per stream, drawn after the two selection words). */
void orc_nfold_exponentials(uint64_t seed, uint64_t n0, int64_t count, uint64_t *out)
{
    int64_t c;
    for (c = 0; c < count; ++c) {
        nf_stream st;
        nf_stream_init(&st, seed, n0 + (uint64_t)c);
        (void)nf_word(&st);
        (void)nf_word(&st);
        out[c] = nf_exponential(&st);
    }
}

/* ----------------------------------------------------- weights */

typedef struct {
    int nbr, proposal, M, S;
    int32_t dims[3];
    int64_t N;
    int32_t J_fx, Q;
    const int32_t *Jp; /* Q x Q bond energies, or NULL for J_fx on every unlike bond */
    const int32_t *B;
    float kT;
    int32_t *spins;
    int64_t *nb;       /* N x M neighbour indices */
} nf_lattice;

/* Energy change of Eq. (7) (J(1-delta), each bond once, plus B of the
 * spin) when site i goes from its spin to q_new; with a pair table the bond
 * between spins a and b costs Jp[a][b] (zero diagonal). */
static int64_t nf_delta(const nf_lattice *L, int64_t i, int32_t q_new)
{
    int32_t q = L->spins[i];
    int64_t before = 0, after = 0;
    int k;
    for (k = 0; k < L->M; ++k) {
        int32_t s = L->spins[L->nb[i * L->M + k]];
        if (L->Jp) {
            if (s < 0 || s >= L->Q) continue;   /* an inert value bonds with nothing */
            before += L->Jp[(int64_t)q * L->Q + s];
            after += L->Jp[(int64_t)q_new * L->Q + s];
        } else {
            if (s != q) before += L->J_fx;
            if (s != q_new) after += L->J_fx;
        }
    }
    return after - before + (int64_t)L->B[q_new] - (int64_t)L->B[q];
}

/* Candidate spin of slot k of site i, or -1 for an empty slot. */
static int32_t nf_candidate(const nf_lattice *L, int64_t i, int k)
{
    int32_t q = L->spins[i];
    if (q < 0 || q >= L->Q) return -1;   /* an inert site never changes */
    if (L->proposal == NF_PROP_NEIGHBOUR) {
        int32_t s = L->spins[L->nb[i * L->M + k]];
        return (s == q || s < 0 || s >= L->Q) ? -1 : s;   /* an inert value is never proposed */
    }
    return (int32_t)(((int64_t)q + 1 + k) % L->Q);
}

static uint64_t nf_slot_weight(const nf_lattice *L, int64_t i, int k)
{
    int32_t c = nf_candidate(L, i, k);
    int64_t d;
    if (c < 0) return 0;
    d = nf_delta(L, i, c);
    if (d <= 0) return (uint64_t)1 << 32;
    return (uint64_t)orc_threshold(d, L->kT);
}

static uint64_t nf_site_weight(const nf_lattice *L, int64_t i)
{
    uint64_t w = 0;
    int k;
    for (k = 0; k < L->S; ++k) w += nf_slot_weight(L, i, k);
    return w;
}

/* ----------------------------------------------------- selection */

/* The entry whose cumulative weight (in index order) first exceeds r, with
 * r reduced by the weight of the entries before it; -1 if r >= the total.
 * Block sums (NF_BLOCK entries each) only skip whole blocks: the result is
 * that of one linear scan. */
static int64_t nf_select(const uint64_t *Wblock, const uint64_t *Wsite, int64_t N, uint64_t *r)
{
    int64_t nblocks = (N + NF_BLOCK - 1) / NF_BLOCK, b, i;
    uint64_t acc = 0;
    for (b = 0; b < nblocks; ++b) {
        if (*r < acc + Wblock[b]) break;
        acc += Wblock[b];
    }
    for (i = b * NF_BLOCK; i < N; ++i) {
        if (*r < acc + Wsite[i]) {
            *r -= acc;
            return i;
        }
        acc += Wsite[i];
    }
    return -1;
}

/* Exposed for the tests: nf_select over a weight array (its block sums are
 * formed here). */
int64_t orc_nfold_select(const uint64_t *w, int64_t n, uint64_t r, uint64_t *rest)
{
    int64_t nblocks = (n + NF_BLOCK - 1) / NF_BLOCK, i, got;
    uint64_t *Wblock = (uint64_t *)calloc((size_t)(nblocks > 0 ? nblocks : 1), sizeof(uint64_t));
    if (!Wblock) return -2;
    for (i = 0; i < n; ++i) Wblock[i / NF_BLOCK] += w[i];
    got = nf_select(Wblock, w, n, &r);
    *rest = r;
    free(Wblock);
    return got;
}

/* ----------------------------------------------------- the run */

/* Advance the lattice with the n-fold way until t_end (MC steps).
 *
 * spins    : int32[N], x fastest; a value outside [0, Q) is inert (its site
 *            never changes, it is never proposed, with a pair table it bonds
 *            with nothing); updated in place.
 * dims     : (Lx, Ly, Lz), every side >= 3 (Lz = 1 for 2D neighbourhoods).
 * B        : int32[Q] grain energies (2^-16 units); J_fx the bond energy.
 * proposal : 0 neighbour slots, 1 the Q-1 other spin values.
 * t_last   : in: time of the last executed event; out: updated.
 * n_events : in: events executed so far (the RNG counter); out: updated.
 * max_events: stop after this many events (< 0: no limit); for the tests.
 *
 * Returns the number of events executed, or -1 on bad arguments, -2 if an
 * energy change leaves int32. */
static int64_t nfold_impl(int32_t *spins, int nbr, int proposal, const int32_t dims_in[3], int32_t J_fx,
                          const int32_t *Jp, const int32_t *B, int32_t Q, float kT, uint64_t seed, double t_end,
                          double *t_last, uint64_t *n_events, int64_t max_events)
{
    nf_lattice L;
    uint64_t *Wsite, *Wblock, W = 0;
    int64_t nblocks, i, done = 0;
    int k;
    memset(&L, 0, sizeof L);
    L.nbr = nbr;
    L.proposal = proposal;
    L.M = orc_num_neighbours(nbr);
    if (L.M < 0 || Q < 1 || !(kT > 0.0f) || !t_last || !n_events) return -1;
    if (proposal != NF_PROP_NEIGHBOUR && proposal != NF_PROP_UNIFORM) return -1;
    L.S = proposal == NF_PROP_NEIGHBOUR ? L.M : Q - 1;
    if (L.S < 1) return 0;
    memcpy(L.dims, dims_in, sizeof L.dims);
    if (L.dims[0] < 3 || L.dims[1] < 3 || L.dims[2] < 1) return -1;
    if ((nbr == 2 || nbr == 3) && L.dims[2] < 3) return -1;
    L.N = (int64_t)L.dims[0] * L.dims[1] * L.dims[2];
    L.J_fx = J_fx;
    L.Jp = Jp;
    L.Q = Q;
    L.B = B;
    L.kT = kT;
    L.spins = spins;
    L.nb = (int64_t *)malloc((size_t)L.N * L.M * sizeof(int64_t));
    nblocks = (L.N + NF_BLOCK - 1) / NF_BLOCK;
    Wsite = (uint64_t *)malloc((size_t)L.N * sizeof(uint64_t));
    Wblock = (uint64_t *)calloc((size_t)nblocks, sizeof(uint64_t));
    if (!L.nb || !Wsite || !Wblock) { free(L.nb); free(Wsite); free(Wblock); return -1; }
    for (i = 0; i < L.N; ++i) orc_neighbours_of(nbr, dims_in, i, L.nb + i * L.M);

    /* every energy change must stay in int32, as in the sweep */
    {
        int64_t bmin = B[0], bmax = B[0], bond = J_fx < 0 ? -(int64_t)J_fx : J_fx, worst, e;
        int32_t q;
        for (q = 1; q < Q; ++q) { if (B[q] < bmin) bmin = B[q]; if (B[q] > bmax) bmax = B[q]; }
        if (Jp) {
            bond = 0;
            for (e = 0; e < (int64_t)Q * Q; ++e) {
                int64_t v = Jp[e] < 0 ? -(int64_t)Jp[e] : Jp[e];
                if (v > bond) bond = v;
            }
        }
        worst = (int64_t)L.M * bond + (bmax - bmin);
        if (worst > INT32_MAX) { free(L.nb); free(Wsite); free(Wblock); return -2; }
    }

    for (i = 0; i < L.N; ++i) {
        Wsite[i] = nf_site_weight(&L, i);
        Wblock[i / NF_BLOCK] += Wsite[i];
        W += Wsite[i];
    }

    for (;;) {
        nf_stream st;
        uint64_t u, r, E, acc;
        double t_next;
        int64_t site = -1;
        int slot = -1;
        int32_t q_new;
        int64_t touched[27];
        int nt, a;
        if (W == 0 || (max_events >= 0 && done >= max_events)) break;
        nf_stream_init(&st, seed, *n_events);
        u = (uint64_t)nf_word(&st);
        u |= (uint64_t)nf_word(&st) << 32;
        E = nf_exponential(&st);
        t_next = *t_last + (double)(E * (uint64_t)L.S) / (double)W;
        if (!(t_next <= t_end)) break;
        r = (uint64_t)(((unsigned __int128)u * (unsigned __int128)W) >> 64);
        /* the site, then the slot: cumulative weights in index order */
        site = nf_select(Wblock, Wsite, L.N, &r);
        if (site < 0) { free(L.nb); free(Wsite); free(Wblock); return -1; }   /* cannot happen: r < W */
        acc = 0;
        for (k = 0; k < L.S; ++k) {
            uint64_t w = nf_slot_weight(&L, site, k);
            if (r < acc + w) { slot = k; break; }
            acc += w;
        }
        if (slot < 0) { free(L.nb); free(Wsite); free(Wblock); return -1; }
        q_new = nf_candidate(&L, site, slot);
        spins[site] = q_new;
        /* the weights of the site and of its neighbours depend on its spin */
        touched[0] = site;
        for (k = 0; k < L.M; ++k) touched[k + 1] = L.nb[site * L.M + k];
        nt = L.M + 1;
        for (a = 0; a < nt; ++a) {
            int64_t j = touched[a];
            uint64_t w = nf_site_weight(&L, j);
            Wblock[j / NF_BLOCK] -= Wsite[j];
            W -= Wsite[j];
            Wsite[j] = w;
            Wblock[j / NF_BLOCK] += w;
            W += w;
        }
        *t_last = t_next;
        *n_events += 1;
        ++done;
    }
    free(L.nb);
    free(Wsite);
    free(Wblock);
    return done;
}

int64_t orc_nfold(int32_t *spins, int nbr, int proposal, const int32_t dims_in[3], int32_t J_fx,
                  const int32_t *B, int32_t Q, float kT, uint64_t seed, double t_end,
                  double *t_last, uint64_t *n_events, int64_t max_events)
{
    return nfold_impl(spins, nbr, proposal, dims_in, J_fx, NULL, B, Q, kT, seed, t_end, t_last, n_events,
                      max_events);
}

/* The same run with a bond energy per pair of spins (Eq. (7)'s J_{q_i,q_n},
 * Jp symmetric with zero diagonal, 2^-16 units). */
int64_t orc_nfold_pair(int32_t *spins, int nbr, int proposal, const int32_t dims_in[3], const int32_t *Jp,
                       const int32_t *B, int32_t Q, float kT, uint64_t seed, double t_end,
                       double *t_last, uint64_t *n_events, int64_t max_events)
{
    if (!Jp) return -1;
    return nfold_impl(spins, nbr, proposal, dims_in, 0, Jp, B, Q, kT, seed, t_end, t_last, n_events,
                      max_events);
}

/* Exposed for the tests: the rate of every slot of every site of a state,
 * as the integer weights above (N x S, row-major); Jp may be NULL. */
int orc_nfold_weights(const int32_t *spins, int nbr, int proposal, const int32_t dims_in[3], int32_t J_fx,
                      const int32_t *Jp, const int32_t *B, int32_t Q, float kT, uint64_t *out)
{
    nf_lattice L;
    int64_t i;
    int k;
    memset(&L, 0, sizeof L);
    L.nbr = nbr;
    L.proposal = proposal;
    L.M = orc_num_neighbours(nbr);
    if (L.M < 0 || Q < 1) return -1;
    L.S = proposal == NF_PROP_NEIGHBOUR ? L.M : Q - 1;
    memcpy(L.dims, dims_in, sizeof L.dims);
    L.N = (int64_t)L.dims[0] * L.dims[1] * L.dims[2];
    L.J_fx = J_fx;
    L.Jp = Jp;
    L.Q = Q;
    L.B = B;
    L.kT = kT;
    L.spins = (int32_t *)spins;
    L.nb = (int64_t *)malloc((size_t)L.N * L.M * sizeof(int64_t));
    if (!L.nb) return -1;
    for (i = 0; i < L.N; ++i) orc_neighbours_of(nbr, dims_in, i, L.nb + i * L.M);
    for (i = 0; i < L.N; ++i)
        for (k = 0; k < L.S; ++k) out[i * L.S + k] = nf_slot_weight(&L, i, k);
    free(L.nb);
    return L.S;
}
