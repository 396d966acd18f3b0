/*
 * mcp_mlp.c -- CPU oracle for the stored-energy part of the method:
 * the Monte Carlo crystal-plasticity (MCP) update and a small MLP.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).  Shares no code with the HIP
 * library.
 *
 * MCP follows Sec. 2 of the paper (Zhang, Dingreville, Bartel, Lusk,
 * arXiv:1007.3509): rate-independent, small-deformation crystal plasticity
 * in which only one slip system is activated per step; the candidates are the
 * systems whose resolved shear stress exceeds the slip resistance; the
 * elastic energy E_a of the crystal with system a activated alone gives the
 * selection probability p_a = exp(-beta E_a) / Z (Eq. (1)); system i is
 * taken when sum_{a<=i} p_a - p_i <= R < sum_{a<=i} p_a (Eq. (2)).  Nickel
 * constants from Table 1.  The stored energy follows Eq. (4):
 * E_rho = rho G b^2 / 2 with rho = (2 sigma_f / (G b))^2, i.e. 2 sigma_f^2 / G.
 *
 * Readings where the paper is silent (listed in the design notes):
 *   - Table 1's "C22" is C12 (cubic crystals have C11, C12, C44).
 *   - stresses and energies in MPa (MJ/m^3); beta = 1000 per MPa.
 *   - slip systems: FCC {111}<110>, 12 systems, a fixed order (normals
 *     (111),(-111),(1-11),(11-1); for each, the <110> directions of the
 *     list [1-10],[10-1],[01-1],[110],[101],[011] lying in the plane).
 *   - isotropic hardening of Voce form: tau_c(G) = tau_s - (tau_s - tau_0)
 *     exp(-h0 G / (tau_s - tau_0)), G the accumulated slip.
 *   - single-slip return with linearised consistency:
 *     dgamma = (|tau| - tau_c) / (P:C:P + h), sigma -= sign(tau) dgamma C:P.
 *   - the input strain is the total strain from the virgin crystal, applied
 *     in K = ceil(max|eps_ij| / 1e-5) equal sub-steps (at most 200).
 *   - sigma_f is the current slip resistance tau_c; G is the Voigt average
 *     (C11 - C12 + 3 C44) / 5.
 *   - R = 53-bit fraction of Philox(key = seed, counter = (sample, step, 0,
 *     0x4D435053)) words 0 (high) and 1 (low).
 *
 * Pins: the elastic response (closed-form cubic moduli), the yield point
 * (Schmid law), Eq. (4) and Eq. (2) identities, the ordering of stored
 * energy with Schmid factor, single slip past yield (second-order
 * convergence in the sub-step to the consistency condition with Voce
 * hardening, the stress left by the return) and the Eq. (1) selection
 * frequencies of several candidates, and the invariance of long paths with
 * several competing systems under a turn of the sample frame.  Parity
 * unpinned: the values of those paths' stress and stored energy, which
 * depend on the readings above and have no published values to check
 * against.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Table 1, MPa */
static const double MCP_C11 = 250800.0, MCP_C12 = 150000.0, MCP_C44 = 123500.0;
static const double MCP_TAU0 = 8.0, MCP_TAUS = 122.0, MCP_H0 = 440.0, MCP_BETA = 1000.0;

double orc_mcp_shear_modulus(void) { return (MCP_C11 - MCP_C12 + 3.0 * MCP_C44) / 5.0; }

static void mcp_systems(double n[12][3], double d[12][3])
{
    static const double normals[4][3] = {{1, 1, 1}, {-1, 1, 1}, {1, -1, 1}, {1, 1, -1}};
    static const double dirs[6][3] = {{1, -1, 0}, {1, 0, -1}, {0, 1, -1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
    int a, b, k, m = 0;
    for (a = 0; a < 4; ++a)
        for (b = 0; b < 6; ++b) {
            double dot = normals[a][0] * dirs[b][0] + normals[a][1] * dirs[b][1] + normals[a][2] * dirs[b][2];
            if (dot != 0.0) continue;
            for (k = 0; k < 3; ++k) {
                n[m][k] = normals[a][k] / sqrt(3.0);
                d[m][k] = dirs[b][k] / sqrt(2.0);
            }
            ++m;
        }
}

/* Exposed for tests: the 12 (normal, direction) pairs in the order used. */
void orc_mcp_slip_systems(double *n_out, double *d_out)
{
    double n[12][3], d[12][3];
    mcp_systems(n, d);
    memcpy(n_out, n, sizeof n);
    memcpy(d_out, d, sizeof d);
}

/* cubic stiffness applied to a symmetric strain (tensor components) */
static void stiff(const double e[3][3], double s[3][3])
{
    double tr = e[0][0] + e[1][1] + e[2][2];
    int i, j;
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) {
            if (i == j) s[i][j] = MCP_C12 * tr + (MCP_C11 - MCP_C12) * e[i][i];
            else s[i][j] = 2.0 * MCP_C44 * e[i][j];
        }
}

/* cubic compliance applied to a symmetric stress */
static void compl(const double s[3][3], double e[3][3])
{
    double den = (MCP_C11 - MCP_C12) * (MCP_C11 + 2.0 * MCP_C12);
    double S11 = (MCP_C11 + MCP_C12) / den, S12 = -MCP_C12 / den;
    double tr = s[0][0] + s[1][1] + s[2][2];
    int i, j;
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) {
            if (i == j) e[i][j] = S12 * tr + (S11 - S12) * s[i][i];
            else e[i][j] = s[i][j] / (2.0 * MCP_C44);
        }
}

static double ddot(const double a[3][3], const double b[3][3])
{
    double r = 0.0;
    int i, j;
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) r += a[i][j] * b[i][j];
    return r;
}

/* passive rotation (sample -> crystal) from Bunge ZXZ angles */
static void bunge(const double e[3], double g[3][3])
{
    double c1 = cos(e[0]), s1 = sin(e[0]), c = cos(e[1]), s = sin(e[1]), c2 = cos(e[2]), s2 = sin(e[2]);
    g[0][0] = c1 * c2 - s1 * s2 * c; g[0][1] = s1 * c2 + c1 * s2 * c; g[0][2] = s2 * s;
    g[1][0] = -c1 * s2 - s1 * c2 * c; g[1][1] = -s1 * s2 + c1 * c2 * c; g[1][2] = c2 * s;
    g[2][0] = s1 * s; g[2][1] = -c1 * s; g[2][2] = c;
}

double orc_mcp_tau_c(double gamma)
{
    return MCP_TAUS - (MCP_TAUS - MCP_TAU0) * exp(-MCP_H0 * gamma / (MCP_TAUS - MCP_TAU0));
}

/* Eq. (2): index i with S_{i-1} <= R < S_i over the cumulative probabilities
 * of p[0..n); the last index if rounding leaves R >= S_{n-1}. */
int orc_mcp_select(const double *p, int n, double R)
{
    double S = 0.0;
    int i;
    for (i = 0; i < n; ++i) {
        S += p[i];
        if (S - p[i] <= R && R < S) return i;
    }
    return n - 1;
}

/* Sub-steps for a strain: K = ceil(max|eps_ij| / 1e-5), in [1, 200]. */
int orc_mcp_substeps(const double eps6[6])
{
    double maxabs = 0.0;
    int i, K;
    for (i = 0; i < 6; ++i) if (fabs(eps6[i]) > maxabs) maxabs = fabs(eps6[i]);
    K = (int)ceil(maxabs / 1e-5);
    if (K < 1) K = 1;
    if (K > 200) K = 200;
    return K;
}

/* One crystal driven to the strain eps6 = (e11, e22, e33, e23, e13, e12)
 * (tensor shear components, sample frame) in K equal sub-steps.  Returns
 * E_rho (MPa); tau_c, the accumulated slip and the crystal-frame stress
 * (s11, s22, s33, s23, s13, s12) through the optional outputs, and, for the
 * tests, the number of candidate systems of each sub-step (ncand_out[K])
 * and the system picked at it (picks_out[K], -1 when elastic). */
double orc_mcp_run(const double euler[3], const double eps6[6], uint64_t seed, uint64_t sample, int K,
                   double *tauc_out, double *gamma_out, double *sig_out, int *ncand_out, int *picks_out)
{
    double n[12][3], d[12][3], P[12][3][3], CP[12][3][3], PCP[12];
    double g[3][3], es[3][3], ec[3][3], de[3][3], sig[3][3];
    double gamma = 0.0, tc = MCP_TAU0;
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    int a, i, j, k, step;
    mcp_systems(n, d);
    for (a = 0; a < 12; ++a) {
        for (i = 0; i < 3; ++i)
            for (j = 0; j < 3; ++j) P[a][i][j] = 0.5 * (d[a][i] * n[a][j] + d[a][j] * n[a][i]);
        stiff(P[a], CP[a]);
        PCP[a] = ddot(P[a], CP[a]);
    }
    es[0][0] = eps6[0]; es[1][1] = eps6[1]; es[2][2] = eps6[2];
    es[1][2] = es[2][1] = eps6[3];
    es[0][2] = es[2][0] = eps6[4];
    es[0][1] = es[1][0] = eps6[5];
    bunge(euler, g);
    for (i = 0; i < 3; ++i)          /* crystal-frame strain g es g^T */
        for (j = 0; j < 3; ++j) {
            double acc = 0.0;
            int p, q;
            for (p = 0; p < 3; ++p)
                for (q = 0; q < 3; ++q) acc += g[i][p] * es[p][q] * g[j][q];
            ec[i][j] = acc;
        }
    if (K < 1) K = 1;
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) { de[i][j] = ec[i][j] / K; sig[i][j] = 0.0; }

    for (step = 1; step <= K; ++step) {
        double dsig[3][3], str[3][3];
        int cand[12], nc = 0;
        stiff(de, dsig);
        for (i = 0; i < 3; ++i)
            for (j = 0; j < 3; ++j) str[i][j] = sig[i][j] + dsig[i][j];
        for (a = 0; a < 12; ++a)
            if (fabs(ddot(str, P[a])) > tc) cand[nc++] = a;
        if (ncand_out) ncand_out[step - 1] = nc;
        if (picks_out) picks_out[step - 1] = -1;
        if (nc == 0) {
            memcpy(sig, str, sizeof sig);
            continue;
        }
        {
            double h = MCP_H0 * exp(-MCP_H0 * gamma / (MCP_TAUS - MCP_TAU0));
            double dg[12], E[12], p[12], Emin = 0.0, Z = 0.0, R;
            uint32_t ctr[4], r[4];
            int pick;
            for (k = 0; k < nc; ++k) {
                double tau = ddot(str, P[cand[k]]);
                double sgn = tau > 0.0 ? 1.0 : -1.0;
                double sa[3][3], ea[3][3];
                dg[k] = (fabs(tau) - tc) / (PCP[cand[k]] + h);
                for (i = 0; i < 3; ++i)
                    for (j = 0; j < 3; ++j) sa[i][j] = str[i][j] - sgn * dg[k] * CP[cand[k]][i][j];
                compl(sa, ea);
                E[k] = 0.5 * ddot(sa, ea);
                if (k == 0 || E[k] < Emin) Emin = E[k];
            }
            for (k = 0; k < nc; ++k) { p[k] = exp(-MCP_BETA * (E[k] - Emin)); Z += p[k]; }
            for (k = 0; k < nc; ++k) p[k] /= Z;
            ctr[0] = (uint32_t)sample; ctr[1] = (uint32_t)step; ctr[2] = 0u; ctr[3] = 0x4D435053u;
            orc_philox4x32_10(ctr, key, r);
            R = (double)((((uint64_t)r[0] << 32) | r[1]) >> 11) * (1.0 / 9007199254740992.0);
            pick = orc_mcp_select(p, nc, R);
            if (picks_out) picks_out[step - 1] = cand[pick];
            {
                double tau = ddot(str, P[cand[pick]]);
                double sgn = tau > 0.0 ? 1.0 : -1.0;
                for (i = 0; i < 3; ++i)
                    for (j = 0; j < 3; ++j) sig[i][j] = str[i][j] - sgn * dg[pick] * CP[cand[pick]][i][j];
            }
            gamma += dg[pick];
            tc = orc_mcp_tau_c(gamma);
        }
    }
    if (tauc_out) *tauc_out = tc;
    if (gamma_out) *gamma_out = gamma;
    if (sig_out) {   /* crystal frame, (s11, s22, s33, s23, s13, s12) */
        sig_out[0] = sig[0][0]; sig_out[1] = sig[1][1]; sig_out[2] = sig[2][2];
        sig_out[3] = sig[1][2]; sig_out[4] = sig[0][2]; sig_out[5] = sig[0][1];
    }
    return 2.0 * tc * tc / orc_mcp_shear_modulus();
}

/* One crystal with the sub-step rule above.  Returns E_rho (MPa); tau_c,
 * gamma, the number of sub-steps and the stress through the optional
 * outputs. */
double orc_mcp_one(const double euler[3], const double eps6[6], uint64_t seed, uint64_t sample,
                   double *tauc_out, double *gamma_out, int *steps_out, double *sig_out)
{
    int K = orc_mcp_substeps(eps6);
    if (steps_out) *steps_out = K;
    return orc_mcp_run(euler, eps6, seed, sample, K, tauc_out, gamma_out, sig_out, NULL, NULL);
}

/* The system picked at sub-step `step` (1-based) of K for one crystal under
 * n sample indices sample0 .. sample0 + n - 1 (each draws its own R of
 * Eq. (2)); for the tests of Eq. (1). */
void orc_mcp_picks(const double euler[3], const double eps6[6], uint64_t seed, uint64_t sample0, int64_t n, int K,
                   int step, int *pick_out, int *ncand_out)
{
    int64_t s;
    int *picks = (int *)malloc(sizeof(int) * (size_t)(K > 0 ? K : 1));
    int *nc = (int *)malloc(sizeof(int) * (size_t)(K > 0 ? K : 1));
    if (!picks || !nc || step < 1 || step > K) {
        free(picks);
        free(nc);
        return;
    }
    for (s = 0; s < n; ++s) {
        orc_mcp_run(euler, eps6, seed, sample0 + (uint64_t)s, K, NULL, NULL, NULL, nc, picks);
        pick_out[s] = picks[step - 1];
        if (ncand_out) ncand_out[s] = nc[step - 1];
    }
    free(picks);
    free(nc);
}

void orc_mcp_solve(const double *euler, const double *eps6, int64_t n, uint64_t seed, uint64_t sample0,
                   double *E_out, double *tauc_out, double *gamma_out, int threads)
{
    int64_t s;
    if (threads < 1) threads = 1;
#pragma omp parallel for num_threads(threads) schedule(dynamic, 64)
    for (s = 0; s < n; ++s) {
        double tc, gm;
        int K;
        E_out[s] = orc_mcp_one(euler + 3 * s, eps6 + 6 * s, seed, sample0 + (uint64_t)s, &tc, &gm, &K, NULL);
        if (tauc_out) tauc_out[s] = tc;
        if (gamma_out) gamma_out[s] = gm;
    }
}

/* ------------------------------------------------------------------ MLP
 * y = w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3, 9 -> 64 -> 64 -> 1.
 * Parameter vector (4865): W1[64][9], b1[64], W2[64][64], b2[64], w3[64], b3.
 * Loss: mean over the batch of (y - t)^2.  Textbook back-propagation with
 * tanh' = 1 - tanh^2.  Adam (Kingma & Ba, 2015) with bias correction. */
enum { MLP_IN = 9, MLP_H = 64, MLP_NP = 64 * 9 + 64 + 64 * 64 + 64 + 64 + 1 };

int orc_mlp_num_params(void) { return MLP_NP; }

static void mlp_views(const double *th, const double **W1, const double **b1, const double **W2,
                      const double **b2, const double **w3, const double **b3)
{
    *W1 = th;
    *b1 = *W1 + MLP_H * MLP_IN;
    *W2 = *b1 + MLP_H;
    *b2 = *W2 + MLP_H * MLP_H;
    *w3 = *b2 + MLP_H;
    *b3 = *w3 + MLP_H;
}

static double mlp_one(const double *th, const double *x, double h1[MLP_H], double h2[MLP_H])
{
    const double *W1, *b1, *W2, *b2, *w3, *b3;
    double y;
    int i, j;
    mlp_views(th, &W1, &b1, &W2, &b2, &w3, &b3);
    for (i = 0; i < MLP_H; ++i) {
        double a = b1[i];
        for (j = 0; j < MLP_IN; ++j) a += W1[i * MLP_IN + j] * x[j];
        h1[i] = tanh(a);
    }
    for (i = 0; i < MLP_H; ++i) {
        double a = b2[i];
        for (j = 0; j < MLP_H; ++j) a += W2[i * MLP_H + j] * h1[j];
        h2[i] = tanh(a);
    }
    y = b3[0];
    for (i = 0; i < MLP_H; ++i) y += w3[i] * h2[i];
    return y;
}

void orc_mlp_forward(const double *th, const double *X, int64_t n, double *y)
{
    int64_t s;
    double h1[MLP_H], h2[MLP_H];
    for (s = 0; s < n; ++s) y[s] = mlp_one(th, X + MLP_IN * s, h1, h2);
}

/* mean squared error over n samples and its gradient with respect to th */
double orc_mlp_loss_grad(const double *th, const double *X, const double *t, int64_t n, double *grad)
{
    const double *W1, *b1, *W2, *b2, *w3, *b3;
    double *gW1 = grad, *gb1 = gW1 + MLP_H * MLP_IN, *gW2 = gb1 + MLP_H, *gb2 = gW2 + MLP_H * MLP_H;
    double *gw3 = gb2 + MLP_H, *gb3 = gw3 + MLP_H;
    double loss = 0.0;
    int64_t s;
    int i, j;
    mlp_views(th, &W1, &b1, &W2, &b2, &w3, &b3);
    memset(grad, 0, sizeof(double) * MLP_NP);
    for (s = 0; s < n; ++s) {
        const double *x = X + MLP_IN * s;
        double h1[MLP_H], h2[MLP_H], d2[MLP_H], d1[MLP_H];
        double y = mlp_one(th, x, h1, h2);
        double dy = 2.0 * (y - t[s]) / (double)n;
        loss += (y - t[s]) * (y - t[s]);
        gb3[0] += dy;
        for (i = 0; i < MLP_H; ++i) {
            gw3[i] += dy * h2[i];
            d2[i] = dy * w3[i] * (1.0 - h2[i] * h2[i]);
        }
        for (i = 0; i < MLP_H; ++i) {
            gb2[i] += d2[i];
            for (j = 0; j < MLP_H; ++j) gW2[i * MLP_H + j] += d2[i] * h1[j];
        }
        for (j = 0; j < MLP_H; ++j) {
            double a = 0.0;
            for (i = 0; i < MLP_H; ++i) a += W2[i * MLP_H + j] * d2[i];
            d1[j] = a * (1.0 - h1[j] * h1[j]);
        }
        for (i = 0; i < MLP_H; ++i) {
            gb1[i] += d1[i];
            for (j = 0; j < MLP_IN; ++j) gW1[i * MLP_IN + j] += d1[i] * x[j];
        }
    }
    return loss / (double)n;
}

/* One Adam step at step number t >= 1 (m, v updated in place). */
void orc_adam_step(double *th, const double *g, double *m, double *v, int64_t t, double lr, double b1, double b2,
                   double eps)
{
    int i;
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (i = 0; i < MLP_NP; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        th[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
