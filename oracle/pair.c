/*
 * pair.c -- CPU oracle for bond energies that depend on the pair of grains
 * (the J_{q_i,q_n} of Eq. (7), which the paper writes per pair and names as
 * the route to misorientation-dependent boundaries in its closing section).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).  Shares no code with the HIP
 * library.
 *
 * The paper gives no law for J; the reading used is the Read-Shockley form
 * (W. T. Read and W. Shockley, Phys. Rev. 78 (1950) 275), the standard
 * low-angle boundary energy:
 *   J(theta) = J_max (theta/theta_m) (1 - ln(theta/theta_m))  for theta < theta_m,
 *   J(theta) = J_max                                          otherwise,
 * with theta the misorientation angle between the two grains: the smallest
 * rotation angle of g2 g1^T over the 24 proper rotations of the cube
 * (orientations g are Bunge ZXZ, passive sample -> crystal).  Fixed point:
 * Jp = round-half-even(J * 65536), symmetric, zero diagonal.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

static const double PI = 3.14159265358979323846;

static void bunge(const double e[3], double g[3][3])
{
    double c1 = cos(e[0]), s1 = sin(e[0]), c = cos(e[1]), s = sin(e[1]), c2 = cos(e[2]), s2 = sin(e[2]);
    g[0][0] = c1 * c2 - s1 * s2 * c;  g[0][1] = s1 * c2 + c1 * s2 * c;  g[0][2] = s2 * s;
    g[1][0] = -c1 * s2 - s1 * c2 * c; g[1][1] = -s1 * s2 + c1 * c2 * c; g[1][2] = c2 * s;
    g[2][0] = s1 * s;                 g[2][1] = -c1 * s;                g[2][2] = c;
}

/* the 24 proper rotations of the cube: signed permutation matrices, det +1 */
static int cube_rotations(double R[24][3][3])
{
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    static const int perm_sign[6] = {1, -1, -1, 1, 1, -1};
    int n = 0, p, sx, sy, sz;
    for (p = 0; p < 6; ++p)
        for (sx = -1; sx <= 1; sx += 2)
            for (sy = -1; sy <= 1; sy += 2)
                for (sz = -1; sz <= 1; sz += 2) {
                    int sg[3] = {sx, sy, sz}, r;
                    if (perm_sign[p] * sx * sy * sz != 1) continue;
                    memset(R[n], 0, sizeof R[n]);
                    for (r = 0; r < 3; ++r) R[n][r][perm[p][r]] = sg[r];
                    ++n;
                }
    return n;
}

/* misorientation angle in degrees between two Bunge orientations */
double orc_misorientation_deg(const double e1[3], const double e2[3])
{
    double R[24][3][3], g1[3][3], g2[3][3], dg[3][3], best = -2.0;
    int n = cube_rotations(R), i, j, k, m;
    bunge(e1, g1);
    bunge(e2, g2);
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) {
            dg[i][j] = 0.0;
            for (k = 0; k < 3; ++k) dg[i][j] += g2[i][k] * g1[j][k];
        }
    for (m = 0; m < n; ++m) {
        double tr = 0.0;   /* trace of R dg */
        for (i = 0; i < 3; ++i)
            for (k = 0; k < 3; ++k) tr += R[m][i][k] * dg[k][i];
        if (tr > best) best = tr;
    }
    double cth = (best - 1.0) / 2.0;
    if (cth > 1.0) cth = 1.0;
    if (cth < -1.0) cth = -1.0;
    return acos(cth) * (180.0 / PI);
}

double orc_read_shockley(double theta_deg, double J_max, double theta_m_deg)
{
    double x;
    if (theta_deg <= 0.0) return 0.0;
    if (theta_deg >= theta_m_deg) return J_max;
    x = theta_deg / theta_m_deg;
    return J_max * x * (1.0 - log(x));
}

/* Q x Q fixed-point pair table from Q orientations (euler: Q x 3) */
void orc_pair_table(const double *euler, int32_t Q, double J_max, double theta_m_deg, int32_t *Jp)
{
    int32_t a, b;
    for (a = 0; a < Q; ++a) {
        Jp[(int64_t)a * Q + a] = 0;
        for (b = a + 1; b < Q; ++b) {
            double th = orc_misorientation_deg(euler + 3 * (int64_t)a, euler + 3 * (int64_t)b);
            int32_t v = (int32_t)rint(orc_read_shockley(th, J_max, theta_m_deg) * 65536.0);
            Jp[(int64_t)a * Q + b] = v;
            Jp[(int64_t)b * Q + a] = v;
        }
    }
}
