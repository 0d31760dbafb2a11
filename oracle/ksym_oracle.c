/*
 * CPU oracle for batched 2x2 / 3x3 real symmetric eigendecomposition
 * (Kronenburg, "A Method for Fast Diagonalization of a 2x2 or 3x3 Real
 * Symmetric Matrix", arXiv:1306.6291).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header or constant with the HIP library.
 *
 * Everything is IEEE double (compiled with -O2 -ffp-contract=off, no fast-math)
 * except the cyclic Jacobi solver, which runs in x87 long double and exists to
 * pin the paper's formulas against an independent method.
 *
 * Entry layout: a 3x3 symmetric matrix is given by its six unique entries in
 * the order (A11, A22, A33, A12, A13, A23); a 2x2 by (A11, A22, A12).  D is
 * row-major (D11, D12, D13, D21, ..., D33); column k of D is the eigenvector of
 * lam[k].
 *
 * Readings of the paper where it is silent or ambiguous (each is marked in the
 * code where it applies):
 *   R-typo  : the 2x2 characteristic equation (3.1) prints A11+A12 where the
 *             trace A11+A22 is meant; (3.2)-(3.3) are used as printed.
 *   R-sign0 : sign(0) = +1 in (3.2)-(3.3).
 *   R-atan  : phi = 1/2 arctan(2 A12/(A11-A22)) (3.5) is evaluated as printed
 *             when A11 != A22; on the tie line A11 = A22 it is
 *             sign(A12)*pi/4 (0 when A12 = 0 too, as the paper states).
 *   R-order : the eigenvalues of (4.10)-(4.12) are returned in the order the
 *             formulas produce, which is lam1 >= lam3 >= lam2 because
 *             Delta lies in [0, pi].
 *   R-clamp : q / (2 sqrt(p^3)) is clamped to [-1, 1] before arccos (4.9);
 *             v and w of (5.1)-(5.2) are clamped to [0, 1].
 *   R-double: the equality case q^2 = 4 p^3 of §5 is taken when the computed
 *             eigenvalues coincide exactly or their smaller split, relative to
 *             sqrt(p), is below tau_dbl.  That branch builds D from (5.20)-(5.25)
 *             with the mean of the two close roots as the repeated value; the
 *             returned eigenvalues are the roots (4.10)-(4.12) themselves,
 *             equal where q^2 = 4 p^3 holds exactly.
 *   R-angle : angle(0) = 0, and -0 is turned into +0 before atan2.
 *   R-select: "smallest absolute difference" between phi1(1) and phi1(2) is
 *             measured on the circle (remainder modulo 2 pi); ties keep the
 *             first combination in the order (+,+), (+,-), (-,+), (-,-).
 *   R-slots : every branch returns lam in the slots (max, min, mid) of the
 *             general branch.  The double branch permutes D's columns into
 *             those slots, negates one column if that made det D = -1, and
 *             re-extracts the angles from D, so D = R1(phi1) R2(phi2) R3(phi3).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KO_PI 3.14159265358979323846

enum { KO_GENERAL = 0, KO_DOUBLE = 1, KO_TRIPLE = 2 };

/* ------------------------------------------------------------------------ */
/* Rotation matrices of paper §2, eqs. (2.5) and (2.7)-(2.9).               */
/* ------------------------------------------------------------------------ */
static void rot2(double phi, double R[2][2])
{
    R[0][0] = cos(phi); R[0][1] = -sin(phi);
    R[1][0] = sin(phi); R[1][1] = cos(phi);
}

static void rot_axis1(double a, double R[3][3])
{
    double c = cos(a), s = sin(a);
    double M[3][3] = {{1, 0, 0}, {0, c, -s}, {0, s, c}};
    memcpy(R, M, sizeof M);
}

static void rot_axis2(double a, double R[3][3])
{
    double c = cos(a), s = sin(a);
    double M[3][3] = {{c, 0, s}, {0, 1, 0}, {-s, 0, c}};
    memcpy(R, M, sizeof M);
}

static void rot_axis3(double a, double R[3][3])
{
    double c = cos(a), s = sin(a);
    double M[3][3] = {{c, -s, 0}, {s, c, 0}, {0, 0, 1}};
    memcpy(R, M, sizeof M);
}

static void matmul3(double A[3][3], double B[3][3], double C[3][3])
{
    double T[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[i][k] * B[k][j];
            T[i][j] = s;
        }
    memcpy(C, T, sizeof T);
}

/* D = R1(phi1) R2(phi2) R3(phi3), eq. (2.6) */
static void euler_to_D(double p1, double p2, double p3, double D[3][3])
{
    double R1[3][3], R2[3][3], R3[3][3];
    rot_axis1(p1, R1);
    rot_axis2(p2, R2);
    rot_axis3(p3, R3);
    matmul3(R1, R2, D);
    matmul3(D, R3, D);
}

/* angle(r): anti-clockwise angle of the 2-vector r from the positive x-axis
 * (§5, before (5.11)); R-angle reading. */
static double angle2(double x, double y)
{
    x += 0.0;
    y += 0.0;
    if (x == 0.0 && y == 0.0) return 0.0;
    return atan2(y, x);
}

/* ------------------------------------------------------------------------ */
/* 2x2: paper §3                                                            */
/* ------------------------------------------------------------------------ */
void ko_eig2(const double a[3], double lam[2], double D[4], double *phi)
{
    double a11 = a[0], a22 = a[1], a12 = a[2];
    double d = a11 - a22;
    double sg = (d >= 0.0) ? 1.0 : -1.0;                     /* R-sign0 */
    double root = sqrt(d * d + 4.0 * a12 * a12);
    lam[0] = 0.5 * (a11 + a22 + sg * root);                  /* (3.2) */
    lam[1] = 0.5 * (a11 + a22 - sg * root);                  /* (3.3) */
    double f;
    if (d != 0.0)
        f = 0.5 * atan(2.0 * a12 / d);                       /* (3.5) */
    else if (a12 != 0.0)
        f = (a12 > 0.0 ? 0.25 : -0.25) * KO_PI;              /* R-atan */
    else
        f = 0.0;                                             /* §3 special case */
    double R[2][2];
    rot2(f, R);                                              /* (2.5) */
    D[0] = R[0][0]; D[1] = R[0][1];
    D[2] = R[1][0]; D[3] = R[1][1];
    *phi = f;
}

/* ------------------------------------------------------------------------ */
/* 3x3: paper §4 (eigenvalues) and §5 (angles)                              */
/* ------------------------------------------------------------------------ */

/* The vectors g1, g2 of (5.7)-(5.8) for given lam1..3, v, w, phi2, phi3. */
static void g_vectors(double l1, double l2, double l3, double v, double w,
                      double p2, double p3, double g1[2], double g2[2])
{
    g1[0] = 0.5 * (l1 - l2) * cos(p2) * sin(2.0 * p3);
    g1[1] = 0.5 * ((l1 - l2) * w + l2 - l3) * sin(2.0 * p2);
    g2[0] = (l1 - l2) * (1.0 + (v - 2.0) * w) + (l2 - l3) * v;
    g2[1] = (l1 - l2) * sin(p2) * sin(2.0 * p3);
}

/* phi1(1) and phi1(2) of (5.13)-(5.14): rotate g by -psi, psi = angle(f). */
static void phi1_estimates(const double f1[2], const double f2[2],
                           const double g1[2], const double g2[2],
                           double *e1, double *e2)
{
    double psi1 = angle2(f1[0], f1[1]);                      /* (5.11) */
    double psi2 = angle2(f2[0], f2[1]);                      /* (5.12) */
    double R[2][2];
    rot2(-psi1, R);
    double h1x = R[0][0] * g1[0] + R[0][1] * g1[1];
    double h1y = R[1][0] * g1[0] + R[1][1] * g1[1];
    rot2(-psi2, R);
    double h2x = R[0][0] * g2[0] + R[0][1] * g2[1];
    double h2y = R[1][0] * g2[0] + R[1][1] * g2[1];
    *e1 = angle2(h1x, h1y);                                  /* (5.13) */
    *e2 = 0.5 * angle2(h2x, h2y);                            /* (5.14) */
}

static double clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

/* Angles out of a rotation D = R1 R2 R3 (rows/cols 0-based):
 * D13 = sin phi2, (D11, D12) = cos phi2 (cos phi3, -sin phi3),
 * (D23, D33) = cos phi2 (-sin phi1, cos phi1); at cos phi2 = 0 take phi3 = 0,
 * then (D22, D32) = (cos phi1, sin phi1). */
static void D_to_euler(double D[3][3], double phi[3])
{
    double c2 = sqrt(D[0][0] * D[0][0] + D[0][1] * D[0][1]);
    phi[1] = atan2(D[0][2], c2);
    if (c2 > 0.0) {
        phi[2] = atan2(-D[0][1], D[0][0]);
        phi[0] = atan2(-D[1][2], D[2][2]);
    } else {
        phi[2] = 0.0;
        phi[0] = atan2(D[2][1], D[1][1]);
    }
}

/* Debug record of the general branch, exposed for the pin tests. */
typedef struct {
    double b, p, q, Delta;
    double v, w;
    double delta[4];         /* |phi1(1) - phi1(2)| per combination (+,+),(+,-),(-,+),(-,-) */
    double f1n, f2n, g1n, g2n;   /* |f1|, |f2|, |g1|, |g2| of the chosen combination */
    int chosen;
    int branch;
} ko_debug3;

int ko_eig3_dbg(const double A[6], double tau_dbl, double lam[3], double Dout[9],
                double phi[3], ko_debug3 *dbg)
{
    const double a11 = A[0], a22 = A[1], a33 = A[2];
    const double a12 = A[3], a13 = A[4], a23 = A[5];
    ko_debug3 scratch;
    if (!dbg) dbg = &scratch;
    memset(dbg, 0, sizeof *dbg);

    /* §4: b (4.2), p (4.7), q (4.8) */
    double b = a11 + a22 + a33;
    double p = 0.5 * ((a11 - a22) * (a11 - a22) + (a11 - a33) * (a11 - a33) +
                      (a22 - a33) * (a22 - a33)) +
               3.0 * (a12 * a12 + a13 * a13 + a23 * a23);
    double q = 18.0 * (a11 * a22 * a33 + 3.0 * a12 * a13 * a23) +
               2.0 * (a11 * a11 * a11 + a22 * a22 * a22 + a33 * a33 * a33) +
               9.0 * (a11 + a22 + a33) * (a12 * a12 + a13 * a13 + a23 * a23) -
               3.0 * (a11 + a22) * (a11 + a33) * (a22 + a33) -
               27.0 * (a11 * a23 * a23 + a22 * a13 * a13 + a33 * a12 * a12);
    dbg->b = b; dbg->p = p; dbg->q = q;

    if (p == 0.0) {
        /* §5 special case p = 0: triple eigenvalue, all angles 0. */
        lam[0] = lam[1] = lam[2] = b / 3.0;
        for (int i = 0; i < 9; ++i) Dout[i] = (i % 4 == 0) ? 1.0 : 0.0;
        phi[0] = phi[1] = phi[2] = 0.0;
        dbg->branch = KO_TRIPLE;
        return KO_TRIPLE;
    }

    /* (4.9): Delta = arccos(q / (2 sqrt(p^3))), R-clamp */
    double r = q / (2.0 * sqrt(p * p * p));
    if (r > 1.0) r = 1.0;
    if (r < -1.0) r = -1.0;
    double Delta = acos(r);
    dbg->Delta = Delta;
    double sp = sqrt(p);
    /* (4.10)-(4.12) */
    double l1 = (b + 2.0 * sp * cos(Delta / 3.0)) / 3.0;
    double l2 = (b + 2.0 * sp * cos((Delta + 2.0 * KO_PI) / 3.0)) / 3.0;
    double l3 = (b + 2.0 * sp * cos((Delta - 2.0 * KO_PI) / 3.0)) / 3.0;

    /* §5 vectors f1 (5.5), f2 (5.6); R-angle canonicalisation of -0 */
    double f1[2] = {a12 + 0.0, -a13 + 0.0};
    double f2[2] = {(a22 - a33) + 0.0, -2.0 * a23 + 0.0};
    double f1n = sqrt(f1[0] * f1[0] + f1[1] * f1[1]);
    double f2n = sqrt(f2[0] * f2[0] + f2[1] * f2[1]);
    dbg->f1n = f1n; dbg->f2n = f2n;

    double den = (l2 - l3) * (l3 - l1);
    double split = fmin(l1 - l3, l3 - l2) / sp;
    double D[3][3];

    if (!(den == 0.0 || split < tau_dbl)) {
        /* General branch. (5.1), (5.2), (5.3)-(5.4) */
        double v = (a12 * a12 + a13 * a13 + (a11 - l3) * (a11 + l3 - l1 - l2)) / den;
        v = clamp01(v);
        double w = (v == 0.0) ? 1.0 : (a11 - l3 + (l3 - l2) * v) / ((l1 - l2) * v);
        w = clamp01(w);
        dbg->v = v; dbg->w = w;
        double best = INFINITY, p1 = 0.0, p2 = 0.0, p3 = 0.0;
        int chosen = 0;
        const double sgn[4][2] = {{1, 1}, {1, -1}, {-1, 1}, {-1, -1}};
        for (int c = 0; c < 4; ++c) {
            double t2 = sgn[c][0] * acos(sqrt(v));
            double t3 = sgn[c][1] * acos(sqrt(w));
            double g1[2], g2[2], e1, e2;
            g_vectors(l1, l2, l3, v, w, t2, t3, g1, g2);
            phi1_estimates(f1, f2, g1, g2, &e1, &e2);
            double delta = fabs(remainder(e1 - e2, 2.0 * KO_PI));   /* R-select */
            dbg->delta[c] = delta;
            if (delta < best) {
                best = delta;
                chosen = c;
                p1 = (f1n >= f2n) ? e1 : e2;                         /* (5.15) */
                p2 = t2;
                p3 = t3;
                dbg->g1n = sqrt(g1[0] * g1[0] + g1[1] * g1[1]);
                dbg->g2n = sqrt(g2[0] * g2[0] + g2[1] * g2[1]);
            }
        }
        dbg->chosen = chosen;
        euler_to_D(p1, p2, p3, D);                                   /* (2.6) */
        lam[0] = l1; lam[1] = l2; lam[2] = l3;
        phi[0] = p1; phi[1] = p2; phi[2] = p3;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Dout[3 * i + j] = D[i][j];
        dbg->branch = KO_GENERAL;
        return KO_GENERAL;
    }

    /* §5 special case q^2 = 4 p^3 != 0 (R-double): two equal eigenvalues.
     * Internal labels (lam, lam, lam_s) as in (5.20). */
    double lm, ls;
    if (l1 - l3 < l3 - l2) {     /* Delta near pi: lam1 = lam3 */
        lm = 0.5 * (l1 + l3);
        ls = l2;
    } else {                     /* Delta near 0: lam3 = lam2 */
        lm = 0.5 * (l3 + l2);
        ls = l1;
    }
    double s = clamp01((a11 - ls) / (lm - ls));                      /* (5.21) */
    dbg->v = s; dbg->w = 1.0;
    double best = INFINITY, p1 = 0.0, p2 = 0.0;
    int chosen = 0;
    for (int c = 0; c < 2; ++c) {
        double t2 = (c == 0 ? 1.0 : -1.0) * acos(sqrt(s));           /* (5.22) */
        double g1[2] = {0.0, 0.5 * (lm - ls) * sin(2.0 * t2)};       /* (5.24) */
        double g2[2] = {(lm - ls) * s, 0.0};                         /* (5.25) */
        double e1, e2;
        phi1_estimates(f1, f2, g1, g2, &e1, &e2);
        double delta = fabs(remainder(e1 - e2, 2.0 * KO_PI));
        dbg->delta[c] = delta;
        if (delta < best) {
            best = delta;
            chosen = c;
            p1 = (f1n >= f2n) ? e1 : e2;
            p2 = t2;
            dbg->g1n = sqrt(g1[0] * g1[0] + g1[1] * g1[1]);
            dbg->g2n = sqrt(g2[0] * g2[0] + g2[1] * g2[1]);
        }
    }
    dbg->chosen = chosen;
    euler_to_D(p1, p2, 0.0, D);                                      /* (5.23) */
    /* R-slots: columns (lm, lm, ls) -> slots (max, min, mid).  R-double: the
     * eigenvalues stay the roots (4.10)-(4.12); they coincide where q^2 = 4p^3
     * holds exactly, and otherwise keep the split the cubic resolves (the
     * mean lm serves (5.21) only).  In slot order the roots are (l1, l2, l3)
     * in both cases: (ls, lm, lm) = (l1, l2, l3) with l3 ~ l2 and
     * (lm, ls, lm) = (l1, l2, l3) with l1 ~ l3. */
    double E[3][3];
    if (ls > lm) {               /* (ls, lm, lm): cyclic permutation, det kept */
        for (int i = 0; i < 3; ++i) {
            E[i][0] = D[i][2]; E[i][1] = D[i][0]; E[i][2] = D[i][1];
        }
    } else {                     /* (lm, ls, lm): a swap, negate one column */
        for (int i = 0; i < 3; ++i) {
            E[i][0] = D[i][0]; E[i][1] = D[i][2]; E[i][2] = -D[i][1];
        }
    }
    lam[0] = l1; lam[1] = l2; lam[2] = l3;
    D_to_euler(E, phi);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Dout[3 * i + j] = E[i][j];
    dbg->branch = KO_DOUBLE;
    return KO_DOUBLE;
}

int ko_eig3(const double A[6], double tau_dbl, double lam[3], double D[9], double phi[3])
{
    return ko_eig3_dbg(A, tau_dbl, lam, D, phi, NULL);
}

/* ------------------------------------------------------------------------ */
/* Independent solver: cyclic Jacobi in x87 long double (textbook, e.g.     */
/* Golub & Van Loan, symmetric Schur 2x2 + cyclic sweeps).                  */
/* Returns eigenvalues sorted descending and the matching eigenvectors      */
/* (columns of V, row-major), det V = +1.                                    */
/* ------------------------------------------------------------------------ */
void ko_jacobi3_ld(const double A6[6], double lam_out[3], double V_out[9],
                   long double lam_ld[3])
{
    long double a[3][3] = {{A6[0], A6[3], A6[4]}, {A6[3], A6[1], A6[5]}, {A6[4], A6[5], A6[2]}};
    long double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    long double fro = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) fro += a[i][j] * a[i][j];
    for (int sweep = 0; sweep < 60; ++sweep) {
        long double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        if (off <= 1e-40L * fro || off == 0) break;
        const int P[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (int k = 0; k < 3; ++k) {
            int p = P[k][0], q = P[k][1];
            if (a[p][q] == 0) continue;
            long double theta = (a[q][q] - a[p][p]) / (2 * a[p][q]);
            long double t = (theta >= 0 ? 1 : -1) / (fabsl(theta) + sqrtl(theta * theta + 1));
            long double c = 1 / sqrtl(t * t + 1), s = t * c;
            /* A <- J^T A J with J = rotation in (p,q) */
            for (int r = 0; r < 3; ++r) {
                long double arp = a[r][p], arq = a[r][q];
                a[r][p] = c * arp - s * arq;
                a[r][q] = s * arp + c * arq;
            }
            for (int r = 0; r < 3; ++r) {
                long double apr = a[p][r], aqr = a[q][r];
                a[p][r] = c * apr - s * aqr;
                a[q][r] = s * apr + c * aqr;
            }
            for (int r = 0; r < 3; ++r) {
                long double vrp = V[r][p], vrq = V[r][q];
                V[r][p] = c * vrp - s * vrq;
                V[r][q] = s * vrp + c * vrq;
            }
        }
    }
    int idx[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (a[idx[j]][idx[j]] > a[idx[i]][idx[i]]) {
                int t = idx[i]; idx[i] = idx[j]; idx[j] = t;
            }
    long double W[3][3];
    for (int k = 0; k < 3; ++k) {
        lam_ld[k] = a[idx[k]][idx[k]];
        lam_out[k] = (double)lam_ld[k];
        for (int r = 0; r < 3; ++r) W[r][k] = V[r][idx[k]];
    }
    long double det = W[0][0] * (W[1][1] * W[2][2] - W[1][2] * W[2][1]) -
                      W[0][1] * (W[1][0] * W[2][2] - W[1][2] * W[2][0]) +
                      W[0][2] * (W[1][0] * W[2][1] - W[1][1] * W[2][0]);
    if (det < 0)
        for (int r = 0; r < 3; ++r) W[r][2] = -W[r][2];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) V_out[3 * r + k] = (double)W[r][k];
}

/* ------------------------------------------------------------------------ */
/* Adjoint (not in the paper; first-order perturbation theory of the        */
/* symmetric eigenproblem): with A = D diag(lam) D^T,                        */
/*   Abar = D [diag(lam_bar) + F o (D^T D_bar)] D^T,                         */
/*   F_ij = (lam_j - lam_i) / ((lam_j - lam_i)^2 + eps^2), F_ii = 0,          */
/* and the six plane gradients gA_ii = Abar_ii, gA_ij = Abar_ij + Abar_ji.   */
/* eps = 0 gives the exact 1 / (lam_j - lam_i).  An exactly repeated pair    */
/* with eps = 0 takes F_ij = 0, the value of the regularised weight at      */
/* lam_j = lam_i for every eps > 0 (the formula would read 0/0 there).       */
/* Angle cotangents (phi, gphi non-NULL): with D = R1 R2 R3 (eq. (2.6)) and  */
/* R_k = exp(phi_k [e_k]x), D^T dD = [w]x with w = M dphi, the columns of M  */
/* R3^T R2^T e1 = (c2 c3, -c2 s3, s2), R3^T e2 = (s3, c3, 0), e3; so gphi     */
/* acts as wbar = M^-T gphi added to (E_32, E_13, E_21) of E = D^T Dbar.      */
/* M^-T divides by c2 = cos phi2 (gimbal lock at c2 = 0), regularised as    */
/* c2 / (c2^2 + delta^2).                                                    */
/* ------------------------------------------------------------------------ */
void ko_eig3_bwd(const double lam[3], const double D9[9], const double glam[3],
                 const double gD9[9], const double phi[3], const double gphi[3], double eps, double delta,
                 double gA[6])
{
    double D[3][3], G[3][3], E[3][3], M[3][3], T[3][3], Abar[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            D[i][j] = D9[3 * i + j];
            G[i][j] = gD9 ? gD9[3 * i + j] : 0.0;
        }
    /* E = D^T Dbar */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += D[k][i] * G[k][j];
            E[i][j] = s;
        }
    if (phi && gphi) {
        const double c2 = cos(phi[1]), s2 = sin(phi[1]), c3 = cos(phi[2]), s3 = sin(phi[2]);
        const double u = (gphi[0] - s2 * gphi[2]) * c2 / (c2 * c2 + delta * delta);
        const double v = gphi[1];
        E[2][1] += c3 * u + s3 * v;
        E[0][2] += -s3 * u + c3 * v;
        E[1][0] += gphi[2];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            if (i == j) {
                M[i][j] = glam ? glam[i] : 0.0;
            } else {
                double d = lam[j] - lam[i];
                M[i][j] = (d != 0.0 ? d / (d * d + eps * eps) : 0.0) * E[i][j];
            }
        }
    /* Abar = D M D^T */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += D[i][k] * M[k][j];
            T[i][j] = s;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += T[i][k] * D[j][k];
            Abar[i][j] = s;
        }
    gA[0] = Abar[0][0];
    gA[1] = Abar[1][1];
    gA[2] = Abar[2][2];
    gA[3] = Abar[0][1] + Abar[1][0];
    gA[4] = Abar[0][2] + Abar[2][0];
    gA[5] = Abar[1][2] + Abar[2][1];
}

/* ------------------------------------------------------------------------ */
/* 2x2 adjoint (not in the paper), the same first-order result for          */
/* A = D diag(lam1, lam2) D^T with D = R(phi) of eq. (2.5): E = D^T Dbar,    */
/* Abar = D [diag(lam_bar) + F o E] D^T.  The angle enters through           */
/* D^T dD = [[0, -dphi], [dphi, 0]], i.e. dphi = d2^T dA d1 / (lam1 - lam2), */
/* so a cotangent phibar adds phibar to E_21.  Planes gA = (A11, A22, A12),  */
/* gA12 = Abar_12 + Abar_21.                                                 */
/* ------------------------------------------------------------------------ */
void ko_eig2_bwd(const double lam[2], const double D4[4], const double glam[2], const double gD4[4],
                 double gphi, double eps, double gA[3])
{
    double D[2][2], G[2][2], E[2][2], M[2][2], T[2][2], Abar[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            D[i][j] = D4[2 * i + j];
            G[i][j] = gD4 ? gD4[2 * i + j] : 0.0;
        }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) E[i][j] = D[0][i] * G[0][j] + D[1][i] * G[1][j];
    E[1][0] += gphi;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            if (i == j) {
                M[i][j] = glam ? glam[i] : 0.0;
            } else {
                double d = lam[j] - lam[i];
                M[i][j] = (d != 0.0 ? d / (d * d + eps * eps) : 0.0) * E[i][j];
            }
        }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) T[i][j] = D[i][0] * M[0][j] + D[i][1] * M[1][j];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) Abar[i][j] = T[i][0] * D[j][0] + T[i][1] * D[j][1];
    gA[0] = Abar[0][0];
    gA[1] = Abar[1][1];
    gA[2] = Abar[0][1] + Abar[1][0];
}

/* ------------------------------------------------------------------------ */
/* The inverse map, from the definitions: A = D diag(lam) D^T with          */
/* D = R1(phi1) R2(phi2) R3(phi3) (eq. (2.6)) for 3x3, D = R(phi) (eq. (2.5)) */
/* for 2x2.  Planes A = (A11, A22, A33, A12, A13, A23) and (A11, A22, A12).  */
/* ------------------------------------------------------------------------ */
void ko_compose3(const double lam[3], const double phi[3], double A[6])
{
    double D[3][3], M[3][3];
    euler_to_D(phi[0], phi[1], phi[2], D);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += D[i][k] * lam[k] * D[j][k];
            M[i][j] = s;
        }
    A[0] = M[0][0];
    A[1] = M[1][1];
    A[2] = M[2][2];
    A[3] = M[0][1];
    A[4] = M[0][2];
    A[5] = M[1][2];
}

void ko_compose2(const double lam[2], double phi, double A[3])
{
    const double c = cos(phi), s = sin(phi);
    const double D[2][2] = {{c, -s}, {s, c}};
    double M[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) M[i][j] = D[i][0] * lam[0] * D[j][0] + D[i][1] * lam[1] * D[j][1];
    A[0] = M[0][0];
    A[1] = M[1][1];
    A[2] = M[0][1];
}

/* ------------------------------------------------------------------------ */
/* Batch drivers over structure-of-arrays planes, split over host threads.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kind;                     /* 3: eig3, 2: eig2, 4: jacobi, 5: bwd, 6: 2x2 bwd, 7/8: compose 3x3/2x2 */
    int64_t lo, hi;
    const double *in[32];
    double *out[16];
    double tau, eps, delta;
    int8_t *flags;
} ko_job;

static void *ko_worker(void *arg)
{
    ko_job *j = (ko_job *)arg;
    for (int64_t i = j->lo; i < j->hi; ++i) {
        if (j->kind == 3) {
            double A[6], lam[3], D[9], phi[3];
            for (int k = 0; k < 6; ++k) A[k] = j->in[k][i];
            int br = ko_eig3(A, j->tau, lam, D, phi);
            for (int k = 0; k < 3; ++k) if (j->out[k]) j->out[k][i] = lam[k];
            for (int k = 0; k < 9; ++k) if (j->out[3 + k]) j->out[3 + k][i] = D[k];
            for (int k = 0; k < 3; ++k) if (j->out[12 + k]) j->out[12 + k][i] = phi[k];
            if (j->flags) j->flags[i] = (int8_t)br;
        } else if (j->kind == 2) {
            double a[3], lam[2], D[4], phi;
            for (int k = 0; k < 3; ++k) a[k] = j->in[k][i];
            ko_eig2(a, lam, D, &phi);
            for (int k = 0; k < 2; ++k) if (j->out[k]) j->out[k][i] = lam[k];
            for (int k = 0; k < 4; ++k) if (j->out[2 + k]) j->out[2 + k][i] = D[k];
            if (j->out[6]) j->out[6][i] = phi;
        } else if (j->kind == 4) {
            double A[6], lam[3], V[9];
            long double ld[3];
            for (int k = 0; k < 6; ++k) A[k] = j->in[k][i];
            ko_jacobi3_ld(A, lam, V, ld);
            for (int k = 0; k < 3; ++k) j->out[k][i] = lam[k];
            for (int k = 0; k < 9; ++k) j->out[3 + k][i] = V[k];
            /* residual of the long-double rounding: lam_ld - (double)lam */
            for (int k = 0; k < 3; ++k)
                if (j->out[12 + k]) j->out[12 + k][i] = (double)(ld[k] - (long double)lam[k]);
        } else if (j->kind == 5) {
            double lam[3], D[9], gl[3], gD[9], ph[3], gp[3], gA[6];
            for (int k = 0; k < 3; ++k) lam[k] = j->in[k][i];
            for (int k = 0; k < 9; ++k) D[k] = j->in[3 + k][i];
            for (int k = 0; k < 3; ++k) gl[k] = j->in[12 + k] ? j->in[12 + k][i] : 0.0;
            for (int k = 0; k < 9; ++k) gD[k] = j->in[15 + k] ? j->in[15 + k][i] : 0.0;
            const int ang = j->in[24] && j->in[27];
            for (int k = 0; k < 3; ++k) ph[k] = ang ? j->in[24 + k][i] : 0.0;
            for (int k = 0; k < 3; ++k) gp[k] = ang ? j->in[27 + k][i] : 0.0;
            ko_eig3_bwd(lam, D, gl, gD, ang ? ph : NULL, ang ? gp : NULL, j->eps, j->delta, gA);
            for (int k = 0; k < 6; ++k) j->out[k][i] = gA[k];
        } else if (j->kind == 6) {
            double lam[2], D[4], gl[2], gD[4], gA[3];
            for (int k = 0; k < 2; ++k) lam[k] = j->in[k][i];
            for (int k = 0; k < 4; ++k) D[k] = j->in[2 + k][i];
            for (int k = 0; k < 2; ++k) gl[k] = j->in[6 + k] ? j->in[6 + k][i] : 0.0;
            for (int k = 0; k < 4; ++k) gD[k] = j->in[8 + k] ? j->in[8 + k][i] : 0.0;
            const double gp = j->in[12] ? j->in[12][i] : 0.0;
            ko_eig2_bwd(lam, D, gl, gD, gp, j->eps, gA);
            for (int k = 0; k < 3; ++k) j->out[k][i] = gA[k];
        } else if (j->kind == 7) {
            double lam[3], phi[3], A[6];
            for (int k = 0; k < 3; ++k) lam[k] = j->in[k][i];
            for (int k = 0; k < 3; ++k) phi[k] = j->in[3 + k][i];
            ko_compose3(lam, phi, A);
            for (int k = 0; k < 6; ++k) j->out[k][i] = A[k];
        } else if (j->kind == 8) {
            double lam[2], A[3];
            for (int k = 0; k < 2; ++k) lam[k] = j->in[k][i];
            ko_compose2(lam, j->in[2][i], A);
            for (int k = 0; k < 3; ++k) j->out[k][i] = A[k];
        }
    }
    return NULL;
}

static void run_jobs(ko_job *tmpl, int64_t n, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (n < 4096) nthreads = 1;
    pthread_t th[256];
    ko_job jobs[256];
    int64_t chunk = (n + nthreads - 1) / nthreads;
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *tmpl;
        jobs[t].lo = t * chunk;
        jobs[t].hi = (t + 1) * chunk < n ? (t + 1) * chunk : n;
        if (jobs[t].lo >= jobs[t].hi) break;
        if (nthreads == 1) {
            ko_worker(&jobs[t]);
        } else {
            pthread_create(&th[t], NULL, ko_worker, &jobs[t]);
            ++started;
        }
    }
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
}

/* in: 6 planes; out: lam[3], D[9], phi[3] (any may be NULL); flags may be NULL */
void ko_eig3_batch(int64_t n, const double *const in[6], double *const lam[3],
                   double *const D[9], double *const phi[3], int8_t *flags,
                   double tau_dbl, int nthreads)
{
    ko_job j;
    memset(&j, 0, sizeof j);
    j.kind = 3;
    for (int k = 0; k < 6; ++k) j.in[k] = in[k];
    for (int k = 0; k < 3; ++k) j.out[k] = lam ? lam[k] : NULL;
    for (int k = 0; k < 9; ++k) j.out[3 + k] = D ? D[k] : NULL;
    for (int k = 0; k < 3; ++k) j.out[12 + k] = phi ? phi[k] : NULL;
    j.flags = flags;
    j.tau = tau_dbl;
    run_jobs(&j, n, nthreads);
}

void ko_eig2_batch(int64_t n, const double *const in[3], double *const lam[2],
                   double *const D[4], double *phi, int nthreads)
{
    ko_job j;
    memset(&j, 0, sizeof j);
    j.kind = 2;
    for (int k = 0; k < 3; ++k) j.in[k] = in[k];
    for (int k = 0; k < 2; ++k) j.out[k] = lam ? lam[k] : NULL;
    for (int k = 0; k < 4; ++k) j.out[2 + k] = D ? D[k] : NULL;
    j.out[6] = phi;
    run_jobs(&j, n, nthreads);
}

void ko_jacobi3_batch(int64_t n, const double *const in[6], double *const lam[3],
                      double *const V[9], double *const lam_lo[3], int nthreads)
{
    ko_job j;
    memset(&j, 0, sizeof j);
    j.kind = 4;
    for (int k = 0; k < 6; ++k) j.in[k] = in[k];
    for (int k = 0; k < 3; ++k) j.out[k] = lam[k];
    for (int k = 0; k < 9; ++k) j.out[3 + k] = V[k];
    for (int k = 0; k < 3; ++k) j.out[12 + k] = lam_lo ? lam_lo[k] : NULL;
    run_jobs(&j, n, nthreads);
}

/* eps: absolute gap regulariser; glam / gD may be NULL (zero cotangent);
   phi and gphi (both or neither): the angle cotangents, delta the gimbal
   regulariser */
void ko_eig3_bwd_batch(int64_t n, const double *const lam[3], const double *const D[9],
                       const double *const glam[3], const double *const gD[9],
                       const double *const phi[3], const double *const gphi[3],
                       double *const gA[6], double eps, double delta, int nthreads)
{
    ko_job j;
    memset(&j, 0, sizeof j);
    j.kind = 5;
    for (int k = 0; k < 3; ++k) j.in[k] = lam[k];
    for (int k = 0; k < 9; ++k) j.in[3 + k] = D[k];
    for (int k = 0; k < 3; ++k) j.in[12 + k] = glam ? glam[k] : NULL;
    for (int k = 0; k < 9; ++k) j.in[15 + k] = gD ? gD[k] : NULL;
    for (int k = 0; k < 3; ++k) j.in[24 + k] = (phi && gphi) ? phi[k] : NULL;
    for (int k = 0; k < 3; ++k) j.in[27 + k] = (phi && gphi) ? gphi[k] : NULL;
    for (int k = 0; k < 6; ++k) j.out[k] = gA[k];
    j.eps = eps;
    j.delta = delta;
    run_jobs(&j, n, nthreads);
}

/* eps: absolute gap regulariser; glam / gD / gphi may be NULL (zero cotangent) */
void ko_eig2_bwd_batch(int64_t n, const double *const lam[2], const double *const D[4],
                       const double *const glam[2], const double *const gD[4], const double *gphi,
                       double *const gA[3], double eps, int nthreads)
{
    ko_job j;
    memset(&j, 0, sizeof j);
    j.kind = 6;
    for (int k = 0; k < 2; ++k) j.in[k] = lam[k];
    for (int k = 0; k < 4; ++k) j.in[2 + k] = D[k];
    for (int k = 0; k < 2; ++k) j.in[6 + k] = glam ? glam[k] : NULL;
    for (int k = 0; k < 4; ++k) j.in[8 + k] = gD ? gD[k] : NULL;
    j.in[12] = gphi;
    for (int k = 0; k < 3; ++k) j.out[k] = gA[k];
    j.eps = eps;
    run_jobs(&j, n, nthreads);
}

void ko_compose3_batch(int64_t n, const double *const lam[3], const double *const phi[3],
                       double *const A[6], int nthreads)
{
    ko_job j;
    memset(&j, 0, sizeof j);
    j.kind = 7;
    for (int k = 0; k < 3; ++k) j.in[k] = lam[k];
    for (int k = 0; k < 3; ++k) j.in[3 + k] = phi[k];
    for (int k = 0; k < 6; ++k) j.out[k] = A[k];
    run_jobs(&j, n, nthreads);
}

void ko_compose2_batch(int64_t n, const double *const lam[2], const double *phi, double *const A[3],
                       int nthreads)
{
    ko_job j;
    memset(&j, 0, sizeof j);
    j.kind = 8;
    for (int k = 0; k < 2; ++k) j.in[k] = lam[k];
    j.in[2] = phi;
    for (int k = 0; k < 3; ++k) j.out[k] = A[k];
    run_jobs(&j, n, nthreads);
}
