/*
 * Least-squares gradients shared by the oracle's diffusion operators (TEST
 * INFRASTRUCTURE ONLY; see oracle.h): an unweighted fit of a polynomial in
 * mesh-unit offsets from the evaluation point, quadratic (10 terms, or 9
 * when the value at the point is prescribed) with a linear fallback when the
 * points are too few or the normal matrix too poorly conditioned
 * (reciprocal 1-norm condition number below 1e-7).
 */
#ifndef EBS_ORACLE_LSQ_H
#define EBS_ORACLE_LSQ_H

#include <math.h>

/* Solve the n x n system M x = r (n <= 10) by Gaussian elimination with
 * partial pivoting; also the 1-norm reciprocal condition number from the
 * explicit inverse.  Returns 0 if singular. */
static int solve_n(int n, const double Min[10][10], const double rin[10], double x[10], double* rcond) {
    double A[10][10], I[10][10], r[10];
    for (int a = 0; a < n; ++a) {
        r[a] = rin[a];
        for (int b = 0; b < n; ++b) {
            A[a][b] = Min[a][b];
            I[a][b] = a == b ? 1.0 : 0.0;
        }
    }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int a = col + 1; a < n; ++a)
            if (fabs(A[a][col]) > fabs(A[piv][col])) piv = a;
        if (!(fabs(A[piv][col]) > 0.0)) return 0;
        if (piv != col) {
            for (int b = 0; b < n; ++b) {
                double t = A[col][b]; A[col][b] = A[piv][b]; A[piv][b] = t;
                t = I[col][b]; I[col][b] = I[piv][b]; I[piv][b] = t;
            }
            double t = r[col]; r[col] = r[piv]; r[piv] = t;
        }
        const double p = A[col][col];
        for (int b = 0; b < n; ++b) { A[col][b] /= p; I[col][b] /= p; }
        r[col] /= p;
        for (int a = 0; a < n; ++a) {
            if (a == col) continue;
            const double f = A[a][col];
            for (int b = 0; b < n; ++b) { A[a][b] -= f * A[col][b]; I[a][b] -= f * I[col][b]; }
            r[a] -= f * r[col];
        }
    }
    double n1 = 0.0, ni = 0.0;
    for (int b = 0; b < n; ++b) {
        double ca = 0.0, cb = 0.0;
        for (int a = 0; a < n; ++a) { ca += fabs(Min[a][b]); cb += fabs(I[a][b]); }
        n1 = fmax(n1, ca);
        ni = fmax(ni, cb);
    }
    *rcond = 1.0 / (n1 * ni);
    for (int a = 0; a < n; ++a) x[a] = r[a];
    return 1;
}

/* basis row of a point at mesh-unit offset e from the evaluation point:
 * with_const: 1, e, e^2 terms (10); without: e, e^2 terms (9) */
static int basis(const double e[3], int quad, int with_const, double row[10]) {
    int n = 0;
    if (with_const) row[n++] = 1.0;
    row[n++] = e[0];
    row[n++] = e[1];
    row[n++] = e[2];
    if (quad) {
        row[n++] = 0.5 * e[0] * e[0];
        row[n++] = 0.5 * e[1] * e[1];
        row[n++] = 0.5 * e[2] * e[2];
        row[n++] = e[0] * e[1];
        row[n++] = e[0] * e[2];
        row[n++] = e[1] * e[2];
    }
    return n;
}

/* Least-squares gradient (physical units) at point x (physical) from the
 * points P (offsets in mesh units) with values q; with_const = 0 fits
 * q - q_wall with no constant term.  Quadratic, then linear fallback. */
static void lsq_gradient(const double dx[3], int np, double (*e)[3], const double* q, int with_const, double grad[3]) {
    grad[0] = grad[1] = grad[2] = 0.0;
    for (int quad = 1; quad >= 0; --quad) {
        double row[10];
        const int nb = basis(e[0], quad, with_const, row);
        if (np < nb) continue;
        double M[10][10] = {{0}}, r[10] = {0};
        for (int s = 0; s < np; ++s) {
            basis(e[s], quad, with_const, row);
            for (int a = 0; a < nb; ++a) {
                r[a] += row[a] * q[s];
                for (int b = 0; b < nb; ++b) M[a][b] += row[a] * row[b];
            }
        }
        double x[10], rc;
        if (!solve_n(nb, M, r, x, &rc)) continue;
        if (!(rc >= 1e-7)) continue;
        const int o = with_const ? 1 : 0;
        for (int d = 0; d < 3; ++d) grad[d] = x[o + d] / dx[d];
        return;
    }
}

#endif
