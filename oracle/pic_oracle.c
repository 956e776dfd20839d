/*
 * pic_oracle.c - plain FP64 CPU oracle of the explicit relativistic PIC cycle of
 * Melzani et al., "Apar-T: code, validation, and physical interpretation of
 * particle-in-cell results" (arXiv:1308.5892).
 *
 * TEST INFRASTRUCTURE. This is the slow, obviously-correct reference that the
 * GPU path is checked against. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product never does, and this
 * file shares no code, header or table with the GPU library.
 *
 * Everything is double precision and in the paper's normalised units
 * (App. A.2): lengths in cells X0, times in X0/c, e and b = cB in
 * m_e c^2/(e X0), u = gamma v / c.  Species s carries k_s = (q_s/e)(m_e/m_s)
 * (normalised equation of motion, App. A.2) and couples to e through
 * alpha_s = sgn(q_s) alpha0 with alpha0 = 2/(n_x^2 rho0) (App. A.2, eq. alpha).
 *
 * Grid (App. A.3.2 and the averaging stencils of App. A.3.3): nodes at integer
 * points; e_x[i,j,k] sits at (i+1/2,j,k), e_y at (i,j+1/2,k), e_z at (i,j,k+1/2);
 * b_x at (i,j+1/2,k+1/2), b_y at (i+1/2,j,k+1/2), b_z at (i+1/2,j+1/2,k); the
 * current j_c sits where e_c sits (App. A.3.4).  All indices are periodic.
 * A field array holds three components of n = nx*ny*nz values each, component
 * c at [c*n + i + nx*(j + ny*k)].
 *
 * Readings of the paper taken where it is silent or garbled are marked
 * READING in the comments.
 *
 * Parity status: every function below is pinned by a CPU test (closed forms,
 * brute force, printed values, a library Philox, Monte-Carlo moments); see the
 * tests directory.
 *
 * Threads: built with OpenMP (only for timing the oracle on all host cores),
 * the independent per-particle loops of the loader, the backward half step
 * and the cycle run in parallel, and the deposit sums into one current array
 * per thread, added in thread order; built without it (the parity build),
 * every loop runs in order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ grid */

static int wrapi(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

static int64_t cell_index(const int g[3], int i, int j, int k)
{
    i = wrapi(i, g[0]);
    j = wrapi(j, g[1]);
    k = wrapi(k, g[2]);
    return (int64_t)i + (int64_t)g[0] * ((int64_t)j + (int64_t)g[1] * k);
}

static int64_t ncells(const int g[3])
{
    return (int64_t)g[0] * g[1] * g[2];
}

/* F[c] at node-offset (di,dj,dk) from (i,j,k), component c */
static double at(const double *F, const int g[3], int c, int i, int j, int k)
{
    return F[c * ncells(g) + cell_index(g, i, j, k)];
}

/* ------------------------------------------------------------- Yee (A.3.2) */

/*
 * curl e evaluated at the b positions (App. A.3.2; the printed b_x update
 * b_x += dt (e_y[k+1] - e_y[k] - e_z[j+1] + e_z[j]) is b_x -= dt (curl e)_x).
 */
void orc_curl_e(const int g[3], const double *e, double *out)
{
    int64_t n = ncells(g);
    for (int k = 0; k < g[2]; ++k)
        for (int j = 0; j < g[1]; ++j)
            for (int i = 0; i < g[0]; ++i) {
                int64_t p = cell_index(g, i, j, k);
                /* (curl e)_x at (i, j+1/2, k+1/2) = d_y e_z - d_z e_y */
                out[0 * n + p] = (at(e, g, 2, i, j + 1, k) - at(e, g, 2, i, j, k))
                               - (at(e, g, 1, i, j, k + 1) - at(e, g, 1, i, j, k));
                /* (curl e)_y at (i+1/2, j, k+1/2) = d_z e_x - d_x e_z */
                out[1 * n + p] = (at(e, g, 0, i, j, k + 1) - at(e, g, 0, i, j, k))
                               - (at(e, g, 2, i + 1, j, k) - at(e, g, 2, i, j, k));
                /* (curl e)_z at (i+1/2, j+1/2, k) = d_x e_y - d_y e_x */
                out[2 * n + p] = (at(e, g, 1, i + 1, j, k) - at(e, g, 1, i, j, k))
                               - (at(e, g, 0, i, j + 1, k) - at(e, g, 0, i, j, k));
            }
}

/* curl b evaluated at the e positions (App. A.3.2, "similarly for e"). */
void orc_curl_b(const int g[3], const double *b, double *out)
{
    int64_t n = ncells(g);
    for (int k = 0; k < g[2]; ++k)
        for (int j = 0; j < g[1]; ++j)
            for (int i = 0; i < g[0]; ++i) {
                int64_t p = cell_index(g, i, j, k);
                /* (curl b)_x at (i+1/2, j, k) = d_y b_z - d_z b_y */
                out[0 * n + p] = (at(b, g, 2, i, j, k) - at(b, g, 2, i, j - 1, k))
                               - (at(b, g, 1, i, j, k) - at(b, g, 1, i, j, k - 1));
                /* (curl b)_y at (i, j+1/2, k) = d_z b_x - d_x b_z */
                out[1 * n + p] = (at(b, g, 0, i, j, k) - at(b, g, 0, i, j, k - 1))
                               - (at(b, g, 2, i, j, k) - at(b, g, 2, i - 1, j, k));
                /* (curl b)_z at (i, j, k+1/2) = d_x b_y - d_y b_x */
                out[2 * n + p] = (at(b, g, 1, i, j, k) - at(b, g, 1, i - 1, j, k))
                               - (at(b, g, 0, i, j, k) - at(b, g, 0, i, j - 1, k));
            }
}

/* b <- b - h * curl e  (a half advance uses h = dt/2; App. A.3.1 steps 1, 4) */
void orc_advance_b(const int g[3], double h, const double *e, double *b)
{
    int64_t n3 = 3 * ncells(g);
    double *c = (double *)malloc(sizeof(double) * n3);
    orc_curl_e(g, e, c);
    for (int64_t p = 0; p < n3; ++p)
        b[p] -= h * c[p];
    free(c);
}

/*
 * Fourth-order curl of e at the b positions, for the fourth-order field
 * solver the paper adds against numerical Cerenkov emission (App. A.3.2,
 * last paragraph; App. B, third item).  READING (the paper names the solver
 * but prints no stencil): every difference along an axis is the staggered
 * fourth-order one,
 *   d_a f (x) = (9/8) (f(x + 1/2) - f(x - 1/2)) - (1/24) (f(x + 3/2) - f(x - 3/2)),
 * and only Faraday's law uses it; Ampere's law keeps the second-order curl,
 * so the discrete divergence of e (second order) still changes only by the
 * charge-conserving current and Gauss's law holds as with Yee.
 */
static double d4(const double *F, const int g[3], int c, int i, int j, int k, int a)
{
    /* d_a of component c at the point half a cell above (i,j,k) along a */
    int o[3] = {0, 0, 0};
    o[a] = 1;
    double near = at(F, g, c, i + o[0], j + o[1], k + o[2]) - at(F, g, c, i, j, k);
    double far = at(F, g, c, i + 2 * o[0], j + 2 * o[1], k + 2 * o[2])
               - at(F, g, c, i - o[0], j - o[1], k - o[2]);
    return 9.0 / 8.0 * near - 1.0 / 24.0 * far;
}

void orc_curl_e4(const int g[3], const double *e, double *out)
{
    int64_t n = ncells(g);
    for (int k = 0; k < g[2]; ++k)
        for (int j = 0; j < g[1]; ++j)
            for (int i = 0; i < g[0]; ++i) {
                int64_t p = cell_index(g, i, j, k);
                /* (curl e)_x at (i, j+1/2, k+1/2) = d_y e_z - d_z e_y */
                out[0 * n + p] = d4(e, g, 2, i, j, k, 1) - d4(e, g, 1, i, j, k, 2);
                /* (curl e)_y at (i+1/2, j, k+1/2) = d_z e_x - d_x e_z */
                out[1 * n + p] = d4(e, g, 0, i, j, k, 2) - d4(e, g, 2, i, j, k, 0);
                /* (curl e)_z at (i+1/2, j+1/2, k) = d_x e_y - d_y e_x */
                out[2 * n + p] = d4(e, g, 1, i, j, k, 0) - d4(e, g, 0, i, j, k, 1);
            }
}

/* b <- b - h * curl e with the fourth-order curl (orc_curl_e4) */
void orc_advance_b4(const int g[3], double h, const double *e, double *b)
{
    int64_t n3 = 3 * ncells(g);
    double *c = (double *)malloc(sizeof(double) * n3);
    orc_curl_e4(g, e, c);
    for (int64_t p = 0; p < n3; ++p)
        b[p] -= h * c[p];
    free(c);
}

/* Faraday half or full advance with the solver's curl of e */
static void advance_b_order(const int g[3], double h, const double *e, double *b, int faraday4)
{
    if (faraday4) orc_advance_b4(g, h, e, b);
    else orc_advance_b(g, h, e, b);
}

/* e <- e + h * curl b  (full advance with h = dt; App. A.3.1 step 6) */
void orc_advance_e(const int g[3], double h, const double *b, double *e)
{
    int64_t n3 = 3 * ncells(g);
    double *c = (double *)malloc(sizeof(double) * n3);
    orc_curl_b(g, b, c);
    for (int64_t p = 0; p < n3; ++p)
        e[p] += h * c[p];
    free(c);
}

/* ------------------------------------------------------ gather (A.3.3) */

/*
 * Field at node (i,j,k).  The paper prints E_x^n = (e_x[i-1]+e_x[i])/2 and
 * B_z^n = (b_z[i,j]+b_z[i-1,j]+b_z[i-1,j-1]+b_z[i,j-1])/4.
 * READING: the other components by cyclic permutation - e_c averaged over the
 * two edges along c that meet at the node, b_c over the four faces normal to c
 * that meet at it.
 */
static void node_fields(const int g[3], const double *e, const double *b,
                        int i, int j, int k, double E[3], double B[3])
{
    E[0] = 0.5 * (at(e, g, 0, i - 1, j, k) + at(e, g, 0, i, j, k));
    E[1] = 0.5 * (at(e, g, 1, i, j - 1, k) + at(e, g, 1, i, j, k));
    E[2] = 0.5 * (at(e, g, 2, i, j, k - 1) + at(e, g, 2, i, j, k));
    B[0] = 0.25 * (at(b, g, 0, i, j, k) + at(b, g, 0, i, j - 1, k)
                 + at(b, g, 0, i, j - 1, k - 1) + at(b, g, 0, i, j, k - 1));
    B[1] = 0.25 * (at(b, g, 1, i, j, k) + at(b, g, 1, i, j, k - 1)
                 + at(b, g, 1, i - 1, j, k - 1) + at(b, g, 1, i - 1, j, k));
    B[2] = 0.25 * (at(b, g, 2, i, j, k) + at(b, g, 2, i - 1, j, k)
                 + at(b, g, 2, i - 1, j - 1, k) + at(b, g, 2, i, j - 1, k));
}

/*
 * Trilinear (volume) weighting of the node fields at x (App. A.3.3): with
 * x = i + dx, node (i+a, j+b, k+c) gets weight W_x^a W_y^b W_z^c, W^0 = 1-d,
 * W^1 = d - the overlap of the unit cube centred on x with the grid-B cell
 * centred on that node.
 */
void orc_gather(const int g[3], const double *e, const double *b,
                const double x[3], double E[3], double B[3])
{
    int c0[3];
    double w[3][2];
    for (int a = 0; a < 3; ++a) {
        double f = floor(x[a]);
        c0[a] = (int)f;
        double d = x[a] - f;
        w[a][0] = 1.0 - d;
        w[a][1] = d;
    }
    E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = 0.0;
    for (int kk = 0; kk < 2; ++kk)
        for (int jj = 0; jj < 2; ++jj)
            for (int ii = 0; ii < 2; ++ii) {
                double En[3], Bn[3];
                node_fields(g, e, b, c0[0] + ii, c0[1] + jj, c0[2] + kk, En, Bn);
                double wt = w[0][ii] * w[1][jj] * w[2][kk];
                for (int a = 0; a < 3; ++a) {
                    E[a] += wt * En[a];
                    B[a] += wt * Bn[a];
                }
            }
}

/* ------------------------------------------------------- mover (A.3.3) */

static void cross(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/*
 * Relativistic Boris step u^{t-h/2} -> u^{t+h/2} in fields E, B for a species
 * with k = (q/e)(m_e/m) (App. A.3.3, eq. mover): half electric kick, rotation
 * about b, half electric kick; gamma^t = sqrt(1 + |u^-|^2).
 * READING: the printed rotation formula is garbled; the rotation is the
 * standard one with t = (k h / (2 gamma)) B and s = 2 t / (1 + |t|^2), which
 * solves (u+ - u-)/h = k/(2 gamma) (u+ + u-) x B exactly.
 */
void orc_boris(double k, double h, const double E[3], const double B[3], double u[3])
{
    double um[3], t[3], s[3], up[3], c1[3], c2[3];
    for (int a = 0; a < 3; ++a)
        um[a] = u[a] + 0.5 * k * h * E[a];
    double gam = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int a = 0; a < 3; ++a)
        t[a] = 0.5 * k * h * B[a] / gam;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int a = 0; a < 3; ++a)
        s[a] = 2.0 * t[a] / (1.0 + t2);
    cross(um, t, c1);
    for (int a = 0; a < 3; ++a)
        up[a] = um[a] + c1[a];
    cross(up, s, c2);
    for (int a = 0; a < 3; ++a)
        u[a] = um[a] + c2[a] + 0.5 * k * h * E[a];
}

/* ------------------------------------------------- current (A.1, A.3.4) */

/*
 * Deposit of one straight sub-move that stays in the unit cell c (start offset
 * d0 in [0,1]^3, displacement D, end offset d0+D in [0,1]^3): the volume change
 * of the particle cube in each of the 8 grid-B cells around c, attributed per
 * component as in App. A.3.4 (eq. current_dep):
 *   dV_x[c + eta y + xi z] = -D_x (W_y^eta W_z^xi + sigma D_y D_z / 12),
 * W^0 = 1 - d0 - D/2, W^1 = d0 + D/2, sigma = +1 if eta == xi else -1, and
 * cyclically for y and z (12 values).  The (0,0) term is the printed one; the
 * others follow from the same expansion of the product of overlaps.
 * J accumulates sgn * dV (a volume), placed where e_c sits.
 */
static void deposit_in_cell(const int g[3], double sgn, const int c[3],
                            const double d0[3], const double D[3], double *J)
{
    int64_t n = ncells(g);
    for (int a = 0; a < 3; ++a) {
        int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
        double w1[2] = {1.0 - d0[b1] - 0.5 * D[b1], d0[b1] + 0.5 * D[b1]};
        double w2[2] = {1.0 - d0[b2] - 0.5 * D[b2], d0[b2] + 0.5 * D[b2]};
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) {
                double sigma = (p == q) ? 1.0 : -1.0;
                double dv = -D[a] * (w1[p] * w2[q] + sigma * D[b1] * D[b2] / 12.0);
                int idx3[3] = {c[0], c[1], c[2]};
                idx3[b1] += p;
                idx3[b2] += q;
                J[a * n + cell_index(g, idx3[0], idx3[1], idx3[2])] += sgn * dv;
            }
    }
}

/*
 * Charge-conserving deposit of the straight move x0 -> x1 (|x1 - x0| < 1 per
 * axis; x1 not wrapped).  READING (the paper refers the cell-crossing case to
 * references that are not given): the segment is cut at every integer plane it
 * crosses, in order of the crossing parameter lambda, and each piece is
 * deposited in the cell that contains it.  An axis crosses iff floor(x0) !=
 * floor(x1); its plane is max(floor(x0), floor(x1)).  Breakpoints put the
 * crossing coordinate exactly on its plane.  Returns the number of pieces.
 */
int orc_deposit_move(const int g[3], double sgn, const double x0[3],
                     const double x1[3], double *J)
{
    double lam[3];
    int ax[3], nb = 0;
    double plane[3];
    int crossed[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        double f0 = floor(x0[a]), f1 = floor(x1[a]);
        if (f0 != f1) {
            plane[a] = f0 > f1 ? f0 : f1;
            lam[nb] = (plane[a] - x0[a]) / (x1[a] - x0[a]);
            ax[nb] = a;
            ++nb;
        }
    }
    /* sort breakpoints by lambda (at most three) */
    for (int p = 0; p < nb; ++p)
        for (int q = p + 1; q < nb; ++q)
            if (lam[q] < lam[p]) {
                double tl = lam[p]; lam[p] = lam[q]; lam[q] = tl;
                int ta = ax[p]; ax[p] = ax[q]; ax[q] = ta;
            }
    double pts[5][3];
    for (int a = 0; a < 3; ++a) {
        pts[0][a] = x0[a];
        pts[nb + 1][a] = x1[a];
    }
    for (int p = 0; p < nb; ++p) {
        crossed[ax[p]] = 1;
        for (int a = 0; a < 3; ++a) {
            if (a == ax[p]) {
                pts[p + 1][a] = plane[a];
                continue;
            }
            double v = x0[a] + lam[p] * (x1[a] - x0[a]);
            /* keep a not-yet-crossed (or already crossed) coordinate on its
             * side of its own plane despite rounding */
            if (floor(x0[a]) != floor(x1[a])) {
                int up = x1[a] > x0[a];
                if (!crossed[a]) v = up ? fmin(v, plane[a]) : fmax(v, plane[a]);
                else v = up ? fmax(v, plane[a]) : fmin(v, plane[a]);
            }
            pts[p + 1][a] = v;
        }
    }
    for (int p = 0; p <= nb; ++p) {
        int c[3];
        double d0[3], D[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = (int)floor(0.5 * (pts[p][a] + pts[p + 1][a]));
            d0[a] = pts[p][a] - c[a];
            D[a] = pts[p + 1][a] - pts[p][a];
        }
        deposit_in_cell(g, sgn, c, d0, D, J);
    }
    return nb + 1;
}

/* CIC weight (overlap volume) of a particle at x on every node: adds sgn*W. */
void orc_deposit_charge(const int g[3], double sgn, const double x[3], double *rho)
{
    int c0[3];
    double w[3][2];
    for (int a = 0; a < 3; ++a) {
        double f = floor(x[a]);
        c0[a] = (int)f;
        w[a][1] = x[a] - f;
        w[a][0] = 1.0 - w[a][1];
    }
    for (int kk = 0; kk < 2; ++kk)
        for (int jj = 0; jj < 2; ++jj)
            for (int ii = 0; ii < 2; ++ii)
                rho[cell_index(g, c0[0] + ii, c0[1] + jj, c0[2] + kk)] +=
                    sgn * w[0][ii] * w[1][jj] * w[2][kk];
}

/* ----------------------------------------------------- main loop (A.3.1) */

static double wrapd(double x, int n)
{
    double r = fmod(x, (double)n);
    if (r < 0.0) r += n;
    if (r >= n) r -= n;
    return r;
}

/*
 * Perfectly conducting walls at the two box faces normal to axis w (App. A.4:
 * the normal b and the tangential e vanish at a conductor's surface).  Both
 * faces lie on the node plane of index 0 along w (index N wraps onto it), so
 * the condition is: b_w = 0 and e_c = 0 (c != w) on that plane.  The Yee
 * values there are then never used across the wall.
 */
void orc_wall_fields(const int g[3], int w, double *e, double *b)
{
    int64_t n = ncells(g);
    for (int k = 0; k < g[2]; ++k)
        for (int j = 0; j < g[1]; ++j)
            for (int i = 0; i < g[0]; ++i) {
                int idx[3] = {i, j, k};
                if (idx[w] != 0) continue;
                int64_t p = cell_index(g, i, j, k);
                b[w * n + p] = 0.0;
                for (int c = 0; c < 3; ++c)
                    if (c != w) e[c * n + p] = 0.0;
            }
}

/*
 * Smoothing of the current (App. A.3.4, last paragraph): each value of a grid
 * becomes the weighted sum of the 27 values around it - weight 1 for itself,
 * 1/2 for its 6 face neighbours, 1/4 for its 12 edge neighbours, 1/8 for its 8
 * corner neighbours - with the weights normalised to sum to one (their sum is
 * 8).  Periodic; applied to each of the ncomp component grids of f in place.
 */
void orc_filter27(const int g[3], int ncomp, double *f)
{
    int64_t n = ncells(g);
    double *t = (double *)malloc(sizeof(double) * n);
    for (int c = 0; c < ncomp; ++c) {
        double *fc = f + (int64_t)c * n;
        memcpy(t, fc, sizeof(double) * n);
        for (int k = 0; k < g[2]; ++k)
            for (int j = 0; j < g[1]; ++j)
                for (int i = 0; i < g[0]; ++i) {
                    double sum = 0.0;
                    for (int dk = -1; dk <= 1; ++dk)
                        for (int dj = -1; dj <= 1; ++dj)
                            for (int di = -1; di <= 1; ++di) {
                                int m = abs(di) + abs(dj) + abs(dk);   /* 0 self, 1 face, 2 edge, 3 corner */
                                double w = m == 0 ? 1.0 : (m == 1 ? 0.5 : (m == 2 ? 0.25 : 0.125));
                                sum += w * t[cell_index(g, i + di, j + dj, k + dk)];
                            }
                    fc[cell_index(g, i, j, k)] = sum / 8.0;
                }
    }
    free(t);
}

/*
 * nsteps leap-frog cycles (App. A.3.1).  On entry x and e are at time t, u and
 * b at t - dt/2; on return they have advanced by nsteps*dt.
 * Particles: x[3p..3p+2] in [0, N), u likewise, species[p] in [0, nsp).
 * kq[s] = (q_s/e)(m_e/m_s), sgn[s] = sgn(q_s), alpha0 = 2/(n_x^2 rho0).
 * filter != 0 smooths the current (orc_filter27) before it enters e.
 * wall in {0, 1, 2} puts perfectly conducting walls at the two box faces
 * normal to that axis (App. A.4; see orc_wall_fields and the move below);
 * wall = -1: every boundary is periodic.
 * faraday4 != 0 advances b with the fourth-order curl of e (orc_curl_e4).
 */
void orc_step(const int g[3], double dt, double alpha0, int nsp,
              const double *kq, const double *sgn, int64_t np,
              const int32_t *species, double *x, double *u,
              double *e, double *b, int nsteps, int filter, int wall, int faraday4)
{
    int64_t n = ncells(g);
    double *J = (double *)malloc(sizeof(double) * 3 * n);
    double *xold = (double *)malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
    (void)nsp;
    double *xwall = (double *)malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
    char *hit = (char *)calloc((size_t)(np > 0 ? np : 1), 1);
#ifdef _OPENMP
    const int nthr = omp_get_max_threads();
    double *Jt = (double *)malloc(sizeof(double) * 3 * n * (size_t)nthr);
#endif
    for (int it = 0; it < nsteps; ++it) {
        /* 1. b^{t-dt/2} -> b^t */
        advance_b_order(g, 0.5 * dt, e, b, faraday4);
        if (wall >= 0) orc_wall_fields(g, wall, e, b);
        /* 2-3. velocity with e^t, b^t at x^t; then position to t+dt */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int64_t p = 0; p < np; ++p) {
            double E[3], B[3];
            int s = species[p];
            orc_gather(g, e, b, &x[3 * p], E, B);
            orc_boris(kq[s], dt, E, B, &u[3 * p]);
            double *up = &u[3 * p];
            double ig = 1.0 / sqrt(1.0 + up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
            double D[3];
            for (int a = 0; a < 3; ++a) {
                xold[3 * p + a] = x[3 * p + a];
                D[a] = dt * up[a] * ig;
                x[3 * p + a] += D[a];
            }
            hit[p] = 0;
            if (wall >= 0) {
                /* READING of the particle reflection (App. A.4): a move that
                 * leaves through a wall is cut where it meets the wall; the rest
                 * of it is mirrored back into the box and the normal momentum
                 * changes sign.  The current is that of the two straight
                 * pieces. */
                double *xp = &x[3 * p];
                double N = g[wall], xw = xp[wall];
                if (xw < 0.0 || xw >= N) {
                    double plane = xw < 0.0 ? 0.0 : N;
                    double lam = (plane - xold[3 * p + wall]) / D[wall];
                    for (int a = 0; a < 3; ++a) xwall[3 * p + a] = xold[3 * p + a] + lam * D[a];
                    xwall[3 * p + wall] = plane;
                    double xr = 2.0 * plane - xw;
                    if (xr >= N) xr = nextafter(N, 0.0);   /* a move ending on the upper wall */
                    xp[wall] = xr;
                    up[wall] = -up[wall];
                    hit[p] = 1;
                }
            }
        }
        /* 4. b^t -> b^{t+dt/2} */
        advance_b_order(g, 0.5 * dt, e, b, faraday4);
        if (wall >= 0) orc_wall_fields(g, wall, e, b);
        /* 6. e^t -> e^{t+dt} with curl b^{t+dt/2} */
        orc_advance_e(g, dt, b, e);
        /* 9. currents from the moves x^t -> x^{t+dt} (READING: the appendix's
         *    old position plus displacement, not item 9's wording) */
        memset(J, 0, sizeof(double) * 3 * n);
#ifdef _OPENMP
#pragma omp parallel
        {
            double *Jm = Jt + (size_t)omp_get_thread_num() * 3 * n;
            memset(Jm, 0, sizeof(double) * 3 * n);
#pragma omp for schedule(static)
            for (int64_t p = 0; p < np; ++p) {
                if (hit[p]) {
                    orc_deposit_move(g, sgn[species[p]], &xold[3 * p], &xwall[3 * p], Jm);
                    orc_deposit_move(g, sgn[species[p]], &xwall[3 * p], &x[3 * p], Jm);
                } else {
                    orc_deposit_move(g, sgn[species[p]], &xold[3 * p], &x[3 * p], Jm);
                }
            }
        }
        /* the per-thread currents added in thread order */
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < 3 * n; ++q) {
            double v = 0.0;
            for (int t = 0; t < nthr; ++t) v += Jt[(size_t)t * 3 * n + q];
            J[q] = v;
        }
#else
        for (int64_t p = 0; p < np; ++p) {
            if (hit[p]) {
                orc_deposit_move(g, sgn[species[p]], &xold[3 * p], &xwall[3 * p], J);
                orc_deposit_move(g, sgn[species[p]], &xwall[3 * p], &x[3 * p], J);
            } else {
                orc_deposit_move(g, sgn[species[p]], &xold[3 * p], &x[3 * p], J);
            }
        }
#endif
        /* 10. optional smoothing of the current (App. A.3.4) */
        if (filter) orc_filter27(g, 3, J);
        /* 12. e += alpha0 * sum_s sgn_s dV  (App. A.2, eq. max2bis) */
        for (int64_t q = 0; q < 3 * n; ++q)
            e[q] += alpha0 * J[q];
        if (wall >= 0) orc_wall_fields(g, wall, e, b);
        /* 8. periodic particle boundary */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int64_t p = 0; p < np; ++p)
            for (int a = 0; a < 3; ++a)
                x[3 * p + a] = wrapd(x[3 * p + a], g[a]);
    }
#ifdef _OPENMP
    free(Jt);
#endif
    free(hit);
    free(xwall);
    free(xold);
    free(J);
}

/*
 * READING of the initial backward half step (App. A.3.1): u is integrated by
 * -dt/2 with one Boris step in the t=0 fields.  The field half step
 * b^{-dt/2} = b^0 + (dt/2) curl e^0 is orc_advance_b with h = -dt/2.
 */
void orc_backward_half(const int g[3], double dt, const double *kq, int64_t np,
                       const int32_t *species, const double *x, double *u,
                       const double *e, const double *b0)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t p = 0; p < np; ++p) {
        double E[3], B[3];
        orc_gather(g, e, b0, &x[3 * p], E, B);
        orc_boris(kq[species[p]], -0.5 * dt, E, B, &u[3 * p]);
    }
}

/* threads used by the parallel build (n > 0 sets them); 1 without OpenMP */
int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------ diagnostics */

/*
 * Diagnostics at time t from the stored state (x^t, u^{t-dt/2}, e^t,
 * b^{t-dt/2}); all sums in FP64.  out layout:
 *   [0..2]  W_E,c = (1/alpha0) sum 1/2 e_c^2        (energy unit of Fig. fluctuations, Sect. 5.3)
 *   [3..5]  W_B,c = (1/alpha0) sum 1/2 (b^t)_c^2, b^t = b - (dt/2) curl e
 *   [6]     max |div e - rho|,  [7] rms of the same,
 *           rho = alpha0 sum_s sgn_s sum_p W(x_p), smoothed like the
 *           current when filter != 0; with walls (wall >= 0) the nodes on
 *           the wall plane (the conductor's surface charge) are left out
 *   then per species s (8 + 6 s): K_s = sum (m_s/m_e)(gamma^t - 1),
 *           P_s[3] = sum u^-, count, sum (gamma^t - 1)
 * READING (the paper does not say at which time it evaluates the energies):
 * gamma^t = sqrt(1 + |u^-|^2), u^- = u^{t-dt/2} + (k dt/2) E(x^t) - the same
 * gamma^t the mover uses.
 * hist (optional, nsp x nbins): counts of log10(gamma^t - 1) in [lo, hi),
 * clamped to the end bins.  faraday4: b^t is formed with the fourth-order
 * curl of e, as the cycle forms it.
 */
void orc_diag(const int g[3], double dt, double alpha0, int nsp, const double *kq,
              const double *sgn, const double *m_over_me, int64_t np,
              const int32_t *species, const double *x, const double *u,
              const double *e, const double *b, double *out,
              int nbins, double lo, double hi, int64_t *hist, int filter, int wall, int faraday4)
{
    int64_t n = ncells(g);
    double *bt = (double *)malloc(sizeof(double) * 3 * n);
    double *rho = (double *)calloc((size_t)n, sizeof(double));
    memcpy(bt, b, sizeof(double) * 3 * n);
    advance_b_order(g, 0.5 * dt, e, bt, faraday4);
    for (int c = 0; c < 3; ++c) {
        double we = 0.0, wb = 0.0;
        for (int64_t p = 0; p < n; ++p) {
            we += 0.5 * e[c * n + p] * e[c * n + p];
            wb += 0.5 * bt[c * n + p] * bt[c * n + p];
        }
        out[c] = we / alpha0;
        out[3 + c] = wb / alpha0;
    }
    for (int s = 0; s < nsp; ++s)
        for (int q = 0; q < 6; ++q)
            out[8 + 6 * s + q] = 0.0;
    if (hist) memset(hist, 0, sizeof(int64_t) * nsp * nbins);
    for (int64_t p = 0; p < np; ++p) {
        int s = species[p];
        double E[3], B[3], um[3];
        orc_gather(g, e, bt, &x[3 * p], E, B);
        for (int a = 0; a < 3; ++a)
            um[a] = u[3 * p + a] + 0.5 * kq[s] * dt * E[a];
        double gam = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
        double *o = &out[8 + 6 * s];
        o[0] += m_over_me[s] * (gam - 1.0);
        o[1] += um[0];
        o[2] += um[1];
        o[3] += um[2];
        o[4] += 1.0;
        o[5] += gam - 1.0;
        if (hist && nbins > 0) {
            double v = log10(gam - 1.0 > 1e-300 ? gam - 1.0 : 1e-300);
            int bin = (int)floor((v - lo) / (hi - lo) * nbins);
            if (bin < 0) bin = 0;
            if (bin >= nbins) bin = nbins - 1;
            hist[s * nbins + bin] += 1;
        }
        orc_deposit_charge(g, sgn[s] * alpha0, &x[3 * p], rho);
    }
    /* with a smoothed current, the conserved charge is the smoothed one */
    if (filter) orc_filter27(g, 1, rho);
    double rmax = 0.0, rsum = 0.0;
    for (int k = 0; k < g[2]; ++k)
        for (int j = 0; j < g[1]; ++j)
            for (int i = 0; i < g[0]; ++i) {
                double div = at(e, g, 0, i, j, k) - at(e, g, 0, i - 1, j, k)
                           + at(e, g, 1, i, j, k) - at(e, g, 1, i, j - 1, k)
                           + at(e, g, 2, i, j, k) - at(e, g, 2, i, j, k - 1);
                double r = div - rho[cell_index(g, i, j, k)];
                int idx[3] = {i, j, k};
                if (wall >= 0 && idx[wall] == 0) r = 0.0;   /* the conductor's surface charge */
                if (fabs(r) > rmax) rmax = fabs(r);
                rsum += r * r;
            }
    out[6] = rmax;
    out[7] = sqrt(rsum / (double)n);
    free(rho);
    free(bt);
}

/* ------------------------------------------------ Philox4x64-10 generator */

/*
 * Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11),
 * Philox-4x64 with 10 rounds, written from its published definition: each
 * round multiplies words 0 and 2 by two fixed odd constants, keeps the 128-bit
 * products' halves, xors the high halves with words 1 and 3 and the key; the
 * key is bumped by two Weyl constants between rounds.
 */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c[0], &hi0, &lo0);
        mulhilo64(M1, c[2], &hi1, &lo1);
        uint64_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

static double u01(uint64_t w) /* [0, 1) with 53 random bits */
{
    return (double)(w >> 11) * 0x1.0p-53;
}

/* --------------------------------------- Maxwell-Juettner loader (App. D) */

/*
 * Unnormalised marginal density of p_y for the drifting Maxwell-Juttner
 * distribution (App. D, eq. distr_y), divided by its peak exponential so that
 * it is O(1) at y = Gamma0 beta0:
 *   j(y) ~ (1 + mu G gy) exp(-mu G (gy - beta0 y) + mu),  gy = sqrt(1 + y^2).
 */
static double jy_shape(double y, double mu, double G, double beta0)
{
    double gy = sqrt(1.0 + y * y);
    return (1.0 + mu * G * gy) * exp(-mu * G * (gy - beta0 * y) + mu);
}

/* 8-point Gauss-Legendre integral of jy_shape over [a, b] */
static double gl8(double a, double b, double mu, double G, double beta0)
{
    static const double xg[4] = {0.1834346424956498, 0.5255324099163290,
                                 0.7966664774136267, 0.9602898564975363};
    static const double wg[4] = {0.3626837833783620, 0.3137066458778873,
                                 0.2223810344533745, 0.1012285362903763};
    double m = 0.5 * (a + b), h = 0.5 * (b - a), s = 0.0;
    for (int q = 0; q < 4; ++q)
        s += wg[q] * (jy_shape(m - h * xg[q], mu, G, beta0)
                    + jy_shape(m + h * xg[q], mu, G, beta0));
    return s * h;
}

/*
 * Support [ylo, yhi] of the p_y marginal: where the exponent has dropped by 70
 * below its maximum (gy - beta0 y = H with H = 1/G + 70/(mu G)).
 */
void orc_mj_range(double mu, double beta0, double *ylo, double *yhi)
{
    double G = 1.0 / sqrt(1.0 - beta0 * beta0);
    double H = 1.0 / G + 70.0 / (mu * G);
    double r = sqrt(H * H - 1.0 / (G * G));
    *ylo = G * G * (H * beta0 - r);
    *yhi = G * G * (H * beta0 + r);
}

/*
 * Inverse cumulative table of the p_y marginal (App. D): y[i] = J^{-1}(i/N)
 * for i = 1..N-1, with y[0] = ylo and y[N] = yhi the truncated support.
 * READING: the paper's table is built by a rectangle-rule search with step
 * halving whose tolerances it does not give; this oracle computes the same
 * quantiles to ~1e-13 by composite Gauss-Legendre quadrature on `nint`
 * sub-intervals and a bracketed Newton solve in the interval that holds each
 * quantile.
 */
void orc_mj_table(double mu, double beta0, int N, int nint, double *y)
{
    double G = 1.0 / sqrt(1.0 - beta0 * beta0);
    double ylo, yhi;
    orc_mj_range(mu, beta0, &ylo, &yhi);
    double h = (yhi - ylo) / nint;
    double *C = (double *)malloc(sizeof(double) * (nint + 1));
    double sum = 0.0, comp = 0.0;
    C[0] = 0.0;
    for (int m = 0; m < nint; ++m) { /* Kahan-compensated running integral */
        double v = gl8(ylo + m * h, ylo + (m + 1) * h, mu, G, beta0) - comp;
        double t = sum + v;
        comp = (t - sum) - v;
        sum = t;
        C[m + 1] = sum;
    }
    double Z = C[nint];
    y[0] = ylo;
    y[N] = yhi;
    int m = 0;
    for (int i = 1; i < N; ++i) {
        double target = Z * (double)i / (double)N;
        while (m < nint - 1 && C[m + 1] <= target) ++m;
        double a = ylo + m * h, b = a + h, lo = a, hi = b;
        double yy = a + h * (target - C[m]) / (C[m + 1] - C[m]);
        for (int it = 0; it < 100; ++it) {
            double F = C[m] + gl8(a, yy, mu, G, beta0) - target;
            if (F > 0) hi = yy; else lo = yy;
            double dn = F / jy_shape(yy, mu, G, beta0);
            double yn = yy - dn;
            if (!(yn > lo && yn < hi)) yn = 0.5 * (lo + hi);
            if (fabs(yn - yy) <= 1e-15 * (fabs(yy) + 1e-3)) { yy = yn; break; }
            yy = yn;
        }
        y[i] = yy;
    }
    free(C);
}

/*
 * u given y (App. D, eqs. distr_u and finding_u): solve l(x) = w l(a) with
 * l(x) = (1+x) e^{-x}, x >= a = mu G sqrt(1+y^2).  READING: Newton on the
 * logarithm, in the unknown d = x - a >= 0 (so that u - 1 = d/a keeps its
 * digits when a is large):  log1p(d/(1+a)) - d - ln w = 0, from d = 0, at least
 * 4 and at most 60 iterations, to |step| <= 1e-15 (d + 1e-300).
 * Returns r = sqrt(u^2 - 1), u = x/a.
 */
double orc_mj_radial(double a, double w)
{
    double lw = log(w), d = 0.0;
    for (int it = 0; it < 60; ++it) {
        double gval = log1p(d / (1.0 + a)) - d - lw;
        double gp = 1.0 / (1.0 + a + d) - 1.0;
        double step = gval / gp;
        d -= step;
        if (d < 0.0) d = 0.0;
        if (it >= 3 && fabs(step) <= 1e-15 * (d + 1e-300)) break;
    }
    double um1 = d / a;
    return sqrt(um1 * (2.0 + um1));
}

/*
 * One momentum draw from the drifting Maxwell-Juttner distribution
 * (Sect. 4.3, eq. Jutt; App. D): p_y from the table by the quantile t
 * (READING: t uniform in [0,1) with linear interpolation between table points,
 * rather than a random table index), r from w in (0,1], azimuth phi = 2 pi v;
 * p_x = gy r cos(phi), p_z = gy r sin(phi).  The drift axis y is then carried
 * onto `axis` by a cyclic permutation (axis 1 = y leaves it in place).
 */
void orc_mj_draw(const double *tab, int N, double mu, double beta0, int axis,
                 double t, double w, double v, double p[3])
{
    double G = 1.0 / sqrt(1.0 - beta0 * beta0);
    double f = t * N;
    int i = (int)floor(f);
    if (i > N - 1) i = N - 1;
    double py = tab[i] + (f - i) * (tab[i + 1] - tab[i]);
    double gy = sqrt(1.0 + py * py);
    double r = orc_mj_radial(mu * G * gy, w);
    double phi = 2.0 * M_PI * v;
    double px = gy * r * cos(phi), pz = gy * r * sin(phi);
    double q[3] = {px, py, pz};
    /* cyclic map sending component 1 (drift) to `axis` */
    int shift = (axis - 1 + 3) % 3;
    for (int a = 0; a < 3; ++a)
        p[(a + shift) % 3] = q[a];
}

/*
 * Generate npairs co-located particle pairs (Sect. 2.1: ions and electrons
 * placed on top of each other so that rho = 0), momenta from two drifting
 * Maxwell-Juttner distributions (species A and B: theta, signed Gamma*beta,
 * drift axis).  Random numbers come from Philox4x64-10, key (seed, stream),
 * counter (pair, j, 0, 0), j = 0, 1, 2:
 *   j=0: w0 w1 w2 -> position, w3 -> A quantile
 *   j=1: w0 -> A radial, w1 -> A azimuth, w2 -> B quantile, w3 -> B radial
 *   j=2: w0 -> B azimuth
 * profile 0: uniform over the box.  profile 1: Harris sheet along `paxis` with
 * density ~ 1/cosh^2((s - centre)/L) on the window |s - centre| < halfw
 * (App. C), drawn by inverse CDF s = centre + L atanh((2U-1) tanh(halfw/L)).
 * Outputs x[3*npairs] (wrapped into the box) and uA, uB [3*npairs].
 */
void orc_load_pairs(const int g[3], uint64_t seed, uint64_t stream, int64_t npairs,
                    int profile, int paxis, double centre, double L, double halfw,
                    const double *tabA, const double *tabB, int N,
                    double thetaA, double gbA, int axisA,
                    double thetaB, double gbB, int axisB,
                    double *x, double *uA, double *uB)
{
    double bA = gbA / sqrt(1.0 + gbA * gbA), bB = gbB / sqrt(1.0 + gbB * gbB);
    uint64_t key[2] = {seed, stream};
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t p = 0; p < npairs; ++p) {
        uint64_t r0[4], r1[4], r2[4];
        uint64_t c0[4] = {(uint64_t)p, 0, 0, 0}, c1[4] = {(uint64_t)p, 1, 0, 0},
                 c2[4] = {(uint64_t)p, 2, 0, 0};
        orc_philox4x64(c0, key, r0);
        orc_philox4x64(c1, key, r1);
        orc_philox4x64(c2, key, r2);
        for (int a = 0; a < 3; ++a) {
            double U = u01(r0[a]);
            double s;
            if (profile == 1 && a == paxis)
                s = centre + L * atanh((2.0 * U - 1.0) * tanh(halfw / L));
            else
                s = U * g[a];
            x[3 * p + a] = wrapd(s, g[a]);
        }
        orc_mj_draw(tabA, N, 1.0 / thetaA, bA, axisA, u01(r0[3]), 1.0 - u01(r1[0]),
                    u01(r1[1]), &uA[3 * p]);
        orc_mj_draw(tabB, N, 1.0 / thetaB, bB, axisB, u01(r1[2]), 1.0 - u01(r1[3]),
                    u01(r2[0]), &uB[3 * p]);
    }
}

/* ---------------------------------------- Harris sheet relations (App. C) */

/*
 * Relativistic Harris equilibrium for electrons and singly charged ions, from
 * the electron temperature Theta_e, the electron drift Gamma_e U_e / c, the
 * temperature ratio chi = (1 + T_i/T_e)/2 and the mass ratio m_i/m_e (App. C,
 * eqs. velocity_Harris and pressure_ad, density contraction n = Gamma n'):
 *   omega_ce/omega'_pe = sqrt(4 chi Theta_e)
 *   L/d'_e             = 2 Theta_e (omega'_pe/omega_ce) / (Gamma_e U_e)
 *   omega_ce/omega_pe  = (omega_ce/omega'_pe) / sqrt(Gamma_e)
 *   L/d_e              = (L/d'_e) sqrt(Gamma_e)
 *   Theta_i = (2 chi - 1) Theta_e (m_e/m_i);  Gamma_i U_i = -(T_i/T_e) Gamma_e U_e
 * out: [wce/w'pe, L/d'e, wce/wpe, L/de, Theta_i, Gamma_i U_i]
 */
void orc_harris_params(double theta_e, double gu_e, double chi, double mi_over_me,
                       double out[6])
{
    double G = sqrt(1.0 + gu_e * gu_e);
    double r = sqrt(4.0 * chi * theta_e);
    double Ldp = 2.0 * theta_e / (r * gu_e);
    double Ti_over_Te = 2.0 * chi - 1.0;
    out[0] = r;
    out[1] = Ldp;
    out[2] = r / sqrt(G);
    out[3] = Ldp * sqrt(G);
    out[4] = Ti_over_Te * theta_e / mi_over_me;
    out[5] = -Ti_over_Te * gu_e;
}
