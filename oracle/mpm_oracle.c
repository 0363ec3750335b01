/*
 * mpm_oracle.c -- plain FP64 CPU explicit MPM step.  TEST INFRASTRUCTURE ONLY:
 * the independent checker of the GPU library (see mpm_oracle.h for the
 * sources it follows).  Written for clarity, not speed: one thread, loops
 * over particles and nodes in index order, every nodal field stored densely
 * and reset every step.
 *
 * Build: gcc -O2 -ffp-contract=off -std=c99 -fPIC -shared (no FMA contraction,
 * so every expression rounds as written).
 */
#include "mpm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- mesh -- */

static int ghost_width(int32_t shape) { return shape == OM_SHAPE_GIMP ? 1 : 0; }

int64_t om_num_cells(const om_mesh *mesh)
{
    return (int64_t)mesh->n[0] * mesh->n[1] * mesh->n[2];
}

int64_t om_num_nodes(const om_mesh *mesh, int32_t shape)
{
    int64_t g = ghost_width(shape);
    return (mesh->n[0] + 1 + 2 * g) * (mesh->n[1] + 1 + 2 * g) * (mesh->n[2] + 1 + 2 * g);
}

int64_t om_node_id(const om_mesh *mesh, int32_t shape, int64_t i, int64_t j, int64_t k)
{
    int64_t g = ghost_width(shape);
    int64_t n0 = mesh->n[0] + 1 + 2 * g, n1 = mesh->n[1] + 1 + 2 * g;
    return (i + g) + n0 * ((j + g) + n1 * (k + g));
}

/* Cell index along one axis: half-open cells [o + h c, o + h (c+1)). */
static int64_t cell_coord(double x, double o, double h) { return (int64_t)floor((x - o) / h); }

/* ------------------------------------------------- isoparametric cells -- */

/* The eight node positions of cell c, node q = i + 2j + 4k at (c + (i,j,k)). */
static void iso_corners(const om_mesh *mesh, const int64_t c[3], double X[8][3])
{
    for (int q = 0; q < 8; ++q) {
        int64_t I = om_node_id(mesh, OM_SHAPE_LINEAR, c[0] + (q & 1), c[1] + ((q >> 1) & 1), c[2] + (q >> 2));
        for (int a = 0; a < 3; ++a)
            X[q][a] = mesh->node_x[3 * I + a];
    }
}

/* Trilinear N_q(xi) = 1/8 prod_a (1 + s_qa xi_a), s_qa = -1 or +1, and
 * dN_q/dxi_a. */
static void trilinear(const double xi[3], double N[8], double dN[8][3])
{
    for (int q = 0; q < 8; ++q) {
        double s[3] = {(q & 1) ? 1.0 : -1.0, ((q >> 1) & 1) ? 1.0 : -1.0, (q >> 2) ? 1.0 : -1.0};
        double f[3];
        for (int a = 0; a < 3; ++a)
            f[a] = 1.0 + s[a] * xi[a];
        N[q] = 0.125 * f[0] * f[1] * f[2];
        dN[q][0] = 0.125 * s[0] * f[1] * f[2];
        dN[q][1] = 0.125 * f[0] * s[1] * f[2];
        dN[q][2] = 0.125 * f[0] * f[1] * s[2];
    }
}

/* x(xi) = sum_q N_q X_q and J_ab = dx_a/dxi_b = sum_q X_qa dN_q/dxi_b. */
static void iso_map(const double X[8][3], const double xi[3], double x[3], double J[3][3])
{
    double N[8], dN[8][3];
    trilinear(xi, N, dN);
    for (int a = 0; a < 3; ++a) {
        x[a] = 0.0;
        for (int b = 0; b < 3; ++b)
            J[a][b] = 0.0;
        for (int q = 0; q < 8; ++q) {
            x[a] += N[q] * X[q][a];
            for (int b = 0; b < 3; ++b)
                J[a][b] += X[q][a] * dN[q][b];
        }
    }
}

/* Inverse of a 3x3 matrix by cofactors; returns the determinant. */
static double inverse3(const double M[3][3], double Mi[3][3])
{
    double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                 M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                 M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    Mi[0][0] = (M[1][1] * M[2][2] - M[1][2] * M[2][1]) / det;
    Mi[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) / det;
    Mi[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) / det;
    Mi[1][0] = (M[1][2] * M[2][0] - M[1][0] * M[2][2]) / det;
    Mi[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) / det;
    Mi[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) / det;
    Mi[2][0] = (M[1][0] * M[2][1] - M[1][1] * M[2][0]) / det;
    Mi[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) / det;
    Mi[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) / det;
    return det;
}

int om_iso_natural(const om_mesh *mesh, const int64_t c[3], const double x[3], double xi[3])
{
    double X[8][3], xc[3], A[3][3], Ai[3][3];
    iso_corners(mesh, c, X);
    /* affine initial guess: the map's value and Jacobian at the centre */
    const double zero[3] = {0.0, 0.0, 0.0};
    iso_map(X, zero, xc, A);
    inverse3(A, Ai);
    for (int a = 0; a < 3; ++a) {
        xi[a] = 0.0;
        for (int b = 0; b < 3; ++b)
            xi[a] += Ai[a][b] * (x[b] - xc[b]);
    }
    for (int it = 1; it <= 50; ++it) {
        double xm[3], J[3][3], Ji[3][3], r[3], d[3];
        iso_map(X, xi, xm, J);
        inverse3(J, Ji);
        for (int a = 0; a < 3; ++a)
            r[a] = xm[a] - x[a];
        double dmax = 0.0;
        for (int a = 0; a < 3; ++a) {
            d[a] = 0.0;
            for (int b = 0; b < 3; ++b)
                d[a] += Ji[a][b] * r[b];
            xi[a] -= d[a];
            if (!isfinite(xi[a]))
                return OM_E_NONFINITE;
            dmax = fmax(dmax, fabs(d[a]));
        }
        /* quadratic convergence: what is left after a correction of 1e-12
         * is of order 1e-24, below the rounding of xi itself */
        if (dmax <= 1e-12)
            return it;
    }
    return 50;
}

/* How far xi lies outside the half-open cube [-1, 1)^3 along the worst axis
 * (<= 0: inside or on a face). */
static double overshoot(const double xi[3])
{
    double o = -1e300;
    for (int a = 0; a < 3; ++a)
        o = fmax(o, fmax(-1.0 - xi[a], xi[a] - 1.0));
    return o;
}

static int inside(const double xi[3])
{
    for (int a = 0; a < 3; ++a)
        if (!(xi[a] >= -1.0 && xi[a] < 1.0))
            return 0;
    return 1;
}

/* Brute-force location in an isoparametric mesh (see om_locate). */
static int iso_locate_one(const om_mesh *mesh, const double x[3], int64_t c_out[3], double xi_out[3])
{
    double best = 1e300;
    int found = 0;
    for (int64_t cz = 0; cz < mesh->n[2]; ++cz)
        for (int64_t cy = 0; cy < mesh->n[1]; ++cy)
            for (int64_t cx = 0; cx < mesh->n[0]; ++cx) {
                const int64_t c[3] = {cx, cy, cz};
                double X[8][3], lo[3], hi[3];
                iso_corners(mesh, c, X);
                for (int a = 0; a < 3; ++a) {
                    lo[a] = hi[a] = X[0][a];
                    for (int q = 1; q < 8; ++q) {
                        lo[a] = fmin(lo[a], X[q][a]);
                        hi[a] = fmax(hi[a], X[q][a]);
                    }
                    double pad = 1e-9 * (hi[a] - lo[a]);
                    if (x[a] < lo[a] - pad || x[a] > hi[a] + pad)
                        goto next;
                }
                {
                    double xi[3];
                    if (om_iso_natural(mesh, c, x, xi) < 0)
                        goto next;
                    if (inside(xi)) {
                        for (int a = 0; a < 3; ++a) {
                            c_out[a] = c[a];
                            xi_out[a] = xi[a];
                        }
                        return OM_OK;
                    }
                    /* a near miss counts only across a face another cell shares */
                    double o = overshoot(xi);
                    int interior = 1;
                    for (int a = 0; a < 3; ++a) {
                        if (xi[a] < -1.0 && c[a] == 0)
                            interior = 0;
                        if (xi[a] >= 1.0 && c[a] == mesh->n[a] - 1)
                            interior = 0;
                    }
                    if (interior && o <= 1e-12 && o < best) {
                        best = o;
                        found = 1;
                        for (int a = 0; a < 3; ++a) {
                            c_out[a] = c[a];
                            xi_out[a] = xi[a];
                        }
                    }
                }
            next:;
            }
    return found ? OM_OK : OM_E_OUT_OF_MESH;
}

int om_locate(const om_mesh *mesh, int64_t n, const double *x, int64_t *cell)
{
    for (int64_t p = 0; p < n; ++p) {
        if (mesh->node_x) {
            int64_t c[3];
            double xi[3];
            for (int a = 0; a < 3; ++a)
                if (!isfinite(x[3 * p + a]))
                    return OM_E_NONFINITE;
            int rc = iso_locate_one(mesh, &x[3 * p], c, xi);
            if (rc != OM_OK)
                return rc;
            cell[p] = c[0] + (int64_t)mesh->n[0] * (c[1] + (int64_t)mesh->n[1] * c[2]);
            continue;
        }
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            double xa = x[3 * p + a];
            if (!isfinite(xa))
                return OM_E_NONFINITE;
            c[a] = cell_coord(xa, mesh->origin[a], mesh->h);
            if (c[a] < 0 || c[a] >= mesh->n[a])
                return OM_E_OUT_OF_MESH;
        }
        cell[p] = c[0] + (int64_t)mesh->n[0] * (c[1] + (int64_t)mesh->n[1] * c[2]);
    }
    return OM_OK;
}

/* ------------------------------------------------------ shape functions -- */

void om_gimp_1d(double r, double h, double l, double out[2])
{
    /* uGIMP: the linear hat of half-width h averaged over a particle domain
     * of half-length l centred at offset r from the node. */
    double a = fabs(r);
    double s = r < 0.0 ? -1.0 : 1.0;
    if (a < l) {
        out[0] = 1.0 - (r * r + l * l) / (2.0 * h * l);
        out[1] = -r / (h * l);
    } else if (a < h - l) {
        out[0] = 1.0 - a / h;
        out[1] = -s / h;
    } else if (a < h + l) {
        double d = h + l - a;
        out[0] = d * d / (4.0 * h * l);
        out[1] = -s * d / (2.0 * h * l);
    } else {
        out[0] = 0.0;
        out[1] = 0.0;
    }
}

/* Isoparametric 8-node hexahedron in cell c: N_q(xi) at the point's natural
 * coordinates xi (Newton-Raphson), grad N_q = J^-T dN_q/dxi with J = dx/dxi
 * there. */
static int iso_shape_in_cell(const om_mesh *mesh, const int64_t c[3], const double x[3],
                             int64_t *node, double *N, double *dN)
{
    double xi[3], X[8][3], xm[3], J[3][3], Ji[3][3], Nq[8], dNq[8][3];
    int rc = om_iso_natural(mesh, c, x, xi);
    if (rc < 0)
        return rc;
    iso_corners(mesh, c, X);
    iso_map(X, xi, xm, J);
    inverse3(J, Ji);
    trilinear(xi, Nq, dNq);
    for (int q = 0; q < 8; ++q) {
        node[q] = om_node_id(mesh, OM_SHAPE_LINEAR, c[0] + (q & 1), c[1] + ((q >> 1) & 1), c[2] + (q >> 2));
        N[q] = Nq[q];
        /* dN/dx_a = sum_b (dxi_b/dx_a) dN/dxi_b = sum_b Ji[b][a] dN/dxi_b */
        for (int a = 0; a < 3; ++a) {
            dN[3 * q + a] = 0.0;
            for (int b = 0; b < 3; ++b)
                dN[3 * q + a] += Ji[b][a] * dNq[q][b];
        }
    }
    return 8;
}

int om_shape(const om_mesh *mesh, int32_t shape, const double x[3],
             int64_t *node, double *N, double *dN)
{
    if (mesh->node_x) {
        if (shape != OM_SHAPE_LINEAR)
            return OM_E_ARG;
        int64_t c[3];
        double xi[3];
        for (int a = 0; a < 3; ++a)
            if (!isfinite(x[a]))
                return OM_E_NONFINITE;
        int rc = iso_locate_one(mesh, x, c, xi);
        if (rc != OM_OK)
            return rc;
        return iso_shape_in_cell(mesh, c, x, node, N, dN);
    }
    const double h = mesh->h;
    int64_t c[3];
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(x[a]))
            return OM_E_NONFINITE;
        c[a] = cell_coord(x[a], mesh->origin[a], h);
        if (c[a] < 0 || c[a] >= mesh->n[a])
            return OM_E_OUT_OF_MESH;
    }
    if (shape == OM_SHAPE_LINEAR) {
        /* Trilinear 8-node hexahedron in natural coordinates xi in [-1, 1]:
         * N_I = 1/8 (1 + xi xi_I)(1 + eta eta_I)(1 + zeta zeta_I). */
        double xi[3];
        for (int a = 0; a < 3; ++a)
            xi[a] = 2.0 * (x[a] - (mesh->origin[a] + h * (double)c[a])) / h - 1.0;
        int q = 0;
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i) {
                    double sx = 2.0 * i - 1.0, sy = 2.0 * j - 1.0, sz = 2.0 * k - 1.0;
                    double fx = 1.0 + xi[0] * sx, fy = 1.0 + xi[1] * sy, fz = 1.0 + xi[2] * sz;
                    node[q] = om_node_id(mesh, shape, c[0] + i, c[1] + j, c[2] + k);
                    N[q] = 0.125 * fx * fy * fz;
                    /* dN/dx_a = (dxi/dx) dN/dxi_a with dxi/dx = 2/h. */
                    dN[3 * q + 0] = (2.0 / h) * 0.125 * sx * fy * fz;
                    dN[3 * q + 1] = (2.0 / h) * 0.125 * fx * sy * fz;
                    dN[3 * q + 2] = (2.0 / h) * 0.125 * fx * fy * sz;
                    ++q;
                }
        return q;
    }
    if (shape == OM_SHAPE_GIMP) {
        /* Tensor product of 1-D uGIMP weights, particle half-length h/4
         * (2 particles per cell per axis).  Support along each axis: the
         * three nodes i0, i0+1, i0+2 with i0 = floor((x - o - l)/h). */
        const double l = 0.25 * h;
        int64_t i0[3];
        double S[3][3], dS[3][3];
        for (int a = 0; a < 3; ++a) {
            i0[a] = (int64_t)floor((x[a] - mesh->origin[a] - l) / h);
            for (int t = 0; t < 3; ++t) {
                double r = x[a] - (mesh->origin[a] + h * (double)(i0[a] + t));
                double w[2];
                om_gimp_1d(r, h, l, w);
                S[a][t] = w[0];
                dS[a][t] = w[1];
            }
        }
        int q = 0;
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j)
                for (int i = 0; i < 3; ++i) {
                    node[q] = om_node_id(mesh, shape, i0[0] + i, i0[1] + j, i0[2] + k);
                    N[q] = S[0][i] * S[1][j] * S[2][k];
                    dN[3 * q + 0] = dS[0][i] * S[1][j] * S[2][k];
                    dN[3 * q + 1] = S[0][i] * dS[1][j] * S[2][k];
                    dN[3 * q + 2] = S[0][i] * S[1][j] * dS[2][k];
                    ++q;
                }
        return q;
    }
    return OM_E_ARG;
}

/* ----------------------------------------------------------- material -- */

void om_dp_coefficients(const om_material *mat, double out[3])
{
    /* Drucker-Prager cone matched to Mohr-Coulomb:
     *   outer (triaxial compression) eta = 6 sin(phi) / (sqrt3 (3 - sin(phi)))
     *   inner (triaxial extension)   eta = 6 sin(phi) / (sqrt3 (3 + sin(phi)))
     *   plane strain                 eta = 3 tan(phi) / sqrt(9 + 12 tan^2(phi))
     * xi is the cohesion factor of the same cone; eta_bar is eta with the
     * dilation angle psi in place of phi. */
    const double r3 = sqrt(3.0);
    double angle[2] = {mat->phi, mat->psi};
    double eta[2], xi = 0.0;
    for (int t = 0; t < 2; ++t) {
        double s = sin(angle[t]), co = cos(angle[t]), ta = tan(angle[t]);
        double e, x;
        if (mat->dp_cone == OM_DP_INNER) {
            e = 6.0 * s / (r3 * (3.0 + s));
            x = 6.0 * co / (r3 * (3.0 + s));
        } else if (mat->dp_cone == OM_DP_PLANE_STRAIN) {
            double d = sqrt(9.0 + 12.0 * ta * ta);
            e = 3.0 * ta / d;
            x = 3.0 / d;
        } else {
            e = 6.0 * s / (r3 * (3.0 - s));
            x = 6.0 * co / (r3 * (3.0 - s));
        }
        eta[t] = e;
        if (t == 0)
            xi = x;
    }
    out[0] = eta[0];
    out[1] = xi;
    out[2] = eta[1];
}

int om_constitutive(const om_material *mat, const double deps[6], double sig[6])
{
    const double E = mat->E, nu = mat->nu;
    const double G = E / (2.0 * (1.0 + nu));
    const double K = E / (3.0 * (1.0 - 2.0 * nu));
    const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));

    /* Elastic (trial) increment: sigma += lambda tr(deps) I + 2 G eps, with
     * engineering shear strains, so the shear terms take G gamma. */
    double tr = deps[0] + deps[1] + deps[2];
    double st[6];
    for (int a = 0; a < 3; ++a)
        st[a] = sig[a] + lam * tr + 2.0 * G * deps[a];
    for (int a = 3; a < 6; ++a)
        st[a] = sig[a] + G * deps[a];

    if (mat->model == OM_LINEAR_ELASTIC) {
        memcpy(sig, st, sizeof st);
        return 0;
    }

    /* Drucker-Prager, perfectly plastic, flow potential with eta_bar:
     * f = sqrt(J2(s)) + eta p - xi c. */
    double co[3];
    om_dp_coefficients(mat, co);
    const double eta = co[0], xi = co[1], etab = co[2];
    double p = (st[0] + st[1] + st[2]) / 3.0;
    double s[6];
    for (int a = 0; a < 3; ++a)
        s[a] = st[a] - p;
    for (int a = 3; a < 6; ++a)
        s[a] = st[a];
    double J2 = 0.5 * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2]) + s[3] * s[3] + s[4] * s[4] + s[5] * s[5];
    double q = sqrt(J2);
    double f = q + eta * p - xi * mat->c;
    if (f <= 0.0) {
        memcpy(sig, st, sizeof st);
        return 0;
    }
    double dgam = f / (G + K * eta * etab);
    if (q - G * dgam >= 0.0) {
        /* Return to the smooth cone: deviator scaled radially, pressure
         * shifted by the plastic volume change K eta_bar dgamma. */
        double scale = 1.0 - G * dgam / q;
        double pn = p - K * etab * dgam;
        for (int a = 0; a < 3; ++a)
            sig[a] = scale * s[a] + pn;
        for (int a = 3; a < 6; ++a)
            sig[a] = scale * s[a];
        return 1;
    }
    /* Return to the apex of the cone (zero deviator, f = 0). */
    double pa = eta > 0.0 ? xi * mat->c / eta : p;
    for (int a = 0; a < 3; ++a)
        sig[a] = pa;
    for (int a = 3; a < 6; ++a)
        sig[a] = 0.0;
    return 2;
}

/* -------------------------------------------------------- constraints -- */

/* Set every constrained component of the nodal vector field w: to the
 * prescribed velocity (accel == 0) or to zero (accel != 0).  Face rules:
 * node index i_b <= 0 lies on face -b (ghost nodes included), i_b >= n_b on
 * face +b; FIXED constrains all three components, SLIP the normal one.
 * Per-node constraints are applied afterwards and take precedence. */
static void apply_constraints(const om_mesh *mesh, int32_t shape, const om_bc *bc,
                              double *w, int accel)
{
    int64_t g = ghost_width(shape);
    for (int64_t k = -g; k <= mesh->n[2] + g; ++k)
        for (int64_t j = -g; j <= mesh->n[1] + g; ++j)
            for (int64_t i = -g; i <= mesh->n[0] + g; ++i) {
                int64_t idx[3] = {i, j, k};
                int fixed[3] = {0, 0, 0};
                for (int b = 0; b < 3; ++b) {
                    int rules[2] = {idx[b] <= 0 ? bc->face[2 * b] : OM_FREE,
                                    idx[b] >= mesh->n[b] ? bc->face[2 * b + 1] : OM_FREE};
                    for (int r = 0; r < 2; ++r) {
                        if (rules[r] == OM_FIXED)
                            fixed[0] = fixed[1] = fixed[2] = 1;
                        else if (rules[r] == OM_SLIP)
                            fixed[b] = 1;
                    }
                }
                int64_t I = om_node_id(mesh, shape, i, j, k);
                for (int a = 0; a < 3; ++a)
                    if (fixed[a])
                        w[3 * I + a] = 0.0;
            }
    for (int64_t e = 0; e < bc->n_extra; ++e)
        w[3 * bc->node[e] + bc->axis[e]] = accel ? 0.0 : bc->value[e];
}

/* ------------------------------------------------------------- step ------ */

typedef struct {
    int64_t node[27];
    double N[27];
    double dN[81];
    int count;
} support;

/* Support of a particle at x; on an isoparametric mesh, in the cell that
 * step 1 located it in (cell id), on a uniform mesh found from x. */
static int support_of(const om_mesh *mesh, int32_t shape, const double *x, int64_t cell, support *s)
{
    int q;
    if (mesh->node_x) {
        const int64_t c[3] = {cell % mesh->n[0], (cell / mesh->n[0]) % mesh->n[1],
                              cell / ((int64_t)mesh->n[0] * mesh->n[1])};
        q = iso_shape_in_cell(mesh, c, x, s->node, s->N, s->dN);
    } else {
        q = om_shape(mesh, shape, x, s->node, s->N, s->dN);
    }
    if (q < 0)
        return q;
    s->count = q;
    return OM_OK;
}

/* Strain increment from a nodal velocity field w and the support s:
 * L_ab = sum_I w_Ia dN_I/dx_b, deps = dt (L_xx, L_yy, L_zz, L_xy + L_yx,
 * L_yz + L_zy, L_xz + L_zx). */
static void strain_increment(const support *s, const double *w, double dt, double deps[6])
{
    double L[3][3] = {{0}};
    for (int q = 0; q < s->count; ++q) {
        const double *wi = &w[3 * s->node[q]];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                L[a][b] += wi[a] * s->dN[3 * q + b];
    }
    deps[0] = dt * L[0][0];
    deps[1] = dt * L[1][1];
    deps[2] = dt * L[2][2];
    deps[3] = dt * (L[0][1] + L[1][0]);
    deps[4] = dt * (L[1][2] + L[2][1]);
    deps[5] = dt * (L[0][2] + L[2][0]);
}

/* Volume and stress update of one particle: V *= 1 + tr(deps), then the
 * material law. */
static void update_stress(const om_material *mat, const double deps[6], double *vol, double *sig)
{
    *vol *= 1.0 + deps[0] + deps[1] + deps[2];
    om_constitutive(mat, deps, sig);
}

/* Internal and external nodal force of one particle:
 * f_I += -V sigma . grad N_I + N_I m g. */
static void add_force(const support *s, double vol, const double *sig, double m,
                      const double *g, double *f)
{
    /* Voigt -> full symmetric tensor rows. */
    double S[3][3] = {{sig[0], sig[3], sig[5]}, {sig[3], sig[1], sig[4]}, {sig[5], sig[4], sig[2]}};
    for (int q = 0; q < s->count; ++q) {
        double *fi = &f[3 * s->node[q]];
        for (int a = 0; a < 3; ++a) {
            double t = 0.0;
            for (int b = 0; b < 3; ++b)
                t += S[a][b] * s->dN[3 * q + b];
            fi[a] += -vol * t + s->N[q] * m * g[a];
        }
    }
}

int om_step(const om_mesh *mesh, const om_material *mat, const om_bc *bc,
            const om_scheme *scheme, int64_t n, double *x, double *v,
            double *sig, double *vol, const double *mass, om_grid *grid,
            int64_t step)
{
    if (!mesh || !mat || !bc || !scheme || !grid || n < 0 || (!mesh->node_x && mesh->h <= 0.0))
        return OM_E_ARG;
    if (mesh->node_x && scheme->shape != OM_SHAPE_LINEAR)
        return OM_E_ARG;
    if (scheme->algo != OM_USF && scheme->algo != OM_USL && scheme->algo != OM_MUSL)
        return OM_E_ARG;
    const int32_t shape = scheme->shape;
    const int64_t nn = om_num_nodes(mesh, shape);
    const int64_t nc = om_num_cells(mesh);
    const double dt = scheme->dt;
    support s;
    int rc;

    /* 1. Locate every particle; count particles per cell (active cells). */
    int64_t *pcell = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!pcell)
        return OM_E_NOMEM;
    memset(grid->cell_count, 0, sizeof(uint32_t) * (size_t)nc);
    for (int64_t p = 0; p < n; ++p) {
        rc = om_locate(mesh, 1, &x[3 * p], &pcell[p]);
        if (rc != OM_OK) {
            free(pcell);
            return rc;
        }
        grid->cell_count[pcell[p]] += 1;
    }

    /* Start-of-step positions: every transfer of the step is evaluated there
     * (USL needs them after the positions have moved). */
    double *x0 = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!x0) {
        free(pcell);
        return OM_E_NOMEM;
    }
    memcpy(x0, x, sizeof(double) * 3 * (size_t)n);

    /* 2. Reset every nodal quantity. */
    memset(grid->m, 0, sizeof(double) * (size_t)nn);
    memset(grid->p, 0, sizeof(double) * 3 * (size_t)nn);
    memset(grid->v, 0, sizeof(double) * 3 * (size_t)nn);
    memset(grid->f, 0, sizeof(double) * 3 * (size_t)nn);
    memset(grid->a, 0, sizeof(double) * 3 * (size_t)nn);
    memset(grid->vn, 0, sizeof(double) * 3 * (size_t)nn);

    double msum = 0.0;
    for (int64_t p = 0; p < n; ++p)
        msum += mass[p];
    const double eps_m = n > 0 ? scheme->mass_eps_rel * (msum / (double)n) : 0.0;

    /* 3. P2G: nodal mass and momentum. */
    for (int64_t p = 0; p < n; ++p) {
        support_of(mesh, shape, &x0[3 * p], pcell[p], &s);
        for (int q = 0; q < s.count; ++q) {
            int64_t I = s.node[q];
            grid->m[I] += s.N[q] * mass[p];
            for (int a = 0; a < 3; ++a)
                grid->p[3 * I + a] += s.N[q] * mass[p] * v[3 * p + a];
        }
    }

    /* 4. Nodal velocity, then velocity constraints. */
    for (int64_t I = 0; I < nn; ++I)
        for (int a = 0; a < 3; ++a)
            grid->v[3 * I + a] = grid->m[I] > eps_m ? grid->p[3 * I + a] / grid->m[I] : 0.0;
    apply_constraints(mesh, shape, bc, grid->v, 0);

    /* 5. USF: stress update from the nodal velocity before the forces. */
    if (scheme->algo == OM_USF) {
        for (int64_t p = 0; p < n; ++p) {
            double deps[6];
            support_of(mesh, shape, &x0[3 * p], pcell[p], &s);
            strain_increment(&s, grid->v, dt, deps);
            update_stress(mat, deps, &vol[p], &sig[6 * p]);
        }
    }

    /* 6. P2G: internal and external forces, then the external forces given
     * at nodes (a surface traction in nodal form). */
    for (int64_t p = 0; p < n; ++p) {
        support_of(mesh, shape, &x0[3 * p], pcell[p], &s);
        add_force(&s, vol[p], &sig[6 * p], mass[p], scheme->gravity, grid->f);
    }
    double ramp = 1.0;
    if (bc->force_ramp_steps > 0 && step < bc->force_ramp_steps) {
        double u = (double)step / (double)bc->force_ramp_steps;
        ramp = u * u * (3.0 - 2.0 * u);
    }
    for (int64_t e = 0; e < bc->n_force; ++e)
        for (int a = 0; a < 3; ++a)
            grid->f[3 * bc->force_node[e] + a] += ramp * bc->force_value[3 * e + a];

    /* 7. Nodal acceleration and updated velocity, with constraints. */
    for (int64_t I = 0; I < nn; ++I)
        for (int a = 0; a < 3; ++a)
            grid->a[3 * I + a] = grid->m[I] > eps_m ? grid->f[3 * I + a] / grid->m[I] : 0.0;
    apply_constraints(mesh, shape, bc, grid->a, 1);
    for (int64_t I = 0; I < 3 * nn; ++I)
        grid->vn[I] = grid->v[I] + dt * grid->a[I];
    apply_constraints(mesh, shape, bc, grid->vn, 0);

    /* 8. G2P: particle velocity (FLIP increment or PIC) and position. */
    for (int64_t p = 0; p < n; ++p) {
        support_of(mesh, shape, &x0[3 * p], pcell[p], &s);
        double dv[3] = {0, 0, 0}, vp[3] = {0, 0, 0};
        for (int q = 0; q < s.count; ++q) {
            int64_t I = s.node[q];
            for (int a = 0; a < 3; ++a) {
                dv[a] += s.N[q] * grid->a[3 * I + a];
                vp[a] += s.N[q] * grid->vn[3 * I + a];
            }
        }
        for (int a = 0; a < 3; ++a) {
            if (scheme->velocity_update == OM_PIC)
                v[3 * p + a] = vp[a];
            else
                v[3 * p + a] += dt * dv[a];
            x[3 * p + a] += dt * vp[a];
        }
    }

    /* 9. USL: stress update last, from the updated nodal velocity and the
     * start-of-step shape functions. */
    if (scheme->algo == OM_USL) {
        for (int64_t p = 0; p < n; ++p) {
            double deps[6];
            support_of(mesh, shape, &x0[3 * p], pcell[p], &s);
            strain_increment(&s, grid->vn, dt, deps);
            update_stress(mat, deps, &vol[p], &sig[6 * p]);
        }
    }
    /* 9'. MUSL: the updated particle momenta back to the nodes with the
     * start-of-step shape functions, the nodal velocity of that momentum
     * under the velocity constraints, and the stress update from it. */
    if (scheme->algo == OM_MUSL) {
        double *vr = (double *)calloc(3 * (size_t)nn, sizeof(double));
        if (!vr) {
            free(x0);
            free(pcell);
            return OM_E_NOMEM;
        }
        for (int64_t p = 0; p < n; ++p) {
            support_of(mesh, shape, &x0[3 * p], pcell[p], &s);
            for (int q = 0; q < s.count; ++q)
                for (int a = 0; a < 3; ++a)
                    vr[3 * s.node[q] + a] += s.N[q] * mass[p] * v[3 * p + a];
        }
        for (int64_t I = 0; I < nn; ++I)
            for (int a = 0; a < 3; ++a)
                vr[3 * I + a] = grid->m[I] > eps_m ? vr[3 * I + a] / grid->m[I] : 0.0;
        apply_constraints(mesh, shape, bc, vr, 0);
        for (int64_t p = 0; p < n; ++p) {
            double deps[6];
            support_of(mesh, shape, &x0[3 * p], pcell[p], &s);
            strain_increment(&s, vr, dt, deps);
            update_stress(mat, deps, &vol[p], &sig[6 * p]);
        }
        free(vr);
    }
    free(x0);
    free(pcell);

    rc = OM_OK;
    for (int64_t p = 0; p < n && rc == OM_OK; ++p) {
        for (int a = 0; a < 3; ++a)
            if (!isfinite(x[3 * p + a]) || !isfinite(v[3 * p + a]))
                rc = OM_E_NONFINITE;
        for (int k = 0; k < 6; ++k)
            if (!isfinite(sig[6 * p + k]))
                rc = OM_E_NONFINITE;
        if (!isfinite(vol[p]))
            rc = OM_E_NONFINITE;
    }
    return rc;
}

int om_run(const om_mesh *mesh, const om_material *mat, const om_bc *bc,
           const om_scheme *scheme, int64_t n, double *x, double *v,
           double *sig, double *vol, const double *mass, om_grid *grid,
           int64_t step0, int64_t nsteps)
{
    for (int64_t s = 0; s < nsteps; ++s) {
        int rc = om_step(mesh, mat, bc, scheme, n, x, v, sig, vol, mass, grid, step0 + s + 1);
        if (rc != OM_OK)
            return rc;
    }
    return OM_OK;
}
