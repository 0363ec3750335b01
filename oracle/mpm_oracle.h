/*
 * mpm_oracle.h -- plain FP64 CPU implementation of one explicit material
 * point method (MPM) time step on a uniform 8-node hexahedral mesh.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent checker of the
 * GPU library: only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, header, table or helper
 * with the GPU path.
 *
 * What it follows (Kumar et al., "Scalable and modular material point method
 * for large-scale simulations", arXiv:1909.13380):
 *   - Introduction: state lives on material points; nodal values are reset
 *     every step; particle quantities are mapped to the nodes and the nodal
 *     solution is interpolated back with the same mapping functions.
 *   - Code overview: Node holds mass, momentum, velocity, acceleration and
 *     force; velocity constraints live at nodes and survive the reset; a cell
 *     and its nodes are active iff the cell holds a material point; Material
 *     returns the updated stress for a strain increment; the explicit
 *     algorithms are update-stress-first (USF) and update-stress-last (USL);
 *     the modified USL (MUSL), which strains with the nodal velocity of the
 *     updated particle momenta mapped back to the nodes, is not in the paper
 *     and follows Sulsky, Zhou & Schreyer (1995) and Buzzi et al. (2008);
 *     shape functions are linear or GIMP.
 *   - Data structures: 6-component Voigt stress.
 * The paper prints no MPM equations.  The steps are the textbook explicit MPM
 * (Sulsky, Chen & Schreyer 1994; USF/USL orderings of Bardenhagen 2002 and
 * Buzzi et al. 2008), uGIMP weights (Bardenhagen & Kober 2004) and the
 * Drucker-Prager return map of de Souza Neto, Peric & Owen (2008).
 *
 * Conventions: tension positive; Voigt order xx, yy, zz, xy, yz, xz;
 * engineering shear in strain increments, tensor shear in stress.
 * Particle arrays are row-major: x[3*p+a], v[3*p+a], sig[6*p+k].
 * Everything is double precision; particles and nodes are visited in index
 * order by a single thread.
 */
#ifndef MPM_ORACLE_H
#define MPM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    OM_OK = 0,
    OM_E_ARG = -1,
    OM_E_NOMEM = -2,
    OM_E_OUT_OF_MESH = -4,
    OM_E_NONFINITE = -5
};
enum { OM_LINEAR_ELASTIC = 0, OM_DRUCKER_PRAGER = 1 };
enum { OM_DP_OUTER = 0, OM_DP_INNER = 1, OM_DP_PLANE_STRAIN = 2 };
enum { OM_FREE = 0, OM_FIXED = 1, OM_SLIP = 2 };
enum { OM_USF = 0, OM_USL = 1, OM_MUSL = 2 };
enum { OM_SHAPE_LINEAR = 0, OM_SHAPE_GIMP = 1 };
enum { OM_FLIP = 0, OM_PIC = 1 };

/* Mesh of n[0] x n[1] x n[2] 8-node hexahedra.  Uniform when node_x is
 * NULL: node (i,j,k) at origin + h*(i,j,k).  Isoparametric otherwise
 * (isoparametric-mesh section): the same logically structured cells and
 * node numbering, node I at node_x[3*I+a], each cell the trilinear image of
 * the natural cube [-1,1]^3 of its eight nodes; origin and h are then unused
 * here.  Isoparametric meshes take linear shape functions only. */
typedef struct {
    int32_t n[3];
    int32_t pad_;
    double origin[3];
    double h;
    const double *node_x;
} om_mesh;

typedef struct {
    int32_t model;   /* OM_LINEAR_ELASTIC or OM_DRUCKER_PRAGER */
    int32_t dp_cone; /* OM_DP_OUTER / INNER / PLANE_STRAIN */
    double rho, E, nu;
    double phi, psi, c; /* friction angle, dilation angle (radians), cohesion */
} om_material;

/* Face rules for faces -x,+x,-y,+y,-z,+z plus optional per-node constraints
 * (node id in this library's node numbering, axis 0..2, prescribed velocity),
 * plus optional external nodal forces (node id, force vector force_value[3e+a])
 * that stand for a traction on the body's surface (benchmark section: uniform
 * tension applied at the ends of the strip); they join the nodal force of
 * every step, scaled in the n-th step (n = 1 first) by the smooth ramp
 * u^2 (3 - 2u), u = n / force_ramp_steps, until n reaches force_ramp_steps
 * and by 1 after (force_ramp_steps = 0: full from the start). */
typedef struct {
    int32_t face[6];
    int32_t pad_;
    int64_t n_extra;
    const int64_t *node;
    const int32_t *axis;
    const double *value;
    int64_t n_force;
    const int64_t *force_node;
    const double *force_value;
    int64_t force_ramp_steps;
} om_bc;

typedef struct {
    int32_t algo;            /* OM_USF, OM_USL or OM_MUSL */
    int32_t shape;           /* OM_SHAPE_LINEAR or OM_SHAPE_GIMP */
    int32_t velocity_update; /* OM_FLIP or OM_PIC */
    int32_t pad_;
    double gravity[3];
    double dt;
    double mass_eps_rel;     /* nodes with m <= mass_eps_rel * mean(m_p) are void */
} om_scheme;

/* Caller-owned nodal workspace, sized by om_num_nodes / om_num_cells.
 * After om_step it holds the step's nodal mass m, momentum p, velocity v
 * (after constraints), force f, acceleration a and updated velocity vn,
 * each vector field row-major [3*I+a], and the particle count per cell. */
typedef struct {
    double *m, *p, *v, *f, *a, *vn;
    uint32_t *cell_count;
} om_grid;

/* Node numbering: linear shape functions use nodes 0..n[a]; GIMP adds one
 * ghost layer, nodes -1..n[a]+1.  Id = (i+g) + N0*((j+g) + N1*(k+g)) with
 * g the ghost width and N0, N1 the node counts along x and y. */
int64_t om_num_nodes(const om_mesh *mesh, int32_t shape);
int64_t om_num_cells(const om_mesh *mesh);
int64_t om_node_id(const om_mesh *mesh, int32_t shape, int64_t i, int64_t j, int64_t k);

/* Cell of each particle, id = cx + nx*(cy + ny*cz).  Uniform mesh:
 * c_a = floor((x_a - o_a)/h); OM_E_OUT_OF_MESH if any particle lies outside
 * [o, o + n h).  Isoparametric mesh: the cell whose inverse map puts the
 * particle at natural coordinates -1 <= xi_a < 1 on every axis (the
 * half-open rule of the uniform mesh), searched over every cell in id
 * order; a particle that rounding leaves just outside two cells sharing a
 * face (no more than 1e-12 past it) goes to the one it overshoots least;
 * OM_E_OUT_OF_MESH if no cell holds it. */
int om_locate(const om_mesh *mesh, int64_t n, const double *x, int64_t *cell);

/* Natural coordinates of point x in cell (cx, cy, cz) of an isoparametric
 * mesh by Newton-Raphson on x(xi) = sum_I N_I(xi) X_I, starting from the
 * affine guess xi0 = A^-1 (x - x_c) (x_c the mean of the eight nodes, A the
 * Jacobian at the cell's centre) and stopping after a correction of at most
 * 1e-12 (the error left is then of order its square; at most 50
 * iterations).  Returns the number of iterations, or
 * OM_E_NONFINITE if the iteration broke down. */
int om_iso_natural(const om_mesh *mesh, const int64_t c[3], const double x[3], double xi[3]);

/* Shape functions of one particle.  Writes node ids, weights and
 * x-gradients of every node in the particle's support (8 or 27) and returns
 * that count, or a negative error code. */
int om_shape(const om_mesh *mesh, int32_t shape, const double x[3],
             int64_t *node, double *N, double *dN /* [3*k+a] */);

/* One-dimensional uGIMP weight and derivative for node offset r = x_p - X_I,
 * cell size h and particle half-length l: out[0] = S, out[1] = dS/dr. */
void om_gimp_1d(double r, double h, double l, double out[2]);

/* Drucker-Prager coefficients for the chosen cone: out = {eta, xi, eta_bar}. */
void om_dp_coefficients(const om_material *mat, double out[3]);

/* Stress update for one strain increment (Voigt, engineering shear).
 * Returns 0 if the step was elastic, 1 for a return to the cone, 2 for a
 * return to the apex. */
int om_constitutive(const om_material *mat, const double deps[6], double sig[6]);

/* Time step number `step` (1 for a scene's first step; it only sets the
 * ramp of the nodal forces) of the algorithm in scheme, for n particles,
 * updated in place.  mass is constant.  Returns OM_OK or an error code. */
int om_step(const om_mesh *mesh, const om_material *mat, const om_bc *bc,
            const om_scheme *scheme, int64_t n, double *x, double *v,
            double *sig, double *vol, const double *mass, om_grid *grid,
            int64_t step);

/* Steps step0 + 1 .. step0 + nsteps through om_step; stops at the first
 * error. */
int om_run(const om_mesh *mesh, const om_material *mat, const om_bc *bc,
           const om_scheme *scheme, int64_t n, double *x, double *v,
           double *sig, double *vol, const double *mass, om_grid *grid,
           int64_t step0, int64_t nsteps);

#ifdef __cplusplus
}
#endif

#endif
