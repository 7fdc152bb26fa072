/*
 * CPU FP64 oracle for the per-leaf hydro step of Octo-Tiger's new hydro module
 * (arXiv 2107.10987, section IV-B).  TEST INFRASTRUCTURE ONLY: the library's
 * tests, its smoke check and the benchmark's CPU-baseline leg call it; the
 * product path never does.  It shares no code with the GPU library.
 *
 * Layouts (all host memory, caller-owned):
 *   U        [n][7][8][8][8]  fields rho, sx, sy, sz, E, tau, X; cell [k][j][i], i fastest
 *   P        [n][7][14][14][14] ghost-padded block, index (k+3, j+3, i+3)
 *   dx       [n]              cell size of each leaf
 *   origin   [n][3]           centre of cell (0,0,0) of each leaf
 *   tree     nb[3] root leaves per axis, bc[3] (0 periodic, 1 outflow),
 *            level[n], coord[n][3] (leaf coordinates at its level)
 * Directions d = (dx,dy,dz) in {-1,0,1}^3 \ {0} are numbered
 *   dir27(d) = 9(dz+1) + 3(dy+1) + (dx+1), and dir26 skips the centre (13).
 */
#ifndef HYDRO_ORACLE_H
#define HYDRO_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double gamma;   /* ratio of specific heats */
    double omega;   /* frame rotation rate about the z axis through x = y = 0 */
    double eta1;    /* dual-energy pressure switch at face points */
    double eta2;    /* dual-energy tracer resync threshold after a step */
    int centre_only; /* 1: the old scheme, one flux point at each face centre */
    int reflux;      /* 1: coarse faces shared with finer leaves take the mean of
                        the finer faces' fluxes */
} oracle_phys;

/* Point values of one padded block into V (layout of
 * oracle_reconstruct_values); returns the number of cells that fell back to
 * plain PPM (0 for plain PPM itself). */
typedef int (*oracle_values_fn)(const double *P, void *ctx, double *V);

/* One-dimensional PPM on five equally spaced values q[0..4] = q_{-2..2}:
 * left and right interface values of the middle cell. */
void oracle_ppm(const double q[5], double *left, double *right);

/* Central-upwind flux through a face normal to axis n at point xq from the
 * left/right conserved states; returns the local signal speed. */
double oracle_point_flux(int n, const double UL[7], const double UR[7], const double xq[3],
                         const oracle_phys *ph, double F[7]);

/* Tree context used for ghost filling. */
void *oracle_tree_create(const int nb[3], const int bc[3], int n, const int *level,
                         const int *coord);
void oracle_tree_destroy(void *t);
/* on = 1: ghost cells inside a coarser leaf's cell take its minmod-limited
 * linear reconstruction instead of its value (see oracle_fill_padded). */
void oracle_tree_set_prolong(void *t, int on);

/* Ghost-padded blocks of leaves [l0, l1) built from U. Returns 0, or -1 when a
 * ghost cell has no covering leaf. */
int oracle_fill_padded(const void *t, const double *U, int l0, int l1, double *P);

/* Reconstructed values at the 26 points of every interior cell of one padded
 * block: out[7][512][26]. */
void oracle_leaf_reconstruct(const double *P, double *out);

/* Reconstructed values of the cells -1..8 per axis of one padded block:
 * V[(k+1)*100 + (j+1)*10 + (i+1)][dir26][7]. */
void oracle_reconstruct_values(const double *P, double *V);

/* Face fluxes and L(U) from a table of point values laid out as above (the
 * plain reconstruction or a learned one); P supplies the cell values used by
 * the source term. */
double oracle_leaf_fluxes_from_values(const double *V, double dx, const double origin[3],
                                      const oracle_phys *ph, double *Fn);
void oracle_leaf_rhs_from_values(const double *V, const double *P, double dx, const double origin[3],
                                 const oracle_phys *ph, double *dU, double *amax);

/* Face fluxes of one leaf: Fn[3][9][8][8][7] (axis, face along the axis, the
 * other two axes in increasing order, field); returns the max signal speed. */
double oracle_leaf_fluxes(const double *P, double dx, const double origin[3], const oracle_phys *ph,
                          double *Fn);

/* L(U) of one leaf from its padded block: dU[7][512]; *amax = max signal speed
 * over the leaf's face points. */
void oracle_leaf_rhs(const double *P, double dx, const double origin[3], const oracle_phys *ph,
                     double *dU, double *amax);

/* One SSP-RK2 stage for leaves [l0, l1): stage 1: Uout = Uin + dt L(Uin);
 * stage 2: Uout = (Un + (Uin + dt L(Uin)))/2 followed by the tracer resync.
 * Ghosts come from Uin over the whole tree. amax[l] for l in [l0, l1).
 * Returns 0, -1 if a ghost cell or (with reflux) a finer neighbour is not
 * covered by leaves, -2 for an unknown stage. */
int oracle_stage(const void *t, int stage, double dt, const double *Uin, const double *Un,
                 const double *dx, const double *origin, const oracle_phys *ph,
                 int l0, int l1, double *Uout, double *amax);

/* Stage `stage` of the SSP Runge-Kutta integrator of order 2 or 3 (Shu-Osher
 * form): stage 1 as above; later stages Uout = a Un + b (Uin + dt L(Uin)) with
 * (a, b) = (1/2, 1/2) for order 2, (3/4, 1/4) then (1/3, 2/3) for order 3; the
 * tracer resync follows the last stage. */
int oracle_stage_rk(const void *t, int order, int stage, double dt, const double *Uin, const double *Un,
                    const double *dx, const double *origin, const oracle_phys *ph, int l0, int l1,
                    double *Uout, double *amax);

/* oracle_stage_rk with the point values of every leaf (and, with reflux, of
 * the finer leaves next to it) from `values`; fallback[l] (if non-NULL)
 * receives the leaf's own fallback count. */
int oracle_stage_with(const void *t, int order, int stage, double dt, const double *Uin,
                      const double *Un, const double *dx, const double *origin, const oracle_phys *ph,
                      int l0, int l1, double *Uout, double *amax, oracle_values_fn values, void *ctx,
                      int *fallback);

/* Maximum signal speed of every leaf in [l0, l1) for the state U. */
int oracle_signal_speed(const void *t, const double *U, const double *dx, const double *origin,
                        const oracle_phys *ph, int l0, int l1, double *amax);

/* Reconstruction of leaves [l0, l1): out[n][7][512][26]. */
int oracle_reconstruct(const void *t, const double *U, int l0, int l1, double *out);

#ifdef __cplusplus
}
#endif
#endif
