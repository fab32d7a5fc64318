/*
 * swe_oracle.h -- reference solver for the 2D shallow water step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a deliberately plain, slow FP64 CPU
 * implementation of the per-patch finite-volume step described in Qin,
 * LeVeque & Motley, "Efficient tsunami modeling on adaptive grids with
 * graphics processing units" (Sec. 2: the shallow water equations, the
 * wave-propagation update and its limited second-order corrections, the
 * dimensionally split 2D form and the CFL condition).  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may call it.  It
 * shares no code with the HIP library and neither includes the other.
 *
 * Storage is array-of-structures: cell (i, j) of a patch with mx x my interior
 * cells and two ghost layers keeps (h, hu, hv) at q[((j * (mx + 4)) + i) * 3],
 * with 0 <= i < mx + 4, 0 <= j < my + 4 and the interior at 2 <= i, j.
 * Bathymetry b uses the same (i, j) indexing with one value per cell.
 */
#ifndef SWE_ORACLE_H
#define SWE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double g;             /* gravity [m s^-2] */
    double drytol;        /* a cell with h <= drytol is dry */
    double manning_n;     /* Manning coefficient, 0 disables friction */
    double cfl_desired;   /* target Courant number for the next step */
    double cfl_max;       /* a step whose Courant number exceeds this is retaken */
    double h_corr;        /* no limited correction at an edge with a cell at or below this depth */
    int32_t method;       /* 0 = dimensionally split, 1 = unsplit with transverse waves */
    int32_t order;        /* 1 = Godunov fluctuations only, 2 = add limited corrections */
    int32_t transverse_order; /* unsplit only: 1 = A+-dQ, 2 = A+-dQ with corrections */
    int32_t pad_;
} orc_params;

enum { ORC_BC_WALL = 0, ORC_BC_EXTRAP = 1, ORC_BC_USER = 2 };

typedef struct {
    int32_t mx, my;       /* interior cells */
    double dx, dy;        /* cell sizes [m] */
    int32_t bc[4];        /* xlo, xhi, ylo, yhi */
} orc_grid;

/* Edge kinds reported by the Riemann solver. */
enum { ORC_EDGE_WET = 0, ORC_EDGE_WALL_R = 1, ORC_EDGE_WALL_L = 2, ORC_EDGE_DRY = 3 };

typedef struct {
    double z[3][3];       /* z[p][k]: f-wave p, component k = (mass, normal mom., transverse mom.) */
    double s[3];          /* speeds */
    int32_t kind;
    int32_t clamped;      /* 1 if the stationary bathymetry jump hit a positivity bound */
    int32_t shallow;      /* 1 if a cell of the edge is at or below h_corr deep */
    int32_t pad_;
} orc_waves;

void orc_riemann(const orc_params *P,
                 double hL, double mL, double tL, double bL,
                 double hR, double mR, double tR, double bR,
                 orc_waves *w);
void orc_fluctuations(const orc_waves *w, double amdq[3], double apdq[3]);
double orc_mc_limiter(double theta);

void orc_ghost_fill(const orc_grid *G, double *q);
void orc_ghost_fill_b(const orc_grid *G, double *b);

/* One step from q_in (ghosts filled) to q_out.  smax[0], smax[1] receive the
 * largest wave speeds over the x- and y-edges of interior cells.  Returns the
 * number of cells whose depth had to be clamped at zero; *nonfinite is set to
 * 1 if an updated value is not finite. */
int64_t orc_step(const orc_params *P, const orc_grid *G, const double *q_in,
                 const double *b, double dt, double *q_out, double smax[2],
                 int32_t *nonfinite);

/* Wave speeds of the state q (ghosts filled) without updating it. */
void orc_speed_scan(const orc_params *P, const orc_grid *G, const double *q,
                    const double *b, double smax[2]);

/* Time loop with the CFL rule.  q is advanced in place nsteps times.  If
 * dt_forced is not NULL the step sizes are taken from it and no CFL control is
 * applied.  Otherwise the first dt comes from dt0 (or from a speed scan when
 * dt0 <= 0) and every later one from the speeds of the previous step; a step
 * whose Courant number exceeds cfl_max is discarded and retaken.  dt_used
 * (nsteps values) receives the accepted step sizes.  Returns clamp count. */
int64_t orc_run(const orc_params *P, const orc_grid *G, double *q, const double *b,
                int32_t nsteps, double dt0, const double *dt_forced,
                double *dt_used, int32_t *retakes, int32_t *nonfinite);

/* Sum of h over interior cells times dx * dy. */
double orc_mass(const orc_grid *G, const double *q);

/* OpenMP thread count of the row loops. */
void orc_set_threads(int32_t n);
int32_t orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
