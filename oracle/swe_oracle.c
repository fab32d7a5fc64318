/*
 * swe_oracle.c -- reference solver for the 2D shallow water step (FP64, CPU).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the library.  Written for readability:
 * every step below follows the paper's Sec. 2 (equations swe, the
 * wave-propagation form, its second-order form, theta and the limiter, the
 * split x/y forms and the CFL condition) in the paper's order.  The paper only
 * cites its Riemann solver (an augmented solver that keeps the ocean at rest,
 * handles dry states and keeps depth non-negative); the reading implemented
 * here is written out from the mathematics in orc_riemann below.
 *
 * Built with -ffp-contract=off so that every product and sum is rounded as
 * written.
 */
#include "swe_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NQ 3
#define IDX(G, i, j) ((size_t)(j) * (size_t)((G)->mx + 4) + (size_t)(i))

/* ------------------------------------------------------------------------ */
/* MC limiter, Sec. 2 (limiter function Phi, MC limiter used in all runs).   */
double orc_mc_limiter(double theta)
{
    double a = 0.5 * (1.0 + theta);
    double c = 2.0 * theta;
    double m = a < 2.0 ? a : 2.0;
    m = m < c ? m : c;
    return m > 0.0 ? m : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Augmented Riemann solver, one edge, normal direction "n".                 */
/*
 * Inputs per side: depth h, normal momentum m, transverse momentum t, bed b.
 * Output: three f-waves Z^p (their sum equals the flux jump plus the bed
 * source, so the update conserves mass) and speeds s^p.
 *
 *  dry test      a side with h <= drytol is dry; its velocities and momenta
 *                are taken as 0 while its stored depth is kept;
 *  wall test     if one side is dry and the water on the other side cannot
 *                reach over its bed (two-rarefaction run-up estimate), the dry
 *                side is replaced by the mirror image of the wet side;
 *  speeds        Einfeldt-type bounds from the Roe average, dry-front speeds
 *                u -/+ 2c when one side is dry;
 *  bed jump      the stationary jump of the depth is -(b_R - b_L), bounded so
 *                that both middle depths of the HLL state stay >= 0;
 *  decomposition mass/momentum jumps into waves at s1, s3 and a corrector
 *                wave at (s1 + s3) / 2 carrying the rest of the momentum flux
 *                and the transverse momentum.
 */
void orc_riemann(const orc_params *P,
                 double hL, double mL, double tL, double bL,
                 double hR, double mR, double tR, double bR,
                 orc_waves *w)
{
    const double g = P->g;
    const double eps = P->drytol;
    memset(w, 0, sizeof(*w));
    w->kind = ORC_EDGE_WET;
    w->shallow = hL <= P->h_corr || hR <= P->h_corr;

    int dryL = hL <= eps;
    int dryR = hR <= eps;
    if (dryL && dryR) {
        w->kind = ORC_EDGE_DRY;
        return;
    }

    double uL = 0.0, vL = 0.0, uR = 0.0, vR = 0.0;
    if (dryL) {
        mL = 0.0;
        tL = 0.0;
    } else {
        uL = mL / hL;
        vL = tL / hL;
    }
    if (dryR) {
        mR = 0.0;
        tR = 0.0;
    } else {
        uR = mR / hR;
        vR = tR / hR;
    }

    /* wall test */
    if (dryR) {
        double a = sqrt(g * hL) + 0.5 * uL;
        if (a < 0.0) a = 0.0;
        double hstar = a * a / g;
        if (hstar < hL) hstar = hL;
        if (hstar + bL < bR) {
            w->kind = ORC_EDGE_WALL_R;
            hR = hL;
            mR = -mL;
            tR = tL;
            bR = bL;
            uR = -uL;
            vR = vL;
            dryR = 0;
        }
    } else if (dryL) {
        double a = sqrt(g * hR) - 0.5 * uR;
        if (a < 0.0) a = 0.0;
        double hstar = a * a / g;
        if (hstar < hR) hstar = hR;
        if (hstar + bR < bL) {
            w->kind = ORC_EDGE_WALL_L;
            hL = hR;
            mL = -mR;
            tL = tR;
            bL = bR;
            uL = -uR;
            vL = vR;
            dryL = 0;
        }
    }

    /* speeds */
    double s1, s3;
    if (dryR) {
        double cL = sqrt(g * hL);
        s1 = uL - cL;
        s3 = uL + 2.0 * cL;
    } else if (dryL) {
        double cR = sqrt(g * hR);
        s1 = uR - 2.0 * cR;
        s3 = uR + cR;
    } else {
        double cL = sqrt(g * hL);
        double cR = sqrt(g * hR);
        double rL = sqrt(hL);
        double rR = sqrt(hR);
        double uhat = (rL * uL + rR * uR) / (rL + rR);
        double chat = sqrt(g * (0.5 * (hL + hR)));
        double a = uL - cL, c = uhat - chat;
        s1 = a < c ? a : c;
        a = uR + cR;
        c = uhat + chat;
        s3 = a > c ? a : c;
    }
    double s2 = 0.5 * (s1 + s3);

    /* HLL middle depth */
    double dm = mR - mL;
    double hm = (s3 * hR - s1 * hL - dm) / (s3 - s1);
    if (hm < 0.0) hm = 0.0;

    /* Stationary bed jump.  Taken as -(b_R - b_L) unless that would make a
     * middle depth of the HLL state negative; the two middle depths of the
     * unclamped decomposition are h_L + beta1 and h_R - beta3.  Testing them
     * (rather than comparing the jump with the bounds h_m (s3 - s1) / s3 and
     * h_m (s3 - s1) / s1 directly) gives the same bounds in exact arithmetic and
     * never clamps a lake at rest, where the surface jump is exactly 0. */
    double db = bR - bL;
    double deta = (hR - hL) + db;
    double delta = -db;
    int clamped = 0;
    int bound = 0; /* 1: the left middle depth was bounded, 3: the right one */
    if (s1 < 0.0 && s3 > 0.0) {
        double b1 = (s3 * deta - dm) / (s3 - s1);
        double b3 = (dm - s1 * deta) / (s3 - s1);
        if (hL + b1 < 0.0) {
            delta = hm * (s3 - s1) / s3;
            clamped = 1;
            bound = 1;
        } else if (hR - b3 < 0.0) {
            delta = hm * (s3 - s1) / s1;
            clamped = 1;
            bound = 3;
        }
    } else if (s1 >= 0.0) {
        if (delta < -hL) {
            delta = -hL;
            clamped = 1;
        }
    } else {
        if (delta > hR) {
            delta = hR;
            clamped = 1;
        }
    }

    /* jumps; the surface jump is formed first so a lake at rest gives 0 */
    double dh = clamped ? (hR - hL) - delta : deta;
    double hbar = 0.5 * (hL + hR);
    double dphi = (mR * uR - mL * uL) + g * hbar * deta;
    double dt = mR * vR - mL * vL;

    /* decomposition.  With the jump at a bound (and a positive HLL middle
     * depth), that side's middle depth is zero in exact arithmetic: beta1 =
     * -h_L at the left bound, beta3 = h_R at the right one.  That coefficient
     * is taken at its exact value (computed, it can come out a rounding error
     * past it and drain a dry cell to a negative depth), and the other one
     * from the mass flux, s1 beta1 + s3 beta3 = dm, as the decomposition
     * satisfies it in exact arithmetic. */
    double beta1, beta3;
    if (bound == 1 && hm > 0.0) {
        beta1 = -hL;
        beta3 = (dm + s1 * hL) / s3;
    } else if (bound == 3 && hm > 0.0) {
        beta3 = hR;
        beta1 = (dm - s3 * hR) / s1;
    } else {
        beta1 = (s3 * dh - dm) / (s3 - s1);
        beta3 = (dm - s1 * dh) / (s3 - s1);
    }
    /* the two subtracted terms are summed first so that the solve is exactly
     * symmetric under reflection x -> -x */
    double beta2 = dphi - (s1 * s1 * beta1 + s3 * s3 * beta3);

    w->z[0][0] = s1 * beta1;
    w->z[0][1] = s1 * s1 * beta1;
    w->z[0][2] = s1 * beta1 * vL;
    w->z[2][0] = s3 * beta3;
    w->z[2][1] = s3 * s3 * beta3;
    w->z[2][2] = s3 * beta3 * vR;
    w->z[1][0] = 0.0;
    w->z[1][1] = beta2;
    w->z[1][2] = dt - (s1 * beta1 * vL + s3 * beta3 * vR);
    w->s[0] = s1;
    w->s[1] = s2;
    w->s[2] = s3;
    w->clamped = clamped;

    /* a wall reflects: waves running into the dry bank are removed */
    for (int p = 0; p < 3; ++p) {
        int drop = (w->kind == ORC_EDGE_WALL_R && w->s[p] > 0.0) ||
                   (w->kind == ORC_EDGE_WALL_L && w->s[p] < 0.0);
        if (drop) {
            w->s[p] = 0.0;
            w->z[p][0] = w->z[p][1] = w->z[p][2] = 0.0;
        }
    }
}

/* Fluctuations, Sec. 2 wave-propagation form: A-dQ collects left-going waves,
 * A+dQ right-going ones; a wave with zero speed is shared half and half.  At a
 * wall edge the side facing the dry bank receives nothing. */
void orc_fluctuations(const orc_waves *w, double amdq[3], double apdq[3])
{
    for (int k = 0; k < NQ; ++k) {
        amdq[k] = 0.0;
        apdq[k] = 0.0;
    }
    for (int p = 0; p < 3; ++p) {
        for (int k = 0; k < NQ; ++k) {
            if (w->s[p] < 0.0) {
                amdq[k] += w->z[p][k];
            } else if (w->s[p] > 0.0) {
                apdq[k] += w->z[p][k];
            } else {
                amdq[k] += 0.5 * w->z[p][k];
                apdq[k] += 0.5 * w->z[p][k];
            }
        }
    }
    if (w->kind == ORC_EDGE_WALL_R)
        for (int k = 0; k < NQ; ++k) apdq[k] = 0.0;
    if (w->kind == ORC_EDGE_WALL_L)
        for (int k = 0; k < NQ; ++k) amdq[k] = 0.0;
}

static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Limited second-order correction at edge e from the waves at e-1, e, e+1
 * (Sec. 2: theta against the upwind edge, MC limiter, correction flux).  The
 * waves are f-waves Z = s W, so |s| W = sign(s) Z.  An edge with a cell at or
 * below h_corr deep (a film of water on the shore) keeps the first-order
 * update: there a limited momentum correction is large against the momentum
 * the film holds, and the film's velocity m / h spikes.  Elsewhere the split
 * mode also bounds each correction by the water of its donor cell
 * (positivity_limit below). */
static void correction(const orc_waves *wl, const orc_waves *w, const orc_waves *wr,
                       double lam, double F[3])
{
    F[0] = F[1] = F[2] = 0.0;
    if (w->shallow) return;
    for (int p = 0; p < 3; ++p) {
        double s = w->s[p];
        if (s == 0.0) continue;
        double zz = dot3(w->z[p], w->z[p]);
        if (zz == 0.0) continue;
        const orc_waves *up = s > 0.0 ? wl : wr;
        double theta = dot3(up->z[p], w->z[p]) / zz;
        double phi = orc_mc_limiter(theta);
        double sg = s > 0.0 ? 1.0 : -1.0;
        double coef = 0.5 * sg * (1.0 - lam * fabs(s)) * phi;
        for (int k = 0; k < NQ; ++k) F[k] += coef * w->z[p][k];
    }
}

/* ------------------------------------------------------------------------ */
/* Boundary conditions: wall mirrors the cells across the boundary and negates
 * the normal momentum; extrapolation copies the nearest interior cell.  The
 * x-ghosts of the interior rows are filled first, then the y-ghosts of every
 * column, which fills the corners. */
static void fill_generic(const orc_grid *G, double *a, int ncomp, int is_state)
{
    const int mx = G->mx, my = G->my;
    for (int j = 2; j < my + 2; ++j) {
        for (int gcell = 0; gcell < 2; ++gcell) {
            /* xlo: ghost i = 1 - gcell mirrors interior 2 + gcell */
            int gi = 1 - gcell;
            int src = G->bc[0] == ORC_BC_WALL ? 2 + gcell : 2;
            if (G->bc[0] != ORC_BC_USER) {
                for (int k = 0; k < ncomp; ++k) a[IDX(G, gi, j) * ncomp + k] = a[IDX(G, src, j) * ncomp + k];
                if (is_state && G->bc[0] == ORC_BC_WALL) a[IDX(G, gi, j) * ncomp + 1] = -a[IDX(G, gi, j) * ncomp + 1];
            }
            /* xhi: ghost i = mx + 2 + gcell mirrors interior mx + 1 - gcell */
            gi = mx + 2 + gcell;
            src = G->bc[1] == ORC_BC_WALL ? mx + 1 - gcell : mx + 1;
            if (G->bc[1] != ORC_BC_USER) {
                for (int k = 0; k < ncomp; ++k) a[IDX(G, gi, j) * ncomp + k] = a[IDX(G, src, j) * ncomp + k];
                if (is_state && G->bc[1] == ORC_BC_WALL) a[IDX(G, gi, j) * ncomp + 1] = -a[IDX(G, gi, j) * ncomp + 1];
            }
        }
    }
    for (int i = 0; i < mx + 4; ++i) {
        for (int gcell = 0; gcell < 2; ++gcell) {
            int gj = 1 - gcell;
            int src = G->bc[2] == ORC_BC_WALL ? 2 + gcell : 2;
            if (G->bc[2] != ORC_BC_USER) {
                for (int k = 0; k < ncomp; ++k) a[IDX(G, i, gj) * ncomp + k] = a[IDX(G, i, src) * ncomp + k];
                if (is_state && G->bc[2] == ORC_BC_WALL) a[IDX(G, i, gj) * ncomp + 2] = -a[IDX(G, i, gj) * ncomp + 2];
            }
            gj = my + 2 + gcell;
            src = G->bc[3] == ORC_BC_WALL ? my + 1 - gcell : my + 1;
            if (G->bc[3] != ORC_BC_USER) {
                for (int k = 0; k < ncomp; ++k) a[IDX(G, i, gj) * ncomp + k] = a[IDX(G, i, src) * ncomp + k];
                if (is_state && G->bc[3] == ORC_BC_WALL) a[IDX(G, i, gj) * ncomp + 2] = -a[IDX(G, i, gj) * ncomp + 2];
            }
        }
    }
}

void orc_ghost_fill(const orc_grid *G, double *q) { fill_generic(G, q, NQ, 1); }
void orc_ghost_fill_b(const orc_grid *G, double *b) { fill_generic(G, b, 1, 0); }

/* ------------------------------------------------------------------------ */
/* One 1D line of a sweep.  line[c] = (h, normal mom., transverse mom., b) for
 * c = 0 .. n + 3 (two ghosts each side).  Cells c = 2 .. n + 1 are updated
 * into out[c][0..2].  Edge e lies between cells e - 1 and e. */
static void friction(const orc_params *P, const orc_grid *G, double *q, double dt);

typedef struct {
    orc_waves *w;       /* n + 4 */
    double (*amdq)[3];
    double (*apdq)[3];
    double (*F)[3];
} line_work;

/* Share of a cell's water that one edge's correction may carry out of it.
 * Sec. 2 asks the scheme to keep depths non-negative.  The first-order
 * update of a sweep keeps them (the solver's middle depths are non-negative;
 * with Courant numbers of the two edges of a cell summing to at most 1); the
 * limited corrections can draw more water out of a cell than it holds, also
 * just above h_corr.  A cell has two edges per sweep, so each correction may
 * take at most half of its donor's first-order depth; the share sits 5e-13
 * below a half so that the rounding of the update cannot take a drained cell
 * below zero. */
#define ORC_DRAIN_SHARE 0.4999999999995

/* Positivity limit of the corrections of one sweep line.  For edge e the
 * donor d is the cell the correction's mass flux F[e][0] leaves (e - 1 if it
 * is positive, e if negative); h1 is d's depth after the first-order part of
 * its update, and the correction takes coef * F[e][0] out of d, with coef
 * the factor of F[e] in d's update.  If that exceeds ORC_DRAIN_SHARE * h1
 * (0 for h1 <= 0), the whole correction F[e] is scaled down to it.
 * kap == NULL: a Cartesian line, coef = lam, h1 = h - lam (A+dQ + A-dQ);
 * otherwise a latitude-longitude line (see sweep_line_metric): coef =
 * lam / kap[d] * len[e] and h1 includes the mass term of that update. */
static void positivity_limit(int n, double lam, const double (*line)[4], line_work *W,
                             const double *kap, const double *len)
{
    for (int e = 2; e <= n + 2; ++e) {
        double f = W->F[e][0];
        if (f == 0.0) continue;
        int d = f > 0.0 ? e - 1 : e;
        double h1, out;
        if (!kap) {
            h1 = line[d][0] - lam * (W->apdq[d][0] + W->amdq[d + 1][0]);
            out = lam * fabs(f);
        } else {
            double lc = lam / kap[d];
            h1 = (line[d][0] - lc * (len[d] * W->apdq[d][0] + len[d + 1] * W->amdq[d + 1][0]))
                 + lc * (line[d][1] * (len[d] - len[d + 1]));
            out = lc * (len[e] * fabs(f));
        }
        double cap = h1 > 0.0 ? ORC_DRAIN_SHARE * h1 : 0.0;
        if (out > cap) {
            double r = cap / out;
            for (int k = 0; k < NQ; ++k) W->F[e][k] = r * W->F[e][k];
        }
    }
}

static void sweep_line(const orc_params *P, int n, double lam, const double (*line)[4],
                       double (*out)[3], line_work *W, double *smax)
{
    for (int e = 1; e <= n + 3; ++e)
        orc_riemann(P, line[e - 1][0], line[e - 1][1], line[e - 1][2], line[e - 1][3],
                    line[e][0], line[e][1], line[e][2], line[e][3], &W->w[e]);
    /* fluctuations of every solved edge: the updated cells use edges 2 .. n + 2,
     * the donors of the positivity limit edges 1 .. n + 3 */
    for (int e = 1; e <= n + 3; ++e) orc_fluctuations(&W->w[e], W->amdq[e], W->apdq[e]);
    for (int e = 2; e <= n + 2; ++e) {
        if (P->order >= 2)
            correction(&W->w[e - 1], &W->w[e], &W->w[e + 1], lam, W->F[e]);
        else
            W->F[e][0] = W->F[e][1] = W->F[e][2] = 0.0;
        for (int p = 0; p < 3; ++p) {
            double a = fabs(W->w[e].s[p]);
            if (a > *smax) *smax = a;
        }
    }
    if (P->order >= 2) positivity_limit(n, lam, line, W, NULL, NULL);
    for (int c = 2; c <= n + 1; ++c)
        for (int k = 0; k < NQ; ++k)
            out[c][k] = line[c][k] - lam * (W->apdq[c][k] + W->amdq[c + 1][k])
                                   - lam * (W->F[c + 1][k] - W->F[c][k]);
}

static void line_work_alloc(line_work *W, int n)
{
    W->w = calloc((size_t)n + 4, sizeof(orc_waves));
    W->amdq = calloc((size_t)n + 4, sizeof(*W->amdq));
    W->apdq = calloc((size_t)n + 4, sizeof(*W->apdq));
    W->F = calloc((size_t)n + 4, sizeof(*W->F));
}

static void line_work_free(line_work *W)
{
    free(W->w);
    free(W->amdq);
    free(W->apdq);
    free(W->F);
}

/* Dry cleanup after a sweep: a cell at or below the dry tolerance holds no
 * momentum; a negative depth is set to zero and counted. */
static int64_t cleanup(const orc_params *P, double *qc, int32_t *nonfinite)
{
    int64_t clamp = 0;
    if (!(isfinite(qc[0]) && isfinite(qc[1]) && isfinite(qc[2]))) *nonfinite = 1;
    if (qc[0] < 0.0) {
        qc[0] = qc[1] = qc[2] = 0.0;
        clamp = 1;
    } else if (qc[0] <= P->drytol) {
        qc[1] = qc[2] = 0.0;
    }
    return clamp;
}

/* Dimensionally split step: x-sweep of every row (ghost rows included) into
 * Q*, then y-sweep of every interior column of Q* into Q^{n+1}. */
static int64_t split_step(const orc_params *P, const orc_grid *G, const double *q_in,
                          const double *b, double dt, double *q_out, double smax[2],
                          int32_t *nonfinite)
{
    const int mx = G->mx, my = G->my;
    const size_t ncell = (size_t)(mx + 4) * (size_t)(my + 4);
    double *qs = malloc(ncell * NQ * sizeof(double));
    memcpy(qs, q_in, ncell * NQ * sizeof(double));
    int64_t clamps = 0;
    double sx = 0.0, sy = 0.0;
    const double lamx = dt / G->dx, lamy = dt / G->dy;

#pragma omp parallel reduction(+ : clamps) reduction(max : sx)
    {
        line_work W;
        line_work_alloc(&W, mx);
        double (*line)[4] = malloc(sizeof(*line) * (size_t)(mx + 4));
        double (*out)[3] = malloc(sizeof(*out) * (size_t)(mx + 4));
        int32_t nf = 0;
#pragma omp for schedule(static)
        for (int j = 0; j < my + 4; ++j) {
            for (int c = 0; c < mx + 4; ++c) {
                const double *qc = &q_in[IDX(G, c, j) * NQ];
                line[c][0] = qc[0];
                line[c][1] = qc[1];
                line[c][2] = qc[2];
                line[c][3] = b[IDX(G, c, j)];
            }
            double s = 0.0;
            sweep_line(P, mx, lamx, (const double (*)[4])line, out, &W, &s);
            int interior = j >= 2 && j < my + 2;
            if (interior && s > sx) sx = s;
            for (int c = 2; c <= mx + 1; ++c) {
                double *qc = &qs[IDX(G, c, j) * NQ];
                qc[0] = out[c][0];
                qc[1] = out[c][1];
                qc[2] = out[c][2];
                int64_t cl = cleanup(P, qc, &nf);
                if (interior) clamps += cl;
            }
        }
        if (nf) {
#pragma omp atomic write
            *nonfinite = 1;
        }
        line_work_free(&W);
        free(line);
        free(out);
    }

    memcpy(q_out, q_in, ncell * NQ * sizeof(double));
#pragma omp parallel reduction(+ : clamps) reduction(max : sy)
    {
        line_work W;
        line_work_alloc(&W, my);
        double (*line)[4] = malloc(sizeof(*line) * (size_t)(my + 4));
        double (*out)[3] = malloc(sizeof(*out) * (size_t)(my + 4));
        int32_t nf = 0;
#pragma omp for schedule(static)
        for (int i = 2; i < mx + 2; ++i) {
            for (int c = 0; c < my + 4; ++c) {
                const double *qc = &qs[IDX(G, i, c) * NQ];
                line[c][0] = qc[0];
                line[c][1] = qc[2]; /* normal momentum of the y-sweep is hv */
                line[c][2] = qc[1];
                line[c][3] = b[IDX(G, i, c)];
            }
            double s = 0.0;
            sweep_line(P, my, lamy, (const double (*)[4])line, out, &W, &s);
            if (s > sy) sy = s;
            for (int c = 2; c <= my + 1; ++c) {
                double *qc = &q_out[IDX(G, i, c) * NQ];
                qc[0] = out[c][0];
                qc[1] = out[c][2];
                qc[2] = out[c][1];
                clamps += cleanup(P, qc, &nf);
            }
        }
        if (nf) {
#pragma omp atomic write
            *nonfinite = 1;
        }
        line_work_free(&W);
        free(line);
        free(out);
    }
    free(qs);
    smax[0] = sx;
    smax[1] = sy;
    return clamps;
}

/* ------------------------------------------------------------------------ */
/* Latitude-longitude patches (an extension; the paper's runs use such grids
 * but state no formulas).  Cells are Dlon x Dlat on a sphere of radius R;
 * the momentum equations keep the pressure gradient exact (the edge-scaled
 * fluctuations supply its metric part) and drop the curvature terms of size
 * u^2 / R; the mass equation is corrected to the conservative form.
 * dx = R Dlon and dy = R Dlat are their extents at the equator.  A cell's
 * area is kappa dx dy with the capacity kappa_j = (sin phi_{j+1/2} -
 * sin phi_{j-1/2}) / Dlat; a meridian edge is dy long, a parallel edge at
 * phi_{e-1/2} is len_e dx long with len_e = cos phi_{e-1/2}.  A cell changes
 * by dt / (kappa dx dy) times the sum over its edges of edge length times
 * what enters through the edge: in x, lam / kappa_j times the fluctuations
 * and correction differences; in y, the same with each edge's amounts scaled
 * by len_e.  The correction at an edge uses the edge's Courant factor lam
 * times the mean inverse capacity of its two cells, and the speed reported
 * for the CFL condition is |s| times that mean.  No curvature or Coriolis
 * source terms.  The mass gets the correction described in the update. */
static void sweep_line_metric(const orc_params *P, int n, double lam, const double (*line)[4],
                              double (*out)[3], line_work *W, double *smax, const double *kap,
                              const double *len)
{
    for (int e = 1; e <= n + 3; ++e)
        orc_riemann(P, line[e - 1][0], line[e - 1][1], line[e - 1][2], line[e - 1][3],
                    line[e][0], line[e][1], line[e][2], line[e][3], &W->w[e]);
    for (int e = 1; e <= n + 3; ++e) orc_fluctuations(&W->w[e], W->amdq[e], W->apdq[e]);
    for (int e = 2; e <= n + 2; ++e) {
        const double a = 0.5 * (1.0 / kap[e - 1] + 1.0 / kap[e]);
        if (P->order >= 2)
            correction(&W->w[e - 1], &W->w[e], &W->w[e + 1], lam * a, W->F[e]);
        else
            W->F[e][0] = W->F[e][1] = W->F[e][2] = 0.0;
        for (int p = 0; p < 3; ++p) {
            double v = fabs(W->w[e].s[p]) * a;
            if (v > *smax) *smax = v;
        }
    }
    if (P->order >= 2) positivity_limit(n, lam, line, W, kap, len);
    for (int c = 2; c <= n + 1; ++c) {
        const double lc = lam / kap[c];
        const double *ap = W->apdq[c], *am = W->amdq[c + 1];  /* edges c, c + 1 */
        for (int k = 0; k < NQ; ++k)
            out[c][k] = line[c][k] - lc * (len[c] * ap[k] + len[c + 1] * am[k])
                                   - lc * (len[c + 1] * W->F[c + 1][k] - len[c] * W->F[c][k]);
        /* the edge-scaled fluctuations of a cell add up to the conservative
         * flux difference plus f(Q_c) (len_c - len_{c+1}); for the mass that
         * term is spurious (the continuity equation has no metric source), so
         * it is taken out: f = the normal momentum */
        out[c][0] += lc * (line[c][1] * (len[c] - len[c + 1]));
    }
}

/* Split step on a latitude-longitude patch: kap[j] for rows j = 0 .. my + 3,
 * len[e] for the edge between rows e - 1 and e, e = 1 .. my + 3. */
int64_t orc_step_sphere(const orc_params *P, const orc_grid *G, const double *q_in,
                        const double *b, double dt, const double *kap, const double *len,
                        double *q_out, double smax[2], int32_t *nonfinite)
{
    const int mx = G->mx, my = G->my;
    const size_t ncell = (size_t)(mx + 4) * (size_t)(my + 4);
    double *qs = malloc(ncell * NQ * sizeof(double));
    memcpy(qs, q_in, ncell * NQ * sizeof(double));
    int64_t clamps = 0;
    double sx = 0.0, sy = 0.0;
    int32_t nf = 0;
    const double lamx = dt / G->dx, lamy = dt / G->dy;
    line_work W;
    line_work_alloc(&W, mx > my ? mx : my);
    const int nmax = (mx > my ? mx : my) + 4;
    double (*line)[4] = malloc(sizeof(*line) * (size_t)nmax);
    double (*out)[3] = malloc(sizeof(*out) * (size_t)nmax);
    double *kline = malloc(sizeof(double) * (size_t)nmax);
    double *ones = malloc(sizeof(double) * (size_t)(nmax + 1));
    for (int c = 0; c <= nmax; ++c) ones[c] = 1.0;
    for (int j = 0; j < my + 4; ++j) {
        for (int c = 0; c < mx + 4; ++c) {
            const double *qc = &q_in[IDX(G, c, j) * NQ];
            line[c][0] = qc[0];
            line[c][1] = qc[1];
            line[c][2] = qc[2];
            line[c][3] = b[IDX(G, c, j)];
            kline[c] = kap[j];
        }
        double s = 0.0;
        sweep_line_metric(P, mx, lamx, (const double (*)[4])line, out, &W, &s, kline, ones);
        int interior = j >= 2 && j < my + 2;
        if (interior && s > sx) sx = s;
        for (int c = 2; c <= mx + 1; ++c) {
            double *qc = &qs[IDX(G, c, j) * NQ];
            qc[0] = out[c][0];
            qc[1] = out[c][1];
            qc[2] = out[c][2];
            int64_t cl = cleanup(P, qc, &nf);
            if (interior) clamps += cl;
        }
    }
    memcpy(q_out, q_in, ncell * NQ * sizeof(double));
    for (int i = 2; i < mx + 2; ++i) {
        for (int c = 0; c < my + 4; ++c) {
            const double *qc = &qs[IDX(G, i, c) * NQ];
            line[c][0] = qc[0];
            line[c][1] = qc[2];
            line[c][2] = qc[1];
            line[c][3] = b[IDX(G, i, c)];
        }
        double s = 0.0;
        sweep_line_metric(P, my, lamy, (const double (*)[4])line, out, &W, &s, kap, len);
        if (s > sy) sy = s;
        for (int c = 2; c <= my + 1; ++c) {
            double *qc = &q_out[IDX(G, i, c) * NQ];
            qc[0] = out[c][0];
            qc[1] = out[c][2];
            qc[2] = out[c][1];
            clamps += cleanup(P, qc, &nf);
        }
    }
    line_work_free(&W);
    free(line);
    free(out);
    free(kline);
    free(ones);
    free(qs);
    friction(P, G, q_out, dt);
    smax[0] = sx;
    smax[1] = sy;
    if (nonfinite) *nonfinite = nf;
    return clamps;
}

/* ------------------------------------------------------------------------ */
/* Unsplit step with transverse waves.  Every edge is solved from Q^n; the
 * fluctuation entering a cell through an x-edge is split by a Roe solver in y
 * into an up-going and a down-going part, which move part of that cell's
 * change into its upper or lower neighbour through the y-correction fluxes
 * (and the same with x and y exchanged). */

/* Transverse split of the amount a = (mass, normal, transverse) entering cell
 * C.  The pair (cl, cr) is ordered along the transverse direction; sgn = +1
 * returns the part moving toward cr (positive speeds), sgn = -1 the part
 * moving toward cl (negative speeds).  States are (h, normal, transverse, b);
 * "transverse" is the momentum along the direction of the split. */
static void transverse_part(const orc_params *P, const double *cl, const double *cr,
                            int c_is_left, const double a[3], int sgn, double out[3])
{
    const double eps = P->drytol, g = P->g;
    out[0] = out[1] = out[2] = 0.0;
    int dl = cl[0] <= eps, dr = cr[0] <= eps;
    if (dl && dr) return;
    const double *C = c_is_left ? cl : cr;
    const double *N = c_is_left ? cr : cl;
    int dn = N[0] <= eps;
    if (dn && N[3] >= C[0] + C[3]) return;
    double hl = cl[0], hr = cr[0];
    double unl = dl ? 0.0 : cl[1] / hl, utl = dl ? 0.0 : cl[2] / hl;
    double unr = dr ? 0.0 : cr[1] / hr, utr = dr ? 0.0 : cr[2] / hr;
    double rl = sqrt(hl), rr = sqrt(hr);
    double un = (rl * unl + rr * unr) / (rl + rr);
    double ut = (rl * utl + rr * utr) / (rl + rr);
    double c = sqrt(g * (0.5 * (hl + hr)));
    double lam[3] = {ut - c, ut, ut + c};
    double gam[3];
    gam[0] = ((ut + c) * a[0] - a[2]) / (2.0 * c);
    gam[1] = a[1] - un * a[0];
    gam[2] = (a[2] - (ut - c) * a[0]) / (2.0 * c);
    double r[3][3] = {{1.0, un, ut - c}, {0.0, 1.0, 0.0}, {1.0, un, ut + c}};
    for (int p = 0; p < 3; ++p) {
        double l = sgn > 0 ? (lam[p] > 0.0 ? lam[p] : 0.0) : (lam[p] < 0.0 ? lam[p] : 0.0);
        for (int k = 0; k < 3; ++k) out[k] += l * gam[p] * r[p][k];
    }
}

static int64_t unsplit_step(const orc_params *P, const orc_grid *G, const double *q_in,
                            const double *b, double dt, double *q_out, double smax[2],
                            int32_t *nonfinite)
{
    const int mx = G->mx, my = G->my;
    const int nx = mx + 4, ny = my + 4;
    const size_t ncell = (size_t)nx * (size_t)ny;
    const double lamx = dt / G->dx, lamy = dt / G->dy;
    /* per-edge arrays, x-edge (e, j) at [j * nx + e], y-edge (i, e) at [e * nx + i];
     * fluctuations and corrections in (h, hu, hv) order */
    double (*xam)[3] = calloc(ncell, sizeof(*xam));
    double (*xap)[3] = calloc(ncell, sizeof(*xap));
    double (*xF)[3] = calloc(ncell, sizeof(*xF));
    double (*yam)[3] = calloc(ncell, sizeof(*yam));
    double (*yap)[3] = calloc(ncell, sizeof(*yap));
    double (*yG)[3] = calloc(ncell, sizeof(*yG));
    double (*Ft)[3] = calloc(ncell, sizeof(*Ft)); /* final x-corrections */
    double (*Gt)[3] = calloc(ncell, sizeof(*Gt)); /* final y-corrections */
    double sx = 0.0, sy = 0.0;

    /* normal solves along x on rows 1 .. my + 2 */
    {
        line_work W;
        line_work_alloc(&W, mx);
        double (*line)[4] = malloc(sizeof(*line) * (size_t)nx);
        for (int j = 1; j <= my + 2; ++j) {
            for (int c = 0; c < nx; ++c) {
                const double *qc = &q_in[IDX(G, c, j) * NQ];
                line[c][0] = qc[0];
                line[c][1] = qc[1];
                line[c][2] = qc[2];
                line[c][3] = b[IDX(G, c, j)];
            }
            for (int e = 1; e <= mx + 3; ++e)
                orc_riemann(P, line[e - 1][0], line[e - 1][1], line[e - 1][2], line[e - 1][3],
                            line[e][0], line[e][1], line[e][2], line[e][3], &W.w[e]);
            for (int e = 2; e <= mx + 2; ++e) {
                size_t k = (size_t)j * nx + e;
                orc_fluctuations(&W.w[e], xam[k], xap[k]);
                if (P->order >= 2) correction(&W.w[e - 1], &W.w[e], &W.w[e + 1], lamx, xF[k]);
                if (j >= 2 && j <= my + 1)
                    for (int p = 0; p < 3; ++p)
                        if (fabs(W.w[e].s[p]) > sx) sx = fabs(W.w[e].s[p]);
            }
        }
        line_work_free(&W);
        free(line);
    }
    /* normal solves along y on columns 1 .. mx + 2 (components stored as h, hu, hv) */
    {
        line_work W;
        line_work_alloc(&W, my);
        double (*line)[4] = malloc(sizeof(*line) * (size_t)ny);
        for (int i = 1; i <= mx + 2; ++i) {
            for (int c = 0; c < ny; ++c) {
                const double *qc = &q_in[IDX(G, i, c) * NQ];
                line[c][0] = qc[0];
                line[c][1] = qc[2];
                line[c][2] = qc[1];
                line[c][3] = b[IDX(G, i, c)];
            }
            for (int e = 1; e <= my + 3; ++e)
                orc_riemann(P, line[e - 1][0], line[e - 1][1], line[e - 1][2], line[e - 1][3],
                            line[e][0], line[e][1], line[e][2], line[e][3], &W.w[e]);
            for (int e = 2; e <= my + 2; ++e) {
                size_t k = (size_t)e * nx + i;
                double am[3], ap[3], F[3] = {0.0, 0.0, 0.0};
                orc_fluctuations(&W.w[e], am, ap);
                if (P->order >= 2) correction(&W.w[e - 1], &W.w[e], &W.w[e + 1], lamy, F);
                yam[k][0] = am[0]; yam[k][1] = am[2]; yam[k][2] = am[1];
                yap[k][0] = ap[0]; yap[k][1] = ap[2]; yap[k][2] = ap[1];
                yG[k][0] = F[0]; yG[k][1] = F[2]; yG[k][2] = F[1];
                if (i >= 2 && i <= mx + 1)
                    for (int p = 0; p < 3; ++p)
                        if (fabs(W.w[e].s[p]) > sy) sy = fabs(W.w[e].s[p]);
            }
        }
        line_work_free(&W);
        free(line);
    }

    memcpy(Ft, xF, ncell * sizeof(*Ft));
    memcpy(Gt, yG, ncell * sizeof(*Gt));

    /* transverse propagation of x-edge fluctuations into the y-corrections */
    for (int j = 1; j <= my + 2; ++j) {
        for (int e = 2; e <= mx + 2; ++e) {
            size_t k = (size_t)j * nx + e;
            for (int side = 0; side < 2; ++side) {
                /* side 0: amount entering cell (e, j); side 1: entering (e - 1, j) */
                int ci = side == 0 ? e : e - 1;
                double a[3];
                for (int m = 0; m < 3; ++m) {
                    double corr = P->transverse_order >= 2 ? xF[k][m] : 0.0;
                    a[m] = side == 0 ? xap[k][m] - corr : xam[k][m] + corr;
                }
                /* in the y-split the normal momentum is hu, transverse is hv */
                double an[3] = {a[0], a[1], a[2]};
                double sc[4], sd[4], su[4];
                const double *qc = &q_in[IDX(G, ci, j) * NQ];
                sc[0] = qc[0]; sc[1] = qc[1]; sc[2] = qc[2]; sc[3] = b[IDX(G, ci, j)];
                if (j + 1 < ny) {
                    const double *qu = &q_in[IDX(G, ci, j + 1) * NQ];
                    su[0] = qu[0]; su[1] = qu[1]; su[2] = qu[2]; su[3] = b[IDX(G, ci, j + 1)];
                    double up[3];
                    transverse_part(P, sc, su, 1, an, +1, up);
                    size_t ky = (size_t)(j + 1) * nx + ci;
                    for (int m = 0; m < 3; ++m) Gt[ky][m] -= 0.5 * lamx * up[m];
                }
                if (j - 1 >= 0) {
                    const double *qd = &q_in[IDX(G, ci, j - 1) * NQ];
                    sd[0] = qd[0]; sd[1] = qd[1]; sd[2] = qd[2]; sd[3] = b[IDX(G, ci, j - 1)];
                    double dn[3];
                    transverse_part(P, sd, sc, 0, an, -1, dn);
                    size_t ky = (size_t)j * nx + ci;
                    for (int m = 0; m < 3; ++m) Gt[ky][m] -= 0.5 * lamx * dn[m];
                }
            }
        }
    }
    /* transverse propagation of y-edge fluctuations into the x-corrections */
    for (int i = 1; i <= mx + 2; ++i) {
        for (int e = 2; e <= my + 2; ++e) {
            size_t k = (size_t)e * nx + i;
            for (int side = 0; side < 2; ++side) {
                int cj = side == 0 ? e : e - 1;
                double a[3];
                for (int m = 0; m < 3; ++m) {
                    double corr = P->transverse_order >= 2 ? yG[k][m] : 0.0;
                    a[m] = side == 0 ? yap[k][m] - corr : yam[k][m] + corr;
                }
                /* local order for the x-split: (h, normal = hv, transverse = hu) */
                double an[3] = {a[0], a[2], a[1]};
                double sc[4], sl[4], sr[4];
                const double *qc = &q_in[IDX(G, i, cj) * NQ];
                sc[0] = qc[0]; sc[1] = qc[2]; sc[2] = qc[1]; sc[3] = b[IDX(G, i, cj)];
                if (i + 1 < nx) {
                    const double *qr = &q_in[IDX(G, i + 1, cj) * NQ];
                    sr[0] = qr[0]; sr[1] = qr[2]; sr[2] = qr[1]; sr[3] = b[IDX(G, i + 1, cj)];
                    double rt[3];
                    transverse_part(P, sc, sr, 1, an, +1, rt);
                    size_t kx = (size_t)cj * nx + (i + 1);
                    Ft[kx][0] -= 0.5 * lamy * rt[0];
                    Ft[kx][1] -= 0.5 * lamy * rt[2];
                    Ft[kx][2] -= 0.5 * lamy * rt[1];
                }
                if (i - 1 >= 0) {
                    const double *ql = &q_in[IDX(G, i - 1, cj) * NQ];
                    sl[0] = ql[0]; sl[1] = ql[2]; sl[2] = ql[1]; sl[3] = b[IDX(G, i - 1, cj)];
                    double lt[3];
                    transverse_part(P, sl, sc, 0, an, -1, lt);
                    size_t kx = (size_t)cj * nx + i;
                    Ft[kx][0] -= 0.5 * lamy * lt[0];
                    Ft[kx][1] -= 0.5 * lamy * lt[2];
                    Ft[kx][2] -= 0.5 * lamy * lt[1];
                }
            }
        }
    }

    memcpy(q_out, q_in, ncell * NQ * sizeof(double));
    int64_t clamps = 0;
    for (int j = 2; j <= my + 1; ++j) {
        for (int i = 2; i <= mx + 1; ++i) {
            size_t kc = (size_t)j * nx + i;
            size_t kr = (size_t)j * nx + (i + 1);
            size_t ku = (size_t)(j + 1) * nx + i;
            double *qc = &q_out[IDX(G, i, j) * NQ];
            const double *q0 = &q_in[IDX(G, i, j) * NQ];
            for (int m = 0; m < 3; ++m)
                qc[m] = q0[m] - lamx * (xap[kc][m] + xam[kr][m] + Ft[kr][m] - Ft[kc][m])
                              - lamy * (yap[kc][m] + yam[ku][m] + Gt[ku][m] - Gt[kc][m]);
            clamps += cleanup(P, qc, nonfinite);
        }
    }
    free(xam); free(xap); free(xF); free(yam); free(yap); free(yG); free(Ft); free(Gt);
    smax[0] = sx;
    smax[1] = sy;
    return clamps;
}

/* ------------------------------------------------------------------------ */
/* Manning friction (Sec. 2, drag D = n^2 g h^(-7/3) |u|), applied implicitly
 * to the momenta of wet cells after the hyperbolic update. */
static void friction(const orc_params *P, const orc_grid *G, double *q, double dt)
{
    if (P->manning_n <= 0.0) return;
    const double n2g = P->manning_n * P->manning_n * P->g;
    for (int j = 2; j < G->my + 2; ++j) {
        for (int i = 2; i < G->mx + 2; ++i) {
            double *qc = &q[IDX(G, i, j) * NQ];
            double h = qc[0];
            if (h <= P->drytol) continue;
            double speed = sqrt(qc[1] * qc[1] + qc[2] * qc[2]) / h;
            double D = n2g * pow(h, -7.0 / 3.0) * speed;
            double f = 1.0 / (1.0 + dt * D);
            qc[1] *= f;
            qc[2] *= f;
        }
    }
}

int64_t orc_step(const orc_params *P, const orc_grid *G, const double *q_in,
                 const double *b, double dt, double *q_out, double smax[2],
                 int32_t *nonfinite)
{
    int32_t nf = 0;
    int64_t c = P->method == 1 ? unsplit_step(P, G, q_in, b, dt, q_out, smax, &nf)
                               : split_step(P, G, q_in, b, dt, q_out, smax, &nf);
    friction(P, G, q_out, dt);
    if (nonfinite) *nonfinite = nf;
    return c;
}

void orc_speed_scan(const orc_params *P, const orc_grid *G, const double *q,
                    const double *b, double smax[2])
{
    double sx = 0.0, sy = 0.0;
    orc_waves w;
    for (int j = 2; j < G->my + 2; ++j) {
        for (int e = 2; e <= G->mx + 2; ++e) {
            const double *l = &q[IDX(G, e - 1, j) * NQ], *r = &q[IDX(G, e, j) * NQ];
            orc_riemann(P, l[0], l[1], l[2], b[IDX(G, e - 1, j)], r[0], r[1], r[2], b[IDX(G, e, j)], &w);
            for (int p = 0; p < 3; ++p)
                if (fabs(w.s[p]) > sx) sx = fabs(w.s[p]);
        }
    }
    for (int i = 2; i < G->mx + 2; ++i) {
        for (int e = 2; e <= G->my + 2; ++e) {
            const double *l = &q[IDX(G, i, e - 1) * NQ], *r = &q[IDX(G, i, e) * NQ];
            orc_riemann(P, l[0], l[2], l[1], b[IDX(G, i, e - 1)], r[0], r[2], r[1], b[IDX(G, i, e)], &w);
            for (int p = 0; p < 3; ++p)
                if (fabs(w.s[p]) > sy) sy = fabs(w.s[p]);
        }
    }
    smax[0] = sx;
    smax[1] = sy;
}

/* Courant rate max(sx / dx, sy / dy): dt times it is the Courant number. */
static double courant_rate(const orc_grid *G, const double smax[2])
{
    double rx = smax[0] / G->dx, ry = smax[1] / G->dy;
    return rx > ry ? rx : ry;
}

int64_t orc_run(const orc_params *P, const orc_grid *G, double *q, const double *b,
                int32_t nsteps, double dt0, const double *dt_forced,
                double *dt_used, int32_t *retakes, int32_t *nonfinite)
{
    const size_t n = (size_t)(G->mx + 4) * (size_t)(G->my + 4) * NQ;
    double *tmp = malloc(n * sizeof(double));
    int64_t clamps = 0;
    int32_t nretake = 0, nf_any = 0;
    double smax[2];
    double dt = dt0;
    if (!dt_forced && dt <= 0.0) {
        orc_ghost_fill(G, q);
        orc_speed_scan(P, G, q, b, smax);
        double r = courant_rate(G, smax);
        dt = r > 0.0 ? P->cfl_desired / r : 1.0;
    }
    for (int32_t s = 0; s < nsteps; ++s) {
        orc_ghost_fill(G, q);
        if (dt_forced) dt = dt_forced[s];
        for (;;) {
            int32_t nf = 0;
            int64_t c = orc_step(P, G, q, b, dt, tmp, smax, &nf);
            double r = courant_rate(G, smax);
            if (!dt_forced && r > 0.0 && dt * r > P->cfl_max) {
                /* too large a step: discard it and retake with the reduced dt */
                dt = P->cfl_desired / r;
                ++nretake;
                continue;
            }
            clamps += c;
            nf_any |= nf;
            memcpy(q, tmp, n * sizeof(double));
            if (dt_used) dt_used[s] = dt;
            if (!dt_forced && r > 0.0) dt = P->cfl_desired / r;
            break;
        }
    }
    free(tmp);
    if (retakes) *retakes = nretake;
    if (nonfinite) *nonfinite = nf_any;
    return clamps;
}

double orc_mass(const orc_grid *G, const double *q)
{
    double s = 0.0;
    for (int j = 2; j < G->my + 2; ++j)
        for (int i = 2; i < G->mx + 2; ++i) s += q[IDX(G, i, j) * NQ];
    return s * G->dx * G->dy;
}

/* Thread count for the OpenMP row loops (only the timing baseline changes it). */
#ifdef _OPENMP
#include <omp.h>
void orc_set_threads(int32_t n) { omp_set_num_threads(n > 0 ? n : 1); }
int32_t orc_get_threads(void) { return omp_get_max_threads(); }
#else
void orc_set_threads(int32_t n) { (void)n; }
int32_t orc_get_threads(void) { return 1; }
#endif
