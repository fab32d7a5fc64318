/*
 * swe.h -- C ABI of the MI355X (gfx950) shallow water patch-step library.
 *
 * The library advances patches of the 2D shallow water equations over
 * bathymetry (Qin, LeVeque & Motley, Sec. 2, equations swe) by one time step
 * of the wave-propagation method: an augmented Riemann solve at every edge
 * with wet/dry handling, the fluctuations A+-dQ and B+-dQ, limited
 * second-order corrections (MC limiter), dimensional splitting x then y
 * (Sec. 2, split x/y forms) or an unsplit update with transverse waves, and
 * the largest wave speed for the CFL condition (Sec. 2, CFL condition;
 * Sec. 4 keeps the Riemann solves, the limiter and the CFL reduction on the
 * GPU).  A patch is a rectangle of cells with two ghost layers and its
 * bathymetry (Sec. 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every pointer argument is a DEVICE pointer unless its comment says
 *    "host".  The caller owns all memory and streams; the library allocates
 *    nothing.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default
 *    stream.  Every call only enqueues work on `stream`: none synchronises,
 *    reads device data on the host or allocates, so every call can be
 *    captured into a HIP graph.  Step sizes are read from device memory, so
 *    a replayed graph needs no host update.
 *  - State planes.  A patch stores (h, hu, hv) in FP64 (precision SWE_F64) or
 *    (eta', hu, hv) in FP32 (precision SWE_F32_DEV, eta' = h + b - sea_level)
 *    as three planes of one element type; the bathymetry b is one plane of
 *    the same type.  Cell (i, j) of a patch, 0 <= i < mx + 4,
 *    0 <= j < my + 4 (interior 2 <= i < mx + 2, 2 <= j < my + 2), is element
 *        off + j * pitch + i
 *    of each plane; the planes of q are plane_stride elements apart (h first).
 *    b uses the same off and pitch.  SI units throughout.
 *  - Ghost cells.  Sides with boundary code SWE_BC_WALL (mirror, normal
 *    momentum negated) or SWE_BC_EXTRAP (copy of the nearest interior cell)
 *    are synthesised from the interior when a step loads the patch; their
 *    memory is neither read nor written by the step.  Sides with
 *    SWE_BC_USER are read from memory (the caller filled them, e.g. from a
 *    neighbouring patch).  The rule is: x-ghosts of interior rows from the
 *    x-sides, then y-ghosts of every column from the y-sides (which fills the
 *    corners).  swe_ghost_fill writes the same values into memory.
 *  - Return codes: SWE_OK (0); SWE_EINVAL (-1) for a bad shape, a null
 *    pointer, in/out aliasing or an unknown enum, detected on the host before
 *    anything is enqueued; SWE_EHIP (-2) for a HIP launch/runtime error.  The
 *    message of the last failure of the calling thread is returned by
 *    swe_last_error().  No C++ exception crosses this boundary.
 *  - Conditions found on the device are OR-ed into status[0] (a device
 *    uint32_t pair; status[1] counts depth clamps): SWE_STATUS_NEG_DEPTH (a
 *    negative depth was reset to 0), SWE_STATUS_NONFINITE (an updated value
 *    is NaN/Inf), SWE_STATUS_CFL_EXCEEDED (the Courant number of a step
 *    exceeded cfl_max and the step stands: the caller retakes it with the
 *    reduced dt that swe_cfl_reduce wrote, or accepts it),
 *    SWE_STATUS_RETAKEN (a step exceeded cfl_max and was marked for a retake
 *    on the device, see swe_cfl_reduce).  The caller reads status after
 *    synchronising.
 */
#ifndef SWE_H
#define SWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWE_OK 0
#define SWE_EINVAL (-1)
#define SWE_EHIP (-2)

#define SWE_STATUS_NEG_DEPTH 1u
#define SWE_STATUS_NONFINITE 2u
#define SWE_STATUS_CFL_EXCEEDED 4u
#define SWE_STATUS_RETAKEN 8u

enum swe_method { SWE_SPLIT = 0, SWE_UNSPLIT = 1 };
/* SWE_F32_STORE: the SWE_F32_DEV planes (eta', hu, hv, b in FP32) with every
 * operation of the step in FP64, the result rounded to FP32 once per step;
 * the single-patch split step only (it measures what FP32 storage alone
 * costs in accuracy; the other entry points take SWE_F64 or SWE_F32_DEV,
 * except those that only read or write the state, which treat it as
 * SWE_F32_DEV). */
enum swe_precision { SWE_F64 = 0, SWE_F32_DEV = 1, SWE_F32_STORE = 2 };
enum swe_bc { SWE_BC_WALL = 0, SWE_BC_EXTRAP = 1, SWE_BC_USER = 2 };

/* Physical and numerical parameters (host struct, passed by pointer). */
typedef struct swe_params {
    double g;            /* gravity, 9.81 m s^-2 */
    double drytol;       /* a cell with h <= drytol is dry (1e-3 m) */
    double h_corr;       /* an edge with a cell at or below this depth (a film on
                            the shore) gets no limited correction (0.1 m); the
                            split step also limits each correction to a share of
                            its donor cell's water, so that no correction drives
                            a depth below 0 */
    double manning_n;    /* Manning coefficient (Sec. 2 drag term); 0 = off */
    double cfl_desired;  /* Courant number aimed at by swe_cfl_reduce (0.9) */
    double cfl_max;      /* a step above this Courant number is flagged (1.0) */
    double sea_level;    /* reference level of eta' in SWE_F32_DEV (0 m) */
    double h_fp64;       /* SWE_F32_DEV: an edge with a cell at or below this
                            depth, or a dry cell, is solved in FP64 (1 m) */
    int32_t method;      /* swe_method */
    int32_t order;       /* 1 = fluctuations only, 2 = with limited corrections */
    int32_t transverse_order; /* SWE_UNSPLIT: 1 or 2 */
    int32_t precision;   /* swe_precision */
} swe_params;

/* One patch (host struct for swe_patch_step, device array for the batched
 * entry points).  See the layout rules above. */
typedef struct swe_patch {
    int64_t off;          /* element offset of cell (0, 0) in every plane */
    int64_t plane_stride; /* elements between the h, hu and hv planes */
    double dx, dy;        /* cell size [m] */
    int32_t mx, my;       /* interior cells, >= 1 each */
    int32_t pitch;        /* elements per row, >= mx + 4 */
    int32_t group;        /* index of the patch's dt slot */
    int32_t tref;         /* substeps of the patch per group step, >= 1 */
    int32_t level;        /* refinement level (1-based), informational */
    int8_t bc[4];         /* swe_bc of the sides xlo, xhi, ylo, yhi */
    int32_t reserved;
} swe_patch;

/* Launch shape of the single-patch step (host struct; results never depend
 * on it).  A zero field takes its default. */
typedef struct swe_launch {
    int32_t rows_per_task;   /* rows of a strip task, 1 .. 60 (default 48) */
    int32_t waves_per_block; /* waves per workgroup: 1, 2 or 4 (default 1) */
    int32_t xcd_run;         /* task ranks dealt to each of the eight XCDs in runs
                                of this many (default 8; 1 deals them in turn;
                                used with one wave per workgroup only) */
    int32_t reserved;        /* 0 */
} swe_launch;

/* Advance one patch by one step: q_out = step(q_in, dt[0]).
 * p, patch: host.  q_in, q_out: plane sets as above, must not overlap.
 * b: bathymetry plane.  dt: device double.  smax: device double[2]; the
 * largest wave speeds over the x- and y-edges of interior cells are
 * max-combined into smax[0], smax[1] (so it must hold 0 or an earlier value
 * on entry; swe_cfl_reduce resets it).  status: device uint32_t[2].
 * Only interior cells of q_out are written.
 * Launch shape: the defaults of swe_launch (strip tasks of 60 columns and 48
 * rows, one wave per workgroup, ranks dealt to the XCDs in runs of 8). */
int swe_patch_step(const swe_params *p, const swe_patch *patch, const void *q_in, void *q_out,
                   const void *b, const double *dt, double *smax, uint32_t *status,
                   void *stream);

/* Ghost cells (Sec. 3: a patch is its cells plus a frame of ghost cells that
 * the step reads; Sec. 4 names filling them as a separate task of small
 * parallelism; the physical boundary rules are this library's reading: the
 * paper states none).  Writes the ghost cells of n patches (device array
 * `patches`) into the planes `q` (all three) and, if fill_b != 0, into `b`,
 * by the rule above.  Sides with SWE_BC_USER are left untouched.
 * max_mx/max_my bound the patch sizes (host ints) and size the launch. */
int swe_ghost_fill(const swe_params *p, const swe_patch *patches, int32_t n, int32_t max_mx,
                   int32_t max_my, void *q, void *b, int32_t fill_b, void *stream);

/* Wave speeds for the first step size (Sec. 2, CFL condition: the step
 * follows from the largest wave speed s on the level; before the first step
 * no step has produced speeds, so they come from the Riemann problems of the
 * initial state).  Solves every edge of n patches without updating them and
 * max-combines the largest |s| over the x- and y-edges of each patch's
 * interior cells into smax_patch[2 k], smax_patch[2 k + 1]. */
int swe_speed_scan(const swe_params *p, const swe_patch *patches, int32_t n, int32_t max_mx,
                   int32_t max_my, const void *q, const void *b, double *smax_patch,
                   void *stream);

/* CFL rule (Sec. 2: the step size follows the largest wave speed so that
 * the Courant number stays at or below 1; a step above the limit is redone
 * with a smaller step).  For each group g, with rate_k = max(smax_x / dx,
 * smax_y / dy) / tref over the patches k of g (patches: device array):
 *   nu = dt_group[g] * max_k rate_k;
 *   nu > cfl_max sets SWE_STATUS_CFL_EXCEEDED in status[0] and
 *   group_flags[g] (if not NULL), or, when retake is not NULL,
 *   SWE_STATUS_RETAKEN instead;
 *   retake[g] (device uint32_t per group, may be NULL) = 1 if nu > cfl_max,
 *   else 0: the flags swe_patch_retake and swe_batched_retake act on;
 *   dt_group[g] = cfl_desired / max_k rate_k (unchanged if that rate is 0),
 *   which is the next step size, or the retake's if nu > cfl_max.
 * smax_patch entries are reset to 0 for the next step.  If
 * initial != 0 the CFL test is skipped (first dt from swe_speed_scan).
 * p: host.  Groups are 0 .. ngroups - 1. */
int swe_cfl_reduce(const swe_params *p, const swe_patch *patches, int32_t n, int32_t ngroups,
                   double *smax_patch, double *dt_group, uint32_t *status,
                   uint32_t *group_flags, uint32_t *retake, int32_t initial, void *stream);

/* Step sizes of the levels of a hierarchy (Sec. 3: a level refined by the
 * ratio r in space takes r steps of dt / r per step of the level below):
 * dt_levels[0] = dt_coarse[0], dt_levels[l] = dt_levels[l - 1] / ratio for
 * l = 1 .. nlevels - 1 (device doubles).  With the hierarchy's patches in one
 * group of swe_cfl_reduce, each with tref = ratio^(level - 1), that reduction
 * writes the coarse step of the CFL condition over all levels and this call
 * the levels' steps, without a host round trip. */
int swe_level_steps(const double *dt_coarse, int32_t ratio, int32_t nlevels, double *dt_levels,
                    void *stream);

/* Retake on the device (Sec. 2, a step above the Courant limit is redone):
 * the same step as swe_patch_step, enqueued unconditionally but carried out
 * only if retake[patch->group] != 0 as written by the swe_cfl_reduce that
 * followed the step; pass the q_in and q_out of the step being redone (q_in
 * is unchanged by a step) and dt_group, which holds the reduced step size.
 * A swe_cfl_reduce after it yields the next dt (with retake NULL it flags
 * SWE_STATUS_CFL_EXCEEDED if the retaken step is still above cfl_max).
 * Lets a device-resident loop or a captured graph follow the rule without
 * a host round trip.  retake: device array, NULL is an error. */
int swe_patch_retake(const swe_params *p, const swe_patch *patch, const void *q_in, void *q_out,
                     const void *b, const double *dt, double *smax, uint32_t *status,
                     const uint32_t *retake, void *stream);

/* swe_patch_step on a latitude-longitude patch (an extension: the paper's
 * transoceanic runs use such grids; the formulas here are derived from the
 * cell geometry).  Cells are Dlon x Dlat on a sphere of radius R; patch->dx
 * = R Dlon and patch->dy = R Dlat are their extents at the equator.  metric:
 * device double[2 my + 9]: kappa_j for the rows j = 0 .. my + 3 of the ghost
 * frame (cell area over its area at the equator, (sin phi_{j+1/2} - sin
 * phi_{j-1/2}) / Dlat), then len_e for e = 0 .. my + 4 (cos of the latitude of
 * the edge between rows e - 1 and e).  A cell changes by dt / (kappa dx) times
 * the x-amounts and dt / (kappa dy) times the y-amounts weighted by their
 * edges' len; an edge's correction uses its Courant factor times the mean
 * inverse capacity of its two cells, and the speeds max-combined into smax
 * are |s| times that mean (so swe_cfl_reduce keeps the Courant number); the
 * mass update omits the term (hv)_c (len_lower - len_upper) that the
 * edge-weighted fluctuations add; no curvature or Coriolis terms.  The
 * ghost rows' entries are the caller's: beyond a wall side (SWE_BC_WALL at
 * ylo or yhi) they should mirror the interior rows (kappa_1 = kappa_2,
 * kappa_0 = kappa_3, len_1 = len_3, len_0 = len_4, likewise at the top), as
 * the ghost state does, so that no mass crosses the wall.  sched: NULL for
 * tasks in index order, else a schedule buffer of sched_len entries as in
 * swe_patch_step_sched (launch order in, work per task out; swe_patch_order
 * sorts it); launch: host, NULL = defaults.  FP64 split step only; other
 * arguments as swe_patch_step. */
int swe_patch_step_sphere(const swe_params *p, const swe_patch *patch, const void *q_in,
                          void *q_out, const void *b, const double *dt, double *smax,
                          uint32_t *status, const double *metric, uint32_t *sched,
                          int64_t sched_len, const swe_launch *launch, void *stream);

/* The step and the CFL rule in one launch (Sec. 2: the step size follows the
 * largest wave speed, and a step above the Courant limit is redone with a
 * smaller one).  swe_patch_step_cfl is swe_patch_step_sched (sched NULL:
 * swe_patch_step; metric not NULL: swe_patch_step_sphere's step, FP64 split
 * only) followed, in the launch's last wave to finish, by what
 * swe_cfl_reduce(initial = 0, retake) does for the patch's group alone:
 * from smax[0], smax[1] and patch->dx, dy, tref the rate r; *dt * r >
 * cfl_max sets retake[patch->group] = 1 and SWE_STATUS_RETAKEN in status[0]
 * (else retake[group] = 0); r NaN sets SWE_STATUS_NONFINITE; *dt =
 * cfl_desired / r when r is positive and finite; smax[0..1] = 0.
 * swe_patch_retake_cfl is swe_patch_retake (metric as above) whose launch,
 * when the flag is set, ends with the CFL rule for the group on the redone
 * step: with last = 0 as the step's (a redone step still above cfl_max sets
 * the flag again, for another redo), with last != 0 as swe_cfl_reduce(retake
 * = NULL) (the next *dt, and SWE_STATUS_CFL_EXCEEDED if the step is still
 * above cfl_max; it stands); with the flag clear it does nothing.  The
 * CFL-ruled loop takes the step, a redo with last = 0 and one with last = 1:
 * three launches instead of six, up to two redos per step.  counter:
 * device uint32_t[3], zero before the first call; each launch that runs
 * leaves it zero (the finished waves, then the launch's own status bits and
 * depth resets, which join status only if its step stands: status counts
 * accepted steps, as the unfused sequence's does not).  dt, smax, status, retake: device, as swe_cfl_reduce; the step
 * reads *dt before any wave of the launch writes it.  Other arguments as the
 * calls named. */
int swe_patch_step_cfl(const swe_params *p, const swe_patch *patch, const void *q_in, void *q_out,
                       const void *b, double *dt, double *smax, uint32_t *status,
                       uint32_t *retake, uint32_t *counter, const double *metric,
                       uint32_t *sched, int64_t sched_len, const swe_launch *launch,
                       void *stream);
int swe_patch_retake_cfl(const swe_params *p, const swe_patch *patch, const void *q_in,
                         void *q_out, const void *b, double *dt, double *smax, uint32_t *status,
                         uint32_t *retake, uint32_t *counter, const double *metric, int32_t last,
                         void *stream);

/* swe_patch_retake on a latitude-longitude patch: the same gated redo of the
 * step (Sec. 2, a step above the Courant limit is redone with a smaller
 * step), launching swe_patch_step_sphere's step with `metric` (device, as
 * there) in index order.  The speeds that swe_patch_step_sphere max-combines
 * into smax are scaled by the edges' inverse capacities, so the
 * swe_cfl_reduce between the step and this call tests the Courant number on
 * the sphere.  Arguments otherwise as swe_patch_retake; FP64 split step
 * only. */
int swe_patch_retake_sphere(const swe_params *p, const swe_patch *patch, const void *q_in,
                            void *q_out, const void *b, const double *dt, double *smax,
                            uint32_t *status, const double *metric, const uint32_t *retake,
                            void *stream);

/* swe_speed_scan on one latitude-longitude patch (`patch`: device array of
 * one patch; metric: device, as for swe_patch_step_sphere): each edge's
 * largest |s| is scaled as swe_patch_step_sphere reports it, by 1 / kappa of
 * the row for an x-edge and by the mean of the two rows' 1 / kappa for a
 * y-edge, and the maxima over the interior cells' edges are max-combined into
 * smax[0] (x) and smax[1] (y).  With swe_cfl_reduce (initial = 1) this gives
 * the first step size on the sphere.  max_mx, max_my: the patch's mx, my (or
 * larger; they size the launch).  FP64 split step only. */
int swe_speed_scan_sphere(const swe_params *p, const swe_patch *patch, int32_t max_mx,
                          int32_t max_my, const void *q, const void *b, const double *metric,
                          double *smax, void *stream);

/* Water volume of one latitude-longitude patch (`patch`: device array of one
 * patch): sum over the interior of h kappa_j dx dy, kappa_j the capacity of
 * row j from `metric` (a cell's area is kappa_j dx dy), in FP64 with the
 * fixed reduction order of swe_mass, written to *mass (device).  FP64 only. */
int swe_mass_sphere(const swe_params *p, const swe_patch *patch, const void *q,
                    const double *metric, double *mass, void *stream);

/* Number of strip tasks (waves) of one step of `patch` (host) with the
 * launch shape `launch` (host, NULL = defaults), or SWE_EINVAL for a bad
 * patch or shape.  The schedule buffer of swe_patch_step_sched holds twice
 * this many uint32 entries. */
int32_t swe_patch_tasks(const swe_patch *patch, const swe_launch *launch);

/* Bytes of the caller-provided schedule buffer that swe_patch_step_sched,
 * swe_patch_order and swe_patch_step_sphere use for `patch` with `launch`
 * (both host; 8 bytes per task), or 0 for a bad patch or shape.  It is the
 * only device memory beyond the states that the single-patch entry points
 * take; the batched step's queue (two uint32) and the CFL slots are sized
 * in their own comments. */
size_t swe_workspace_bytes(const swe_patch *patch, const swe_launch *launch);

/* swe_patch_step with its tasks launched in a given order (scheduling only:
 * q_out, smax and status are bitwise those of swe_patch_step), meant for
 * heaviest first.  Tasks over water at rest or dry land skip their Riemann
 * solves (Sec. 2: such edges carry no waves) and end several times sooner
 * than tasks under a moving wave; launched in index order, a few long tasks
 * start late and the launch ends on them.
 * sched: device uint32_t[sched_len], sched_len >= 2 n with n =
 * swe_patch_tasks(patch, launch), that the caller allocates once per patch,
 * fills with zeros and passes to every step of that patch (with the same
 * launch); between calls the library owns its contents.  launch: host, NULL
 * = defaults; a shorter sched_len or a bad shape is SWE_EINVAL.  sched[0, n) is the
 * launch order: rank r runs task sched[r] - 1 (task r where sched[r] is 0, as
 * after the zero fill, or out of range).  Ranks are dealt to launch positions
 * so that each of the eight XCDs takes runs of consecutive ranks (neighbouring
 * strips share cache lines), which keeps the launch in rank order in blocks
 * of 8 runs; the mapping is a permutation.  Each task writes its work
 * (row sweeps that needed solves) into sched[n + task].  NULL sched is an
 * error. */
int swe_patch_step_sched(const swe_params *p, const swe_patch *patch, const void *q_in,
                         void *q_out, const void *b, const double *dt, double *smax,
                         uint32_t *status, uint32_t *sched, int64_t sched_len,
                         const swe_launch *launch, void *stream);

/* Launch order for the next swe_patch_step_sched of `patch` (host) from the
 * work its last one recorded: sched[0, n) = the tasks by work, largest
 * first, ties by task index (one small launch; work above 127 sorts as 127).
 * Enqueue it after the step on the same stream, every step or every few
 * steps.  sched_len and launch as for swe_patch_step_sched; NULL sched is an
 * error. */
int swe_patch_order(const swe_patch *patch, uint32_t *sched, int64_t sched_len,
                    const swe_launch *launch, void *stream);

/* Water volume (Sec. 2: the equations are conservation laws for the depth,
 * and Sec. 3 notes where AMR gives up exact conservation of mass; this is the
 * quantity such statements are about): sum(h) dx dy over the interior of each
 * patch, in FP64, written to mass_patch[k] (deterministic order).  In
 * SWE_F32_DEV, h is eta' + sea_level - b accumulated in FP64. */
int swe_mass(const swe_params *p, const swe_patch *patches, int32_t n, const void *q,
             const void *b, double *mass_patch, void *stream);

/* State in the precision's planes from FP64 data (the layout of Sec. 4's
 * structure-of-arrays pool; the surface-deviation form is this library's
 * FP32 storage, eta' = h + b - sea_level).  For the interior cells of n
 * patches (device table `patches`): element e = off + j * pitch + i of plane
 * k of q takes src[e - src_shift + k * S] (S = src_stride, or the patch's
 * plane_stride when src_stride is 0) and element e of b takes
 * src_b[e - src_shift]: with src_shift = 0 and src_stride = 0, src has q's
 * layout; a caller staging one patch alone passes src_shift = the patch's
 * off and src_stride = its staged plane length.  SWE_F64 copies them;
 * SWE_F32_DEV and SWE_F32_STORE store eta' = (h > 0 ? h + b : b) - sea_level,
 * formed in FP64 and rounded once, and hu, hv, b rounded to FP32.  Ghost
 * cells are not written (fill them with swe_ghost_fill).  max_mx/max_my
 * bound the patch sizes. */
int swe_state_import(const swe_params *p, const swe_patch *patches, int32_t n, int32_t max_mx,
                     int32_t max_my, const double *src, const double *src_b, int64_t src_shift,
                     int64_t src_stride, void *q, void *b, void *stream);

/* The inverse for reading results: interior (h, hu, hv) of n patches into
 * FP64 planes dst (element e of plane k at dst[e - dst_shift + k * S], S as
 * in swe_state_import); the FP32 planes give h = max(eta' + sea_level - b, 0)
 * in FP64. */
int swe_state_export(const swe_params *p, const swe_patch *patches, int32_t n, int32_t max_mx,
                     int32_t max_my, const void *q, const void *b, double *dst, int64_t dst_shift,
                     int64_t dst_stride, void *stream);

/* ------------------------------------------------------------------------
 * Batched step: many patches (e.g. the patches of an AMR hierarchy, or the
 * grids of several scenarios) in one call of at most two launches (Sec. 3:
 * patches of several levels, each level refining dx and dt by an integer
 * ratio; Sec. 4: memory pool and many small patches, whose launch overhead
 * the paper could not hide).
 *
 * A plan splits every patch into strip tasks (a strip of seg - 4 columns and
 * a run of rows, marched by a segment of seg lanes).  A patch with tref > 1
 * forms an item: persistent workgroups take items from a queue ordered
 * longest first, and an item's workgroup runs its tref substeps back to back
 * with a barrier in between.  The tasks of patches with tref == 1 ("plain"
 * tasks, the last nplain of the plan's tasks) run one wave each in a second
 * launch.  With per_substep = 1 every task is plain and a call makes one
 * launch per substep (patches are independent, so substep s of every patch
 * with tref > s can run together; the launch boundary orders a patch's
 * substeps).
 *
 * seg = 0 packs strips of any width side by side into the waves: every task
 * is plain (one launch per substep, as per_substep = 1), the rows of each
 * patch are cut into equal runs of at most rows_per_task (0: 48), and the
 * runs of patches of one tref, tallest first, are laid into 64 lanes left to
 * right, a run's columns cut wherever a wave fills up (a segment of c
 * columns takes c + 4 lanes, c >= 4 unless the patch is narrower).  A pack
 * (one wave) is returned as an item: its tasks [task_begin, task_end) lie
 * side by side from lane 0, `substeps` is the tref of its patches, patch is
 * -1; items are ordered by tref, largest first.
 */
typedef struct swe_schedule {
    int32_t seg;             /* lanes per strip: 64 or 32; 0 = packed strips */
    int32_t rows_per_task;   /* rows per task; 0 = 32 for tref == 1, else enough
                                tasks for the workgroup (at least 8 rows); with
                                seg = 0 the largest run of rows (0 = 48) */
    int32_t waves_per_group; /* waves per workgroup: 1, 2, 4 or 8 */
    int32_t per_substep;     /* 0: patches with substeps run as items of one
                                persistent launch; 1: every patch's tasks are
                                plain and substep s of all patches with tref > s
                                is one launch (max tref launches per call) */
    int32_t order;           /* 0 = longest item first, 1 = patch order */
    int32_t groups_per_cu;   /* persistent workgroups per compute unit; 0 = occupancy */
} swe_schedule;

typedef struct swe_task {
    int32_t patch;  /* index into the patch table */
    int32_t strip;  /* strip index within the patch's row run */
    int32_t row0;   /* first updated row (2 = first interior row) */
    int32_t rows;   /* updated rows */
    int32_t col0;   /* column of the segment's first lane (ghosts included):
                       strip * (seg - 4) for seg 64 or 32 */
    int32_t lanes;  /* lanes of the segment (seg, or 5 .. 64 with seg = 0);
                       it updates columns col0 + 2 .. col0 + lanes - 3 */
} swe_task;

typedef struct swe_item {
    int32_t task_begin, task_end; /* tasks [begin, end) of one patch */
    int32_t patch;
    int32_t substeps;             /* tref of the patch if the item covers it whole, else 1 */
} swe_item;

/* Build a plan on the host.  patches: host array of n patches.  With items
 * and tasks NULL only the counts are returned in *nitems, *ntasks (all
 * tasks), *nplain (the plain ones among them) and *nsub (the launches the
 * plain tasks take: 1, or the largest tref with per_substep = 1; 0 without
 * plain tasks); otherwise the arrays (host, sized from a previous query) are
 * filled: the items' tasks first, then the nplain plain tasks (ordered by
 * tref, largest first).  With seg = 0 the items are the packs and every
 * task is plain (nplain = ntasks, in pack order); swe_batched_step then
 * reads the packs from `items` and their tasks from `plain`.  Fails with
 * SWE_EINVAL for a bad patch or if a
 * SWE_BC_USER side has tref > 1 (its ghost cells are not refreshed between
 * substeps). */
int swe_batched_plan(const swe_patch *patches, int32_t n, const swe_schedule *sched,
                     swe_item *items, int32_t *nitems, swe_task *tasks, int32_t *ntasks,
                     int32_t *nplain, int32_t *nsub);

/* Advance every patch of the plan: patch k takes tref_k substeps of
 * dt_group[group_k] / tref_k from pool_in to pool_out (pool_in is not
 * modified; pool_work holds intermediate substeps of patches with tref > 1
 * and is required when the plan has items or nsub > 1, else it may be NULL).
 * pool_in, pool_out and pool_work hold pool_elems elements each and must not
 * overlap.  The largest
 * speeds of all substeps are max-combined into smax_patch[2 k], [2 k + 1].
 * patches, items, tasks: device copies of the table and of the plan; plain:
 * device pointer to the plan's nplain plain tasks (tasks + ntasks - nplain),
 * nsub: the plan's launch count for them.
 * group_status: NULL, or device uint32_t[2 x groups]: the status conditions
 * and depth resets of the patches of group g are also OR-ed into
 * group_status[2 g] and added to group_status[2 g + 1] (a caller serving
 * independent requests, one group each, learns which request they belong
 * to).
 * queue: device uint32_t[2], zero before the first call; the launch leaves it
 * zero again.  sched: host, the schedule the plan was built with. */
int swe_batched_step(const swe_params *p, const swe_patch *patches, const swe_item *items,
                     int32_t nitems, const swe_task *tasks, const swe_task *plain,
                     int32_t nplain, int32_t nsub, const void *pool_in, void *pool_out,
                     void *pool_work, int64_t pool_elems,
                     const void *pool_b, const double *dt_group, double *smax_patch,
                     uint32_t *status, uint32_t *group_status, uint32_t *queue,
                     const swe_schedule *sched, void *stream);

/* Retake on the device for the batched step: redoes, from pool_in to
 * pool_out, the items of the patches whose group g has retake[g] != 0 (as
 * written by swe_cfl_reduce after swe_batched_step); the items of every
 * other patch are skipped, so their results stand, and with no flagged group
 * the launch ends at once.  Arguments as for swe_batched_step, with the same
 * pools as the step being redone; retake: device uint32_t[ngroups]. */
int swe_batched_retake(const swe_params *p, const swe_patch *patches, const swe_item *items,
                       int32_t nitems, const swe_task *tasks, const swe_task *plain,
                       int32_t nplain, int32_t nsub, const void *pool_in, void *pool_out,
                       void *pool_work, int64_t pool_elems,
                       const void *pool_b, const double *dt_group, double *smax_patch,
                       uint32_t *status, uint32_t *group_status, uint32_t *queue,
                       const swe_schedule *sched, const uint32_t *retake, int32_t ngroups,
                       void *stream);

/* nsteps coarse steps of the batched step under the CFL rule, each as
 * swe_batched_step, then swe_cfl_reduce with the retake flags, the gated
 * swe_batched_retake of the flagged groups, swe_cfl_reduce with the retake
 * flags again, a second gated retake of the groups still above the limit
 * and swe_cfl_reduce of the redone steps (Sec. 2: the step size follows the
 * largest wave speed, and a step above the Courant limit is redone with a
 * smaller one; a second redo still above it stands and is flagged
 * SWE_STATUS_CFL_EXCEEDED), all enqueued on `stream` by one call.  The state alternates between pool_0 and pool_1
 * starting from pool_<first> (first = 0 or 1), so after the call it is in
 * pool_<(first + nsteps) % 2>.  npatches, ngroups: the table's patches and
 * the groups of dt_group, group_flags (may be NULL) and retake (device
 * uint32_t[ngroups], required).  pending: device uint32_t[2 ngroups], zero
 * before the first call and left zero: each step's conditions (status bits,
 * depth resets) wait there per group until the CFL rule settles them, so
 * that status and group_status (may be NULL) count accepted steps only (a
 * step the rule redoes reports nothing; its redo reports its own).  When a
 * step is one launch (nsub = 1 and either no items with seg 64 or 32, or
 * packs with seg 0) and ngroups <= 256, a non-NULL queue (device
 * uint32_t[2], zero before the first call and left zero) makes the CFL rule
 * run in the last workgroup of each launch instead of as launches of its
 * own: its two words count the finished workgroups and say whether a redo
 * is due, and a redo launch with nothing to redo ends at once.  The results
 * are bitwise the same either way.  Other arguments as swe_batched_step.
 * For a caller that advances many steps between host decisions (a serving
 * loop's round) this replaces four library calls per step. */
int swe_batched_advance(const swe_params *p, const swe_patch *patches, int32_t npatches,
                        int32_t ngroups, const swe_item *items, int32_t nitems,
                        const swe_task *tasks, const swe_task *plain, int32_t nplain,
                        int32_t nsub, void *pool_0, void *pool_1, int32_t first,
                        void *pool_work, int64_t pool_elems, const void *pool_b,
                        double *dt_group, double *smax_patch, uint32_t *status,
                        uint32_t *group_status, uint32_t *group_flags, uint32_t *retake,
                        uint32_t *pending, uint32_t *queue, const swe_schedule *sched,
                        int32_t nsteps, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * swe_batched_step without the queue and pool_work arguments.  The item
 * queue and the intermediate substep pool live in one static device array
 * of the library (256 bytes of queue, then SWE_STATIC_WORK_BYTES of substep
 * pool), which each device that the library runs on holds until the process
 * ends; the call allocates nothing.  A plan with items or nsub > 1 needs
 * pool_elems elements of the precision's type to fit in the substep pool,
 * else the call fails with SWE_EINVAL before enqueueing anything.  The
 * queue is zeroed by a small kernel at the start of every call with items.
 * Every call on one device shares that device's array and leaves its
 * intermediate substeps there: calls that overlap on one device (different
 * streams without ordering between them) race and give wrong results.
 * Results are bitwise those of swe_batched_step with the same plan. */
#define SWE_STATIC_WORK_BYTES (32u * 1024u * 1024u)
int swe_batched_step_static(const swe_params *p, const swe_patch *patches,
                            const swe_item *items, int32_t nitems, const swe_task *tasks,
                            const swe_task *plain, int32_t nplain, int32_t nsub,
                            const void *pool_in, void *pool_out, int64_t pool_elems,
                            const void *pool_b, const double *dt_group, double *smax_patch,
                            uint32_t *status, uint32_t *group_status,
                            const swe_schedule *sched, void *stream);

/* ------------------------------------------------------------------------
 * Coupling of AMR levels (Sec. 3: a finer level's ghost cells come from an
 * adjacent patch of the same level or, where none exists, from the level
 * below, interpolated in space and time; after the finer level's r substeps
 * the cells of the level below that it covers take averages of the fine
 * cells, the updating process; refluxing is left out, as in the paper's GPU
 * code).  Both keep a sea at rest at rest: they interpolate and average the
 * surface h + b and recover h from the bed of the cell written.  Sec. 3's
 * interpolation strategy: away from the shoreline plain linear interpolation
 * (here bilinear in space, linear in time); near it, where a cell of the
 * stencil is dry, the coarse cell under the fine cell alone.  FP64 planes,
 * or FP32 surface-deviation planes (eta' = h + b - sea_level; read into FP64,
 * combined there and rounded once; a dry cell stores eta' = b - sea_level).
 * Each level keeps its patches in one plane set (layout as above; all
 * patches of a level share its plane stride); a host plan lists every entry
 * once, so an entry's writes never collide with another's and its reads
 * touch only interior cells, which no entry writes.
 */
#define SWE_AMR_COPY 0   /* ghost cell over another patch of the same level */
#define SWE_AMR_COARSE 1 /* ghost cell filled from the cell of the level below */

typedef struct swe_amr_fill_op {
    int64_t dst;      /* element offset of the fine ghost cell in the fine planes */
    int64_t src;      /* SWE_AMR_COPY: element offset of the same-level interior
                         cell (fine planes); SWE_AMR_COARSE: element offset of the
                         coarse cell under the ghost cell (coarse planes) */
    int64_t st[4];    /* SWE_AMR_COARSE: element offsets (coarse planes) of the
                         bilinear stencil cells (i0, j0), (i0 + 1, j0), (i0, j0 + 1),
                         (i0 + 1, j0 + 1), where the fine cell's centre lies at
                         X = (I + 1/2) / r - 1/2, Y = (J + 1/2) / r - 1/2 in coarse
                         cell units (coarse centres at whole numbers) and
                         i0 = floor(X), j0 = floor(Y); -1 for a cell that lies in no
                         coarse patch's interior.  A cell of weight 0 (wx == 0 drops
                         the i0 + 1 column, wy == 0 the j0 + 1 row) is not read. */
    double wx, wy;    /* SWE_AMR_COARSE: X - i0 and Y - j0, in [0, 1) */
    int32_t kind;     /* SWE_AMR_COPY or SWE_AMR_COARSE */
    int32_t reserved;
} swe_amr_fill_op;

typedef struct swe_amr_avg_op {
    int64_t dst;      /* element offset of the coarse cell (coarse planes) */
    int64_t src;      /* element offset of the fine cell over its lowest row and
                         column (fine planes) */
    int32_t pitch;    /* fine patch pitch: elements between the fine rows */
    int32_t reserved;
} swe_amr_avg_op;

/* Fill the ghost cells of a finer level at time t_n + alpha dt_coarse,
 * 0 <= alpha <= 1 (alpha = k / r before substep k).  ops: device array of
 * nops entries.  q_fine, b_fine: the finer level's planes (written: the dst
 * cells of all three planes).  q_coarse_old, q_coarse_new: the coarser
 * level's planes before and after its step (read only), b_coarse its bed.
 * SWE_AMR_COPY: q_fine[dst] = q_fine[src] (three planes).  SWE_AMR_COARSE,
 * with b_f = b_fine[dst] and, for a coarse cell k, ho_k, hn_k its depths
 * before and after the step, b_k its bed, its values at alpha
 *   eta_k = (1 - alpha)(ho_k + b_k) + alpha (hn_k + b_k),
 *   m_k   = (1 - alpha) m_old,k + alpha m_new,k   (m = hu, hv):
 * linear, when every stencil cell of non-zero weight has st >= 0 and both of
 * its depths > drytol: per value v in (eta, hu, hv), with c0..c3 the stencil
 * cells in the order of st,
 *   line_0 = (1 - wx) v_c0 + wx v_c1,  line_1 = (1 - wx) v_c2 + wx v_c3,
 *   v = (1 - wy) line_0 + wy line_1   (a zero-weight term is left out);
 * constant, otherwise: the cell src alone, and (0, 0, 0) if both its depths
 * are <= drytol.  Then h = max(eta - b_f, 0), and hu = hv = 0 if h <= drytol.
 * Every product and sum rounds as written (no fused multiply-add). */
int swe_amr_fill(const swe_params *p, const swe_amr_fill_op *ops, int64_t nops, void *q_fine,
                 int64_t fine_plane_stride, const void *b_fine, const void *q_coarse_old,
                 const void *q_coarse_new, int64_t coarse_plane_stride, const void *b_coarse,
                 double alpha, void *stream);

/* Replace the coarse cells listed in ops by averages of the r x r fine cells
 * over each (ratio = r): with the wet fine cells (h > drytol) W,
 * W empty gives (0, 0, 0); else h = max(mean over W of (h + b_f) - b_c, 0),
 * (hu, hv) = mean over all r x r fine cells, or 0 if h <= drytol. */
int swe_amr_average(const swe_params *p, const swe_amr_avg_op *ops, int64_t nops, int32_t ratio,
                    const void *q_fine, int64_t fine_plane_stride, const void *b_fine,
                    void *q_coarse, int64_t coarse_plane_stride, const void *b_coarse,
                    void *stream);

/* Regridding (Sec. 3: cells are flagged where the sea surface departs from
 * rest, a buffer of cells around them too, the flags are clustered into
 * rectangles that balance their number against the unflagged cells they
 * cover, and the new patches take values from old patches of their level
 * where those overlap, else from the level below).
 *
 * swe_amr_flag: flags of the interior cells of n level-l patches (device
 * table `patches`, the level's planes q and bed b) into `flags`, a device
 * uint8 plane with the state planes' layout (element offsets as q): 1 where
 * a cell lies within `buffer` cells (max norm, same patch) of a wet cell
 * (h > drytol) with |h + b - sea_level| > tol, and not within `margin`
 * cells of the patch's edge; else 0.  max_mx, max_my bound the patch sizes. */
int swe_amr_flag(const swe_params *p, const swe_patch *patches, int32_t n, int32_t max_mx,
                 int32_t max_my, const void *q, const void *b, double tol, int32_t buffer,
                 int32_t margin, uint8_t *flags, void *stream);

/* swe_amr_cluster (HOST pointers, no device work): boxes covering the set
 * flags of an mx x my field (flags[j * pitch + i] != 0), written as (i0, j0,
 * i1, j1) inclusive to boxes[4 k ..], at most max_boxes; *nboxes = the count
 * (also when it exceeds max_boxes, which is an error).  Recursive, on a box
 * (first: the whole field): shrink it to the bounding box of its flags (none:
 * no box); accept it if flagged / area >= efficiency or if neither side is
 * at least 2 min_side long; else split it, in order of preference, at a zero
 * of a signature (flags per column or per row) nearest the box centre, in
 * the longer splittable dimension first (x on ties), then the smaller index;
 * else at the strongest sign change of the signature's second difference,
 * D(k) = sig(k - 1) - 2 sig(k) + sig(k + 1), with strength |D(s + 1) - D(s)|
 * (ties: dimension order, nearest the centre, smaller index); else at the
 * middle of the first splittable dimension.  A split at s keeps [lo, s] and
 * [s + 1, hi] and needs both at least min_side long.  Boxes come in the
 * order of the recursion (the lower part first). */
int swe_amr_cluster(const uint8_t *flags, int32_t mx, int32_t my, int32_t pitch,
                    double efficiency, int32_t min_side, int32_t *boxes, int32_t max_boxes,
                    int32_t *nboxes);

/* A patch of a level as swe_amr_init reads it: interior cells (i0 .. i0 +
 * mx - 1, j0 .. j0 + my - 1) in the level's global cell index, cell (I, J)
 * stored at element off + (J - j0 + 2) pitch + (I - i0 + 2) of each plane
 * (two ghost cells each side, as swe_patch). */
typedef struct swe_amr_rect {
    int64_t off;
    int32_t i0, j0;
    int32_t mx, my;   /* >= 1 each */
    int32_t pitch;    /* >= mx + 4 */
    int32_t reserved;
} swe_amr_rect;

/* swe_amr_init: the interior cells of n_new new patches of a level (device
 * table new_rects; planes q_new, bed b_new), built on the device from the
 * patch tables alone.  A cell (I, J) takes, per the first rule that applies:
 *   - the same cell of the first old patch of the level (device table
 *     old_rects, n_old >= 0 entries, planes q_old; NULL when n_old == 0)
 *     whose interior holds it: a copy of its three values;
 *   - the level below (device table coarse_rects, planes q_coarse, bed
 *     b_coarse, refinement ratio r): the rule of swe_amr_fill with alpha = 1
 *     and q_coarse as both states, the cell under it being the coarse cell
 *     (floor(I / r), floor(J / r)) and the stencil (i0, j0) .. (i0 + 1, j0 +
 *     1) with i0 = floor(X), j0 = floor(Y), X = (I + 1/2) / r - 1/2,
 *     Y = (J + 1/2) / r - 1/2, each looked up in the first coarse patch whose
 *     interior holds it (none: that stencil cell is missing);
 *   - else the cell is not written (a new patch must lie over the level
 *     below: regridding builds it from flags inside a coarse patch).
 * max_cells bounds mx my over the new patches.  q_new must differ from q_old
 * and q_coarse; the tables are read on the device during the call's work. */
int swe_amr_init(const swe_params *p, int32_t ratio, const swe_amr_rect *new_rects, int32_t n_new,
                 int64_t max_cells, void *q_new, int64_t new_plane_stride, const void *b_new,
                 const swe_amr_rect *old_rects, int32_t n_old, const void *q_old,
                 int64_t old_plane_stride, const swe_amr_rect *coarse_rects, int32_t n_coarse,
                 const void *q_coarse, int64_t coarse_plane_stride, const void *b_coarse,
                 void *stream);

/* swe_amr_plans: the plans swe_amr_fill and swe_amr_average take for the
 * n_fine patches of a level (device table `fine`) over the n_coarse patches
 * of the level below (`coarse`, ratio r), built on the device from the two
 * rectangle tables (Sec. 3: a finer level's ghost cells come from its own
 * level or from the level below; the updating process averages the fine
 * cells onto the coarse cells under them).  Fine patch k writes its ghost
 * cells, row by row of its frame (two rows, then the four ghost cells of
 * each interior row, then two rows), to fill_ops[fill_first[k] ..]: a cell
 * over another fine patch's interior (the first in order) as SWE_AMR_COPY
 * from that cell, else as SWE_AMR_COARSE from the coarse cell (floor(I / r),
 * floor(J / r)) with the bilinear stencil documented for swe_amr_fill_op,
 * each cell looked up in the first coarse patch that holds it; and its
 * coarse cells (floor(i0 / r) .. floor((i0 + mx) / r) - 1 by the same in j,
 * row by row) to avg_ops[avg_first[k] ..] (dst in the first coarse patch
 * that holds the cell, src = the fine cell (r Ic, r Jc), pitch = the fine
 * pitch).  fill_first, avg_first: device int64 arrays of the caller's
 * offsets (patch k has (mx + 4)(my + 4) - mx my ghost entries); max_entries
 * bounds a patch's ghost plus averaging entries.  err: device uint32, OR-ed
 * with 1 if a ghost cell lies over no cell of either level and 2 if a coarse
 * cell under a fine patch lies in no coarse patch (those entries then hold
 * offset 0: the caller must not use the plan). */
int swe_amr_plans(const swe_amr_rect *fine, int32_t n_fine, const swe_amr_rect *coarse,
                  int32_t n_coarse, int32_t ratio, int64_t max_entries, swe_amr_fill_op *fill_ops,
                  const int64_t *fill_first, swe_amr_avg_op *avg_ops, const int64_t *avg_first,
                  uint32_t *err, void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *swe_last_error(void);

/* Library version string. */
const char *swe_version(void);

#ifdef __cplusplus
}
#endif
#endif
