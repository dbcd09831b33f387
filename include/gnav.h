/*
 * gnav.h -- C ABI of the MI355X gamma-navigation library (libgnav.so).
 *
 * The library answers the two navigation questions stated in Sec. 3.2 of
 * Seiskari, Kommeri, Niemi, "GPU in Physics Computation: Case Geant4
 * Navigation" (which volumes hold a point; where a ray next crosses a volume
 * boundary), and runs the photon free-path sampling of Sec. 3.1 (Alg. 1,
 * Eqs. 1-8) repeated after every interaction as a gamma transport loop.  Its
 * call sequence follows the benchmark phases of Sec. 3.4 (Alg. 2): upload the
 * geometry once (phase 1), hand over primaries that already live in device
 * memory (phases 2-4), transport them (phase 5, the timed part), read the
 * results back (phase 6).
 *
 * Conventions
 *   Units: mm, MeV, rad; densities in g/cm3.
 *   "dev" pointers are HIP device pointers (e.g. a torch tensor's data_ptr on
 *   ROCm); "host" pointers are ordinary host memory.  The caller owns every
 *   pointer it passes; the library owns geometry tables, cross-section
 *   tables, voxel tables and tally buffers.
 *   Compute calls take a HIP stream as `void*` (NULL = the null stream), are
 *   ordered on it, enqueue and return; device inputs must stay alive until the
 *   stream has passed the call.
 *   Errors are returned as a negative gnav_status; gnav_last_error() gives a
 *   message.  Outputs are unspecified after an error.  After GNAV_EHIP the
 *   context should be destroyed.  No exception or abort crosses the ABI.
 *   One context per host thread; calls on one context are not thread safe.
 *   Transport launches of one context share its work-queue counter and
 *   pending-photon buffer: a launch (or graph replay) on another stream than
 *   the context's previous launch first waits, on the device, for that
 *   launch, so launches of one context never overlap.
 */
#ifndef GNAV_H
#define GNAV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gnav_status;
#define GNAV_OK 0
#define GNAV_EINVAL (-1)       /* bad argument (null pointer, size, id) */
#define GNAV_ENOMEM (-2)       /* device or host allocation failed */
#define GNAV_EHIP (-3)         /* a HIP runtime call failed */
#define GNAV_EGEOM (-4)        /* invalid geometry description */
#define GNAV_ESTATE (-5)       /* call out of order (e.g. no geometry yet) */
#define GNAV_EUNSUPPORTED (-6) /* valid request the library does not implement */

/* Solid families (Sec. 3.5 names boxes, tubes, cones and balls, and its CMS
 * case other Geant4 solids such as trapezoids).
 * Parameters, 8 doubles per solid:
 *   GNAV_BOX  hx, hy, hz                               (half lengths)
 *   GNAV_TUBS rmin, rmax, dz, sphi, dphi               (tube section, half length dz)
 *   GNAV_CONS rmin1, rmax1, rmin2, rmax2, dz, sphi, dphi (cone section; 1 at -dz, 2 at +dz)
 *   GNAV_ORB  r                                        (full ball)
 *   GNAV_TRD  dx1, dx2, dy1, dy2, dz                   (trapezoid: x half width dx1 at
 *                                                       z = -dz, dx2 at +dz, linear between;
 *                                                       likewise y; all positive)
 *   GNAV_SPHERE rmin, rmax, sphi, dphi, stheta, dtheta (sphere section: shell, phi wedge,
 *                                                       polar angles stheta .. stheta + dtheta
 *                                                       from +z, within [0, pi])
 * Sections need 0 <= rmin < rmax at both ends and dphi in (0, pi] or 2 pi. */
#define GNAV_BOX 0
#define GNAV_TUBS 1
#define GNAV_CONS 2
#define GNAV_ORB 3
#define GNAV_TRD 4
#define GNAV_SPHERE 5
#define GNAV_NFAMILIES 6 /* family slots of the work counters */

/* Surface tolerance (mm): points within half of it of a surface lie on it. */
#define GNAV_TOLERANCE 1e-9

/* Largest max_steps_per_track of a batch (the per-track step count is kept
 * in 23 bits). */
#define GNAV_MAX_STEPS_PER_TRACK 8388607

/* Counter slots returned by gnav_read_tallies. */
#define GNAV_C_STEPS 0          /* navigation steps (one per transport-loop iteration) */
#define GNAV_C_PE 1             /* photoelectric absorptions */
#define GNAV_C_COMPTON 2        /* Compton scatters */
#define GNAV_C_PAIR 3           /* pair conversions */
#define GNAV_C_CROSSINGS 4      /* geometry-limited steps */
#define GNAV_C_ESCAPED 5        /* tracks that left the world */
#define GNAV_C_CUTOFF 6         /* tracks ended below the energy cut */
#define GNAV_C_PUSHES 7         /* zero-step pushes */
#define GNAV_C_STUCK 8          /* tracks killed after repeated zero steps */
#define GNAV_C_TRUNCATED 9      /* tracks stopped at max_steps_per_track */
#define GNAV_C_TRACKS 10        /* tracks started (primaries + annihilation photons) */
#define GNAV_C_SHORTCUTS 11     /* physics steps taken inside the safety (no ComputeStep) */
#define GNAV_C_DIST_IN 12       /* daughter entry distances evaluated in FP64 (count_work = 1) */
#define GNAV_C_DIST_OUT 13      /* mother exit-distance evaluations (count_work = 1) */
#define GNAV_C_INSIDE 14        /* point-in-solid tests, locate / relocate (count_work = 1) */
#define GNAV_C_VOXEL_NODES 15   /* voxel nodes visited by the step walk (count_work = 1) */
#define GNAV_C_INVALID 16       /* primaries skipped: bad event/geometry id, non-finite state, E <= 0 */
#define GNAV_C_DIST_IN_F32 17   /* daughter entry distances evaluated in FP32 (FP32 precisions) */
#define GNAV_C_SCORED 18        /* learned order: steps whose start-node candidates the network ordered */
/* Work by solid family (batches with count_work = 1; zero otherwise): slot
 * base + family (GNAV_BOX .. GNAV_TRD; GNAV_NFAMILIES slots each). */
#define GNAV_C_DIST_IN_BY 19    /* daughter entry distances (FP64 and FP32) by the daughter's family */
#define GNAV_C_DIST_OUT_BY 25   /* mother exit distances by the mother's family */
#define GNAV_C_SAFETY_BY 31     /* isotropic distances (mother and daughter safeties) by family */
#define GNAV_C_INSIDE_BY 37     /* point-in-solid tests by family */
#define GNAV_C_FRAME_MAPS 43    /* frame maps: one per daughter candidate examined, one per placement
                                   level of each touchable frame formed (level by level, Sec. 3.2) */
#define GNAV_NCOUNTERS 44

/* Limiter codes of a step. */
#define GNAV_LIM_MOTHER (-1)    /* left the current volume (>= 0: entered that daughter slot) */
#define GNAV_LIM_PE (-2)
#define GNAV_LIM_COMPTON (-3)
#define GNAV_LIM_PAIR (-4)
#define GNAV_LIM_MAX_STEP (-5)  /* ComputeStep queries: the caller's maximum step was shorter */

/* Track fates in the per-track log. */
#define GNAV_FATE_ABSORBED 1
#define GNAV_FATE_ESCAPED 2
#define GNAV_FATE_CUTOFF 3
#define GNAV_FATE_STUCK 4
#define GNAV_FATE_TRUNCATED 5
#define GNAV_FATE_PAIR 6

typedef struct gnav_ctx gnav_ctx;
typedef struct gnav_tally gnav_tally;

/* One step of a track in the optional parity log (32 bytes). */
typedef struct {
  int32_t touchable; /* touchable id (per geometry) where the step started */
  int32_t code;      /* limiter code (see GNAV_LIM_*) */
  double step;       /* step length, mm */
  double edep;       /* energy deposited at the end of the step, MeV */
  double energy;     /* photon energy after the step, MeV (0 when absorbed) */
} gnav_logrec;

/* Summary of one track for comparisons at full size (32 bytes): what the
 * per-track log would hold, folded.  hash is 64-bit FNV-1a (offset basis
 * 14695981039346656037, prime 1099511628211) over the bytes of every step
 * record's touchable and code, each as a little-endian int32, in record
 * order; the sums add the records' step lengths and deposits in record
 * order. */
typedef struct {
  uint64_t hash;
  int32_t n;        /* step records */
  int32_t fate;     /* GNAV_FATE_* (0: slot unused) */
  double sum_step;  /* mm */
  double sum_edep;  /* MeV, logged deposits (an energy cut's or a kill's deposit is not logged) */
} gnav_digest;

/* Flat description of a placement hierarchy (Sec. 3.2: volumes nested in a
 * hierarchy).  All arrays are host memory owned by the caller and copied
 * before gnav_upload_geometry returns. */
typedef struct {
  int32_t n_solids;
  const int32_t* solid_type; /* [n_solids] GNAV_BOX..GNAV_ORB */
  const double* solid_par;   /* [n_solids][8] see above */
  int32_t n_mats;
  const double* mat_density; /* [n_mats] g/cm3, 0 = vacuum */
  const int32_t* mat_el_off; /* [n_mats + 1] element ranges into el_* */
  const int32_t* el_Z;       /* [mat_el_off[n_mats]] atomic number */
  const double* el_A;        /* atomic mass, g/mol */
  const double* el_wfrac;    /* mass fraction */
  int32_t n_lv;
  const int32_t* lv_solid;   /* [n_lv] solid index */
  const int32_t* lv_mat;     /* [n_lv] material index */
  const int32_t* lv_dau_off; /* [n_lv] first placement of the LV's daughters */
  const int32_t* lv_dau_cnt; /* [n_lv] number of daughters (slots 0..cnt-1) */
  const uint8_t* lv_voxelize;/* [n_lv] 1: build a voxel grid for this LV (NULL: all) */
  int32_t n_pv;
  const int32_t* pv_lv;      /* [n_pv] placed (child) LV */
  const double* pv_rot;      /* [n_pv][9] row-major R, x_mother = R x_local + t */
  const double* pv_trans;    /* [n_pv][3] t */
  int32_t world_lv;          /* the unplaced top volume (its frame is the global frame) */
  int32_t voxel_lists;        /* 0: a voxel node lists the daughters whose solid may meet it
                                 (shape-aware, with a finer-grid search for nested shells);
                                 1: the daughters whose bounding box meets it, on the
                                 bounding-box grid search only (as Geant4's smart voxels) */
} gnav_geometry_desc;

/* Create a context on HIP device `device`. */
gnav_status gnav_create(int32_t device, gnav_ctx** out);

/* Destroy a context and every library-owned buffer (tallies included). */
void gnav_destroy(gnav_ctx* ctx);

/* Message of the last error on ctx (valid until the next call on ctx). */
const char* gnav_last_error(const gnav_ctx* ctx);

/* Validate a geometry, expand its touchables (distinct placement paths,
 * numbered breadth first from the world = 0, children of touchable T at
 * child_base[T] + slot), build voxel grids and attenuation tables, and copy
 * everything to the device (Alg. 2, phase 1: load the geometry and transfer
 * it to the GPU once).  Several geometries may be resident; each gets an id.
 * The copies are ordered on `stream` and the call returns once they are
 * complete.  Every resident table is reallocated, so graphs captured before
 * the call become stale (gnav_graph_launch then returns GNAV_ESTATE).
 * GNAV_EGEOM on bad parameters, indices or a touchable count above 2^30. */
gnav_status gnav_upload_geometry(gnav_ctx* ctx, const gnav_geometry_desc* desc, int32_t* geom_id,
                                 int32_t* n_touchables, void* stream);

/* Host copies of the touchable table of one geometry; each output may be
 * NULL, otherwise it has n_touchables entries. */
gnav_status gnav_touchables(gnav_ctx* ctx, int32_t geom_id, int32_t* parent, int32_t* pv,
                            int32_t* lv, int32_t* depth);

/* Distance arithmetic of the navigation queries and of transport (Sec. 5
 * names FP64 throughput as a limit of the GPU port).  In both FP32 forms
 * positions, optical depths, point-in-volume decisions, the voxel walk and
 * tallies stay FP64 and the daughter candidates' solid arithmetic runs in
 * FP32 on coordinates local to each candidate.
 *   GNAV_PREC_FP64: every distance in FP64.
 *   GNAV_PREC_FP32_SCREENED: FP32 entry distances rank the candidates; the
 *     first is evaluated in FP64, the others in FP64 unless a rigorous FP32
 *     lower bound shows they cannot reach the best distance.  Steps,
 *     limiters and therefore whole transports equal the FP64 results.
 *   GNAV_PREC_FP32: the step is the FP32 distance (mother and daughters);
 *     results deviate from FP64 by FP32 rounding. */
#define GNAV_PREC_FP64 0
#define GNAV_PREC_FP32_SCREENED 1
#define GNAV_PREC_FP32 2

/* LocateGlobalPoint (Sec. 3.2, first question: which volumes hold a point):
 * the deepest touchable holding each point.  pos_dev [n][3]; dir_dev [n][3]
 * or NULL.  On a surface a point belongs to a volume only when its direction
 * points strictly inward through every face it lies on (without a
 * direction, surface points count as in).  touchable_dev [n] receives the
 * per-geometry touchable id, -1 outside.  `precision` is one of GNAV_PREC_*;
 * point-in-volume decisions are FP64 in every form, so all three give the
 * same answer. */
gnav_status gnav_locate(gnav_ctx* ctx, int32_t geom_id, int64_t n, const double* pos_dev,
                        const double* dir_dev, int32_t* touchable_dev, int32_t precision,
                        void* stream);

/* ComputeStep (Sec. 3.2, second question: where a ray next crosses a volume
 * boundary): the distance along dir to the next boundary from each point of
 * its touchable, the smaller of the mother's exit distance and the
 * daughters' entry distances, the mother winning ties, then the lowest
 * daughter slot.
 *   touchable_dev [n] or NULL (locate first, with the direction);
 *   max_step_dev [n] or NULL (no limit): when max_step <= the geometric
 *     step, the step is max_step, the limiter GNAV_LIM_MAX_STEP and the next
 *     touchable the current one (ties go to the caller's limit, as an
 *     interaction wins a tie with the boundary in transport);
 *   step_dev [n] (mm, +inf when no boundary lies ahead), limiter_dev [n]
 *     (GNAV_LIM_MOTHER, a daughter slot >= 0, or GNAV_LIM_MAX_STEP);
 *   next_touchable_dev [n] or NULL: the touchable after relocation at the
 *     end point (-1 = left the world);
 *   precision: GNAV_PREC_*;
 *   learned: order in which the start voxel node's candidates are examined,
 *     0 slot order, 1 smallest lower bound first, 2 the network set with
 *     gnav_set_mlp (GNAV_ESTATE without one); every order gives the same
 *     results (see gnav_batch.order); 1 and 2 need GNAV_PREC_FP64. */
gnav_status gnav_compute_step(gnav_ctx* ctx, int32_t geom_id, int64_t n, const double* pos_dev,
                              const double* dir_dev, const int32_t* touchable_dev,
                              const double* max_step_dev, double* step_dev, int32_t* limiter_dev,
                              int32_t* next_touchable_dev, int32_t precision, int32_t learned,
                              void* stream);

/* Validity codes of the surface normal (gnav_step_outputs.normal_valid_dev). */
#define GNAV_NORMAL_NONE 0  /* no boundary reached: infinite or max-step limited step */
#define GNAV_NORMAL_FACE 1  /* the end point lies on exactly one face of the crossed solid */
#define GNAV_NORMAL_EDGE 2  /* it lies on two or more faces (edge or corner): the normal is that
                               of the face with the largest signed value, lowest face on ties */

/* Outputs of gnav_compute_step_ex: device arrays of n entries. */
typedef struct {
  double* step_dev;            /* [n] required */
  int32_t* limiter_dev;        /* [n] required */
  int32_t* next_touchable_dev; /* [n] or NULL */
  double* safety_dev;          /* [n] or NULL: voxel-limited safety at the start point (a lower
                                  bound on the distance to any boundary in the FP64 and screened
                                  forms, the FP32 value in the GNAV_PREC_FP32 form) */
  double* normal_dev;          /* [n][3] or NULL: exit normal of the boundary crossed at the end
                                  point, global frame, unit length: the outward normal of the
                                  mother when the mother limits the step, the inward normal of
                                  the entered daughter otherwise, so it points along the
                                  direction of travel (the entering normal is its negation);
                                  (0, 0, 0) with GNAV_NORMAL_NONE */
  int32_t* normal_valid_dev;   /* [n] or NULL: GNAV_NORMAL_* */
} gnav_step_outputs;

/* ComputeStep with the outputs above.  The normal answers the second half
 * of the navigation question of Sec. 3.2 (the normal of the boundary surface
 * at the crossing point), which the navigator state of Sec. 3.2 also keeps
 * for the last crossed boundaries.  Arguments as gnav_compute_step. */
gnav_status gnav_compute_step_ex(gnav_ctx* ctx, int32_t geom_id, int64_t n, const double* pos_dev,
                                 const double* dir_dev, const int32_t* touchable_dev,
                                 const double* max_step_dev, int32_t precision, int32_t learned,
                                 const gnav_step_outputs* out, void* stream);

/* ComputeSafety: a lower bound >= 0 on the isotropic distance from each point
 * to any boundary of its touchable (mother or daughter), limited to the
 * point's voxel node.  touchable_dev NULL: locate first.  precision
 * GNAV_PREC_*: FP64 and screened give lower bounds (screened from rigorously
 * lowered FP32 safeties in nodes of six or more candidates); GNAV_PREC_FP32
 * gives the FP32 value. */
gnav_status gnav_compute_safety(gnav_ctx* ctx, int32_t geom_id, int64_t n, const double* pos_dev,
                                const int32_t* touchable_dev, double* safety_dev, int32_t precision,
                                void* stream);

/* Free path of Alg. 1 alone, the paper's timed phase (Alg. 2 phase 5, the
 * measurements of Table 1): for each particle i, starting at pos_dev[i] along
 * dir_dev[i] with lifetime life_dev[i] (an optical depth, Y in Alg. 1), cross
 * boundaries accumulating S_j = sum mu s (Eq. 6) and return the first
 * interaction distance T = t_{j-1} + (Y - S_{j-1}) / mu_j (Eq. 7) in
 * t_dev[i] (mm; +inf when the particle leaves the world) and the boundaries
 * crossed in n_bounds_dev[i] (may be NULL).  mu_mass > 0 selects the paper's
 * attenuation mu = rho mu_mass (Eq. 9, mu_mass in cm2/g, e.g. 0.06146 for
 * aluminium at 1 MeV); mu_mass = 0 uses the tabulated total attenuation at
 * `energy` (MeV).  Device arrays of n entries (pos/dir [n][3]). */
gnav_status gnav_free_path(gnav_ctx* ctx, int32_t geom_id, int64_t n, const double* pos_dev,
                           const double* dir_dev, const double* life_dev, double energy, double mu_mass,
                           double* t_dev, int32_t* n_bounds_dev, void* stream);

/* Device energy tallies, sized to every touchable resident at creation and to
 * n_events events.  Created zeroed.  gnav_tally_reset zeroes them again on
 * `stream` (one kernel launch, no memset node, so a graph may capture it). */
gnav_status gnav_tally_create(gnav_ctx* ctx, int32_t n_events, gnav_tally** out);
gnav_status gnav_tally_reset(gnav_ctx* ctx, gnav_tally* tally, void* stream);
gnav_status gnav_tally_free(gnav_ctx* ctx, gnav_tally* tally);

/* One recorded crossing: a ComputeStep limited by a daughter whose start
 * voxel node holds 2 or more candidates, the daughter being candidate number
 * `label` (< 64) of that node.  x = point in the mother frame divided by the
 * mother's voxel-grid half size (relative to the grid centre), v = direction
 * in the mother frame, cls = the mother's ordering class (32 bytes). */
typedef struct gnav_crossing {
  int32_t cls;
  float x[3];
  float v[3];
  int32_t label;
} gnav_crossing;

/* One batch of primaries; every *_dev array is device memory of n_primaries
 * entries (pos_dev and dir_dev [n][3]) owned by the caller. */
typedef struct {
  int64_t n_primaries;
  const int32_t* event_dev;   /* event id of each primary, 0 <= id < n_events of the tally */
  const int32_t* prim_id_dev; /* id of the primary inside its event (track key = id << 2) */
  const double* pos_dev;
  const double* dir_dev;      /* unit vectors */
  const double* energy_dev;   /* MeV */
  const int32_t* event_geom_dev; /* [n_events] geometry id of each event; NULL: geom_id for all */
  int32_t geom_id;
  uint64_t seed;              /* Philox key of the transport stream */
  double e_cut;               /* MeV: photons below it deposit locally and stop */
  int64_t max_steps_per_track;/* <= 0: 1e6; at most GNAV_MAX_STEPS_PER_TRACK (GNAV_EINVAL above) */
  int32_t precision;          /* GNAV_PREC_*; FP32 forms need order 0 and no recorder */
  int32_t block;              /* track-pool slots (= threads) per block: 64, 128 or 256; 0 = 64 */
  int32_t grid;               /* blocks, 0 = library default (fills the device) */
  int32_t count_work;         /* 1: also count navigation work (GNAV_C_DIST_IN..VOXEL_NODES) */
  int32_t order;              /* start-node candidate order: 0 slot order, 1 smallest lower bound
                                 first, 2 learned (network set with gnav_set_mlp); same results.
                                 Orders 1 and 2 apply in mothers whose voxel nodes hold three or
                                 more candidates on average; elsewhere the walk is in slot order */
  struct gnav_crossing* record_dev; /* optional recorder of daughter-limited steps (training data) */
  int64_t record_capacity;
  uint64_t* record_count_dev; /* crossings seen (may exceed the capacity; extra ones dropped) */
  gnav_logrec* log_dev;       /* optional per-track log: 3 slots per primary (primary and */
  int64_t log_capacity;       /*   its two annihilation photons), log_capacity records each */
  int32_t* log_n_dev;         /*   [3 n] records written per slot (may exceed the capacity), */
  int32_t* log_fate_dev;      /*   [3 n] GNAV_FATE_* per slot (0 = slot unused); both required
                                   with log_dev */
  int32_t chunk;              /* primaries a block claims from the device queue at once; 0: each
                                 wave claims exactly what its idle lanes need (one atomic) */
  int32_t sort_period;        /* every sort_period-th round the step phase groups tracks by their
                                 current logical volume instead of solid family; 0: never */
  int32_t tuned;              /* 1: take block, grid, chunk and sort_period from gnav_autotune's cache
                                 for this geometry, precision and order when present */
  gnav_digest* digest_dev;    /* optional [3 n] per-track digests (slots as for the log); the
                                 caller zeroes them; log_dev may then be NULL */
  int32_t keep_order;         /* 0: blocks take the primaries in decreasing energy (half-octave
                                 classes, sorted on the device before the transport, in a buffer
                                 of the context), so that the tracks still running when the
                                 batch runs dry are short ones; with per-event geometries sorted
                                 by geometry first (a block's tracks stay in one geometry), for
                                 up to 16 resident geometries; 1: in the order given (always so
                                 in gnav_transport_batch_noalloc, and with more than 16
                                 geometries).  Results do not depend on it */
} gnav_batch;

/* Transport a batch (Alg. 1 repeated after each interaction; Alg. 2 phase
 * 5): photoelectric absorption, Klein-Nishina Compton scattering and pair
 * conversion, with deposits accumulated into `tally`.  Random numbers come
 * from Philox4x32-10 keyed by (event, track key, draw), so results do not
 * depend on launch shape or scheduling. */
gnav_status gnav_transport_batch(gnav_ctx* ctx, const gnav_batch* batch, gnav_tally* tally,
                                 void* stream);

/* gnav_transport_batch for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results; it calls no allocator (no
 * hipMalloc or hipFree, no allocating library routine).  The transport's
 * scratch -- the work-queue counter and one pending annihilation photon (48
 * bytes) per track-pool slot -- lives in a fixed array of the library on each
 * device, 256 + 48 * GNAV_NOALLOC_MAX_SLOTS bytes (9 MiB), held until the
 * process ends, instead of the context's buffers.  grid * block (the default
 * grid when grid is 0: 3 * 256 slots per compute unit) above
 * GNAV_NOALLOC_MAX_SLOTS returns GNAV_EINVAL.  Each call resets the counter
 * with a kernel and writes a pending entry before reading it, so nothing
 * carries over from the last call; but every call on one device shares the
 * array, so calls that can run at the same time on one GPU (on other streams,
 * contexts or host threads) race on it and give wrong results. */
#define GNAV_NOALLOC_MAX_SLOTS 196608
gnav_status gnav_transport_batch_noalloc(gnav_ctx* ctx, const gnav_batch* batch, gnav_tally* tally,
                                         void* stream);

/* Launch settings of gnav_transport_batch chosen by gnav_autotune. */
typedef struct {
  int32_t block;              /* track-pool slots (threads) per block */
  int32_t grid;
  int32_t chunk;
  int32_t sort_period;
  float ms;                   /* median kernel time of the setting, milliseconds */
} gnav_tuning;

/* Autotuner (the scheduling knobs of Sec. 5: how tracks are grouped and
 * refilled).  Times the transport of `batch` (trials runs per setting after
 * one warm-up, median, hipEvents on `stream`) over a coordinate search of
 * block (64, 128, 256 pool slots, each with its default grid: 1.5 times the
 * resident blocks), grid (a half, one, two and three times the resident
 * blocks), chunk (0, 256, 1024,
 * 4096) and sort_period (0, 1, 4, 16), keeps the fastest in the context for
 * this geometry, precision, order and batch size (power-of-two class), and
 * returns it in `out` (may be NULL).  Batches with tuned = 1 then use it.
 * `tally` is scratch (left zeroed); batch must not carry a log or recorder.
 * Synchronous; trials in 1..100. */
gnav_status gnav_autotune(gnav_ctx* ctx, const gnav_batch* batch, gnav_tally* tally, int32_t trials,
                          void* stream, gnav_tuning* out);

/* Copy tallies to host memory (Alg. 2, phase 6) after the stream passes the
 * earlier calls; synchronises `stream`.  Outputs may be NULL:
 * edep_touchable [total resident touchables, geometries in id order],
 * edep_event and escaped_event [n_events], counters [GNAV_NCOUNTERS]. */
gnav_status gnav_read_tallies(gnav_ctx* ctx, const gnav_tally* tally, double* edep_touchable,
                              double* edep_event, double* escaped_event, uint64_t* counters,
                              void* stream);

/* Repeated batches as one HIP graph: {zero the tally, reset the work queue,
 * transport} captured once for a batch description (same device buffers,
 * same tally) and replayed with gnav_graph_launch.  The graph holds only
 * kernel nodes (no memset nodes).  The batch's buffers and the tally must
 * outlive the graph; the call synchronises `stream` while capturing.
 * The graph also holds the library's geometry tables, its pending-photon
 * buffer and (order 2) the network's weights: gnav_graph_launch returns
 * GNAV_ESTATE, without touching the device, once any of them has been
 * reallocated or unbound since the capture (a later gnav_upload_geometry, a
 * batch needing a larger grid than any before, gnav_set_mlp or
 * gnav_mlp_free of the bound network); capture the graph again then. */
typedef struct gnav_graph gnav_graph;
gnav_status gnav_graph_create(gnav_ctx* ctx, const gnav_batch* batch, gnav_tally* tally, void* stream,
                              gnav_graph** out);
gnav_status gnav_graph_launch(gnav_ctx* ctx, gnav_graph* graph, void* stream);
gnav_status gnav_graph_free(gnav_ctx* ctx, gnav_graph* graph);

/* Candidate-ordering MLP (learned part).  Inputs per sample: 6 floats (point
 * in the mother frame divided by the mother's voxel-grid half size, then the
 * direction) and a mother class id in [0, n_class); two hidden layers of 128
 * ReLU units; 64 logits, one per candidate position of the start voxel node.
 * Parameters are float32 in the order w1x [128][6], w1m [n_class][128],
 * b1 [128], w2 [128][128], b2 [128], w3 [64][128], b3 [64]; matrix products
 * run on bf16 MFMA with float32 accumulation.  Batches are multiples of 16
 * up to max_batch.  x_dev [B][6] float, cls_dev / label_dev [B] int32. */
typedef struct gnav_mlp gnav_mlp;
gnav_status gnav_mlp_create(gnav_ctx* ctx, int32_t n_class, int32_t max_batch, const float* params_host,
                            gnav_mlp** out);
int64_t gnav_mlp_n_params(const gnav_mlp* mlp);
/* Softmax cross-entropy gradient of the mean loss over the batch; optional
 * copies of the gradient (float [n_params]) and of the loss (one float). */
gnav_status gnav_mlp_grad(gnav_ctx* ctx, gnav_mlp* mlp, int64_t batch, const float* x_dev,
                          const int32_t* cls_dev, const int32_t* label_dev, float* grad_dev,
                          float* loss_dev, void* stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with the last gradient. */
gnav_status gnav_mlp_adam(gnav_ctx* ctx, gnav_mlp* mlp, float lr, void* stream);
/* Logits [B][64] (float). */
gnav_status gnav_mlp_forward(gnav_ctx* ctx, gnav_mlp* mlp, int64_t batch, const float* x_dev,
                             const int32_t* cls_dev, float* logits_dev, void* stream);
/* The ordering network as the transport and gnav_compute_step evaluate it
 * (order 2): features x_dev [n][6] float rounded to bf16, classes cls_dev [n]
 * (clamped to [0, n_class)), the layers on bf16 MFMA tiles of 16 rows with
 * FP32 accumulation and bf16 hidden activations; logits_dev [n][64] float
 * (or NULL) and pred_dev [n], the position of the highest logit, the lowest
 * on ties (or NULL).  Any n >= 0. */
gnav_status gnav_mlp_score(gnav_ctx* ctx, gnav_mlp* mlp, int64_t n, const float* x_dev,
                           const int32_t* cls_dev, float* logits_dev, int32_t* pred_dev, void* stream);
/* Host copy of the float parameters (synchronous). */
gnav_status gnav_mlp_get_params(gnav_ctx* ctx, gnav_mlp* mlp, float* params_host);
/* Free a network (after the device has passed its last use); every binding
 * of it made with gnav_set_mlp is dropped. */
gnav_status gnav_mlp_free(gnav_ctx* ctx, gnav_mlp* mlp);

/* Number of ordering classes (voxelised mothers) of a geometry. */
gnav_status gnav_ordering_classes(gnav_ctx* ctx, int32_t geom_id, int32_t* n_class);
/* Use `mlp` (NULL to clear) for order 2 on geometry geom_id; the network must
 * have been created on the same context and its class count must equal the
 * geometry's.  Batches and graphs read its weights when they run. */
gnav_status gnav_set_mlp(gnav_ctx* ctx, int32_t geom_id, gnav_mlp* mlp);

/* Total touchables over all resident geometries, and the offset of one
 * geometry's touchables in that concatenation. */
gnav_status gnav_touchable_offset(gnav_ctx* ctx, int32_t geom_id, int32_t* offset,
                                  int32_t* total);

#ifdef __cplusplus
}
#endif

#endif /* GNAV_H */
