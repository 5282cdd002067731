/*
 * rt.h -- C ABI of the MI355X formal-solution library.
 *
 * The library computes the formal solution of the radiative transfer
 * equation (Osborne 2025, Eqs. Rte/RteRay/RteIntegral) along long
 * characteristics through a sparse brick grid of emissivity eta and opacity
 * chi, with variance-limited mipmapping (VLM, Sect. 2.2), hierarchical DDA
 * traversal (HDDA, Sect. 2.3 and Alg. 1) and, for moving media, velocity
 * interpolation (Sect. 3.1) or "Core and Voigt" (Sect. 3.2).  Each segment
 * applies the piecewise-constant update I <- I exp(-tau) + S (1 - exp(-tau)),
 * tau = chi dt ds0, S = eta / chi (accumulated front-to-back on the device,
 * which equals the recurrence up to rounding).
 *
 * Conventions (all calls):
 *   - Index space: a MIP-0 voxel has side 1; physical length = index length
 *     x ds0.  Voxel (i,j,k) covers [i,i+1)x[j,j+1)x[k,k+1); voxel linear
 *     index = i + nx*(j + ny*k).  2D scenes use n[2] = 1.
 *   - A ray is x(t) = p - t w, t in [0, t_exit], from the probe p (a voxel
 *     centre) upwind to the bounding box, where the boundary intensity I0
 *     enters (Sect. 2.3, Eq. Ray: rays are clipped to the bounding box).  The
 *     result is the intensity arriving at p travelling along w.
 *   - Blocks ("bricks", Sect. 2.3) are B^D voxels, B a power of two; block
 *     linear index = bx + nbx*(by + nby*bz).  Active blocks are stored in
 *     Morton order (Sect. 2.3.1).
 *   - "Probes" of the all-probes mode are the voxel centres of the active
 *     blocks, numbered slot*B^D + local, local = x + B*(y + B*z) inside the
 *     block, slot = rank of the block in Morton order among active blocks.
 *   - Pointers named d_* are device pointers (HIP device memory) owned by
 *     the caller; pointers named h_* are host pointers.  `stream` is a
 *     hipStream_t passed as void*.  Every device-side call is asynchronous on
 *     that stream unless documented as synchronising; a synchronising call
 *     waits for that stream only.
 *   - Ownership: the caller allocates all device memory -- inputs, outputs
 *     and every workspace (scene, batch, cache), each sized by a host-only
 *     *_workspace_bytes query and at least 256-byte aligned.  The library
 *     sub-allocates inside a workspace and never calls hipMalloc on these
 *     paths; a handle owns only host memory, and the workspace must outlive
 *     it and any work still in flight on the stream.  Only the debugging
 *     helpers rt_scene_cell_values and rt_debug_visited allocate (and free)
 *     small temporary device buffers.
 *   - Errors: every call returns rt_status; no C++ exception crosses the
 *     ABI; rt_last_error() gives a thread-local message for the last failure.
 *     Arguments are validated on the host before any device work.  Device
 *     anomalies (traversal step cap exceeded) never abort a kernel: they are
 *     counted and read with rt_scene_device_error().
 */
#ifndef RT_H
#define RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rt_status {
    RT_OK = 0,
    RT_E_ARG = 1,         /* invalid argument (shape, enum, null pointer, size) */
    RT_E_UNSUPPORTED = 2, /* valid but not supported by the library */
    RT_E_STATE = 3,       /* call order (e.g. trace before build) */
    RT_E_HIP = 4,         /* a HIP runtime call failed */
    RT_E_DEVICE = 5       /* a device-side anomaly was recorded */
} rt_status;

enum { RT_MAX_LINES = 4 };    /* lines evaluated per cell (Sect. 4.1.2: compile-time 4) */
enum { RT_LAM_BATCH = 8 };    /* wavelengths per build/trace batch (Sect. 3.2.1, 4.1: 8) */
enum { RT_MAX_LEVELS = 5 };   /* MIP levels 0..4 (B = 16 in 2D) */

typedef enum rt_model {
    RT_MODEL_STATIC = 0, /* eta, chi given per wavelength per voxel */
    RT_MODEL_LINES = 1   /* line parameters + grey background + bulk velocity per voxel */
} rt_model;

typedef enum rt_profile {
    RT_PROFILE_GAUSS = 0, /* peak-normalised Gaussian exp(-x^2), no wavelength scaling */
    RT_PROFILE_VOIGT = 1  /* H(a,x)/(sqrt(pi) dlD) with Sect. 3.2.1 wavelength scalings */
} rt_profile;

/* PREFILTER (Sect. 5.1, prefiltering: the transfer equation precomputed along
 * the +-x, y, z axes and interpolated between them) is static emission whose
 * merged cells (levels >= 1) also store, per signed axis, the homogeneous cell
 * with the same transfer as the cell's MIP-0 voxels: the exact row transfer
 * (I, T) along that axis averaged over the cell's rows, tau_eff = -ln(Tbar),
 * chi_eff = tau_eff / side, eta_eff = Ibar tau_eff / ((1 - Tbar) side)
 * (Ibar / side when Tbar = 1), computed in FP64 from the MIP-0 values.  A ray
 * of direction w blends the axes it propagates along with weights w_a^2 / sum;
 * level 0 uses the stored MIP-0 values.  2 dim times the stored-value storage
 * of the merged levels. */
typedef enum rt_emission {
    RT_EMIS_STATIC = 0,    /* stored eta, chi per wavelength (lines model: evaluated at rest, u = 0) */
    RT_EMIS_VELINTERP = 1, /* velocity-grid interpolation (Sect. 3.1), lines model only */
    RT_EMIS_CAV = 2,       /* Core and Voigt (Sect. 3.2): profile evaluated on the fly, lines model only */
    RT_EMIS_PREFILTER = 3  /* static emission with prefiltered merged cells (Sect. 5.1); both models */
} rt_emission;

/* Stored level values.  LINEAR is the box filter of Sect. 2.1 and the one the
 * thin bypass of Sect. 2.2 assumes (the emergent intensity of a thin cell is
 * linear in eta); LOG keeps the geometric mean, which underestimates the
 * emission of cells mixing dense and near-empty voxels. */
typedef enum rt_avg {
    RT_AVG_LOG = 0,   /* level value = exp(mean of ln(q ds0)) / ds0 (geometric mean) */
    RT_AVG_LINEAR = 1 /* level value = arithmetic mean of the children (box filter) */
} rt_avg;

typedef enum rt_dtype { RT_F32 = 0, RT_BF16 = 1, RT_F16 = 2 } rt_dtype;

/* Node grids of velocity interpolation.  Every level cell carries n_v nodes
 * uniform over a range of projected velocities u = v . w (Sect. 3.1: from the
 * MIP-0 voxels the cell contains).
 *   FULL:    one grid over [-V, V], V = max |v|, for every direction.
 *   ORTHANT: one grid per orthant of directions (2^dim classes; class bit a
 *            set when w_a < 0), over the projections reachable from that
 *            orthant: the paper's deployment solves the angles quadrant by
 *            quadrant with a grid per quadrant (Sect. 4.1), so that n_v nodes
 *            per quadrant give up to 4 n_v effective bins.  2^dim times the
 *            node storage; a trace reads only its directions' grids. */
typedef enum rt_vgrid { RT_VGRID_FULL = 0, RT_VGRID_ORTHANT = 1 } rt_vgrid;

typedef enum rt_trace_mode {
    RT_TRACE_LEVEL0 = 0, /* every active block at MIP 0 (SPARSE; DENSE if the scene is dense) */
    RT_TRACE_VLM = 1     /* each block at its VLM level of the current batch */
} rt_trace_mode;

/*
 * Scene description (host struct, copied by rt_scene_create).
 *   dim        2 or 3.
 *   n          voxels per axis, each a positive multiple of brick; n[2] = 1 in 2D.
 *   brick      block side B: 8 or 16.
 *   n_levels   MIP levels 0..n_levels-1, 1 <= n_levels <= log2(B) + 1 (<= RT_MAX_LEVELS).
 *   model      rt_model.
 *   emission   rt_emission the scene is built for (STATIC for the static model).
 *   profile    rt_profile (lines model).
 *   n_lines    1..RT_MAX_LINES (lines model).
 *   n_v        velocity nodes per cell and direction class, >= 2 (velocity
 *              interpolation).
 *   dense      nonzero: every block is active (the dense comparator); 0: blocks
 *              whose inputs are all zero (or masked out) are empty.
 *   n_lam      number of wavelengths of the scene.
 *   ds0        physical side of a MIP-0 voxel (> 0).
 *   vgrid      rt_vgrid: velocity-interpolation node grids (Sect. 3.1, 4.1).
 *   h_lam      host [n_lam] wavelengths in nm (lines model; may be NULL for static).
 *   h_lam0     host [n_lines] rest wavelengths in nm (lines model).
 */
typedef struct rt_scene_desc {
    int32_t dim;
    int32_t n[3];
    int32_t brick;
    int32_t n_levels;
    int32_t model;
    int32_t emission;
    int32_t profile;
    int32_t n_lines;
    int32_t n_v;
    int32_t dense;
    int32_t n_lam;
    int32_t vgrid;
    double ds0;
    const double* h_lam;
    const double* h_lam0;
} rt_scene_desc;

/*
 * Device inputs (caller-owned, float32, x fastest).  They must stay valid and
 * unchanged for the lifetime of the scene: every rt_scene_build reads them.
 *   static model:  d_eta, d_chi  [n_lam][nvox].
 *   lines model:   d_eta_star, d_chi_star, d_damp, d_inv_dld  [n_lines][nvox]
 *                  (eta*, chi* at lam0; Voigt damping at lam0; 1/Doppler width
 *                  in 1/nm); d_eta_bg, d_chi_bg [nvox] (grey background);
 *                  d_vel [dim][nvox] bulk velocity in km/s.
 *   d_block_mask   optional uint8 [nblocks]; nonzero = active.  NULL: a block
 *                  is active when any of its inputs is nonzero.
 */
typedef struct rt_scene_inputs {
    const float* d_eta;
    const float* d_chi;
    const float* d_eta_star;
    const float* d_chi_star;
    const float* d_damp;
    const float* d_inv_dld;
    const float* d_eta_bg;
    const float* d_chi_bg;
    const float* d_vel;
    const uint8_t* d_block_mask;
} rt_scene_inputs;

/*
 * Build parameters of one wavelength batch (Sect. 2.2, 4.1).
 *   iod_threshold  T: a level-m cell passes if IoD[ln(eta ds0)] <= T and
 *                  IoD[ln(chi ds0)] <= T, IoD = |Var/Mean| over its 2^D children.
 *   tau_thin       a cell also passes if chi_a 2^m ds0 < tau_thin, chi_a being the
 *                  arithmetic (box-filter, Sect. 2.1) mean of the MIP-0 chi it covers.
 *   max_level      cap on the selected level (-1: none).
 *   avg_mode       rt_avg for the stored level values (the IoD always uses ln values).
 *   storage        rt_dtype of the stored values (BF16/F16 round to nearest even):
 *                  static emission values, Core-and-Voigt line parameters,
 *                  velocity-interpolation node values (computed in FP32, then rounded;
 *                  a BF16/F16 node record is 32 bytes instead of 64, in the same
 *                  buffer).  Level selection does not depend on it.
 *   iod_frame      line model with velocity interpolation: the frame in which the
 *                  MIP-0 eta, chi of the level test are evaluated.  RT_IOD_REST (0):
 *                  every line at rest (Sect. 3.1); RT_IOD_CORE (1): each voxel's line
 *                  at the projected velocity within [-|v|, |v|] closest to putting the
 *                  batch wavelength in its core (the Core-and-Voigt frame of Sect. 3.2,
 *                  which sees velocity gradients in line cores).  Core and Voigt always
 *                  uses RT_IOD_CORE; static emission ignores it.
 */
typedef enum rt_iod_frame { RT_IOD_REST = 0, RT_IOD_CORE = 1 } rt_iod_frame;

typedef struct rt_build_params {
    double iod_threshold;
    double tau_thin;
    int32_t max_level;
    int32_t avg_mode;
    int32_t storage;
    int32_t iod_frame;
} rt_build_params;

/*
 * Trace parameters.
 *   mode       rt_trace_mode.
 *   max_level  cap on the level sampled by the trace (-1: none).
 *   I0         boundary intensity entering at the upwind end of every ray.
 *   step_cap   maximum traversal steps per ray (0: sum of the grid sides x 2 + 16).
 *              A ray that reaches it stops and is recorded as a device error.
 *   d_stats    optional device uint64 [5], accumulated (not cleared):
 *              [0] segments applied (non-empty cells), [1] rays,
 *              [2] empty-block steps, [3] level changes, [4] the sum over
 *              wavefronts of their longest ray in steps ([0] + [2]), so that
 *              ([0] + [2]) / (64 [4]) is the SIMD lane utilisation.
 *   level_dist distance-graded level cap (VLM mode): level m >= 1 is used only
 *              in blocks the ray enters at path length t >= level_dist[m]
 *              (index units; the probe's own block is entered at t = 0).
 *              All zeros: no grading.  The paper's cascade caps [0,0,1,2,3,4]
 *              over radiance intervals ending at 1.5 x 4^i voxels (Sect. 4.1)
 *              correspond to level_dist = {0, 6, 24, 96, 384}.  Values are
 *              compared exactly (use small dyadic numbers).
 *   grade_mode rt_grade_mode: where the level_dist cap is taken.
 *              RT_GRADE_BLOCK_ENTRY: at the path length at which the ray
 *              enters each block, for the whole block (level changes stay on
 *              block faces).  RT_GRADE_PATH: at every point of the ray, so the
 *              cap rises exactly at t = level_dist[m], inside a cell if need
 *              be (the cell is split there and the ray re-located at the new
 *              level, with the same exact predicates as an interval start);
 *              this is the cascade intervals' caps of Sect. 4.1 along one
 *              ray, equal to the composition of rt_trace_interval calls over
 *              [level_dist[m], level_dist[m+1]] with max_level = m.
 */
typedef enum rt_grade_mode { RT_GRADE_BLOCK_ENTRY = 0, RT_GRADE_PATH = 1 } rt_grade_mode;

typedef struct rt_trace_params {
    int32_t mode;
    int32_t max_level;
    float I0;
    int32_t step_cap;
    unsigned long long* d_stats;
    float level_dist[RT_MAX_LEVELS];
    int32_t grade_mode;
} rt_trace_params;

typedef struct rt_scene_info {
    int64_t n_blocks;        /* total blocks */
    int64_t n_active;        /* active blocks */
    int64_t n_probes;        /* n_active * B^D */
    int64_t cells_per_brick; /* sum over levels of (B/2^m)^D */
    int64_t storage_bytes;   /* device bytes held by the scene */
    int32_t batch_begin;     /* wavelength batch currently built, -1 if none */
    int32_t batch_end;
    int32_t n_state_words;   /* ceil(n_blocks / 21) */
    int32_t reserved_;
} rt_scene_info;

typedef struct rt_device_err {
    unsigned long long step_cap_hits; /* rays stopped at the step cap */
    long long first_ray;              /* smallest ray id that hit it, -1 if none */
    unsigned long long bad_probes;    /* caller probe indices outside [0, nvox): not traced, outputs NaN */
} rt_device_err;

typedef struct rt_scene rt_scene;

/*
 * rt_scene_workspace_bytes -- size of the device workspace a scene with
 * n_active active blocks needs (the scene's whole device storage: block
 * tables, level structure, and the stored values of one wavelength batch).
 * n_active = the block count gives the upper bound for any inputs;
 * n_active = 0 gives at least what rt_scene_count_active needs.  After
 * creation rt_scene_info.storage_bytes is the same figure.  Host only: no
 * device work, inputs not needed.  Errors: RT_E_ARG, RT_E_UNSUPPORTED as for
 * rt_scene_create.
 */
rt_status rt_scene_workspace_bytes(const rt_scene_desc* desc, int64_t n_active, size_t* h_bytes);

/*
 * rt_scene_count_active -- the first phase of a two-phase creation: checks
 * every input value, classifies the blocks (a block is active when any of its
 * inputs is nonzero, or as d_block_mask says; Sect. 2.3.1) and returns the
 * number of active blocks, so that the caller can size the workspace of
 * rt_scene_create exactly.  d_ws: device workspace of at least
 * rt_scene_workspace_bytes(desc, 0) bytes, used as scratch only (its contents
 * are not needed afterwards).  Synchronises `stream`.  Errors as
 * rt_scene_create.
 */
rt_status rt_scene_count_active(const rt_scene_desc* desc, const rt_scene_inputs* inputs, void* d_ws, size_t ws_bytes,
                                void* stream, int64_t* h_n_active);

/*
 * rt_scene_create -- classify blocks, order the active ones in Morton order,
 * assign storage slots (Sect. 2.3.1 offset table) and lay the scene's device
 * storage out in the caller's workspace d_ws (ws_bytes at least
 * rt_scene_workspace_bytes(desc, n_active) for the inputs' active-block
 * count, from rt_scene_count_active, or the upper bound).  For the lines
 * model it also builds the wavelength-independent level chains (velocity grid
 * parameters, Core-and-Voigt line parameters).  Synchronises `stream` (the
 * active-block count decides the layout).  Every input value is checked on
 * the device first: eta, chi, line strengths, damping, Doppler widths and
 * background must be finite and >= 0, velocities finite.  The workspace must
 * stay allocated and untouched by the caller until rt_scene_destroy.
 * Errors: RT_E_ARG (shape/enum/pointer, negative / non-finite input values
 * counted in the message, a null, misaligned or too small workspace, with the
 * size needed in the message), RT_E_UNSUPPORTED, RT_E_HIP.
 */
rt_status rt_scene_create(const rt_scene_desc* desc, const rt_scene_inputs* inputs, void* d_ws, size_t ws_bytes,
                          void* stream, rt_scene** out);

/*
 * rt_scene_build -- for wavelengths [lam_begin, lam_end) (at most
 * RT_LAM_BATCH): MIP-0 values of the batch, the mip chain of every active
 * block (Sect. 2.1), the VLM level of every block (min over the batch of the
 * per-wavelength levels, Sect. 2.2 / 4.1) and the packed 3-bit block states,
 * 21 per 64-bit word (Sect. 2.3.1).  Asynchronous.  Errors: RT_E_ARG.
 */
rt_status rt_scene_build(rt_scene* scene, const rt_build_params* params, int32_t lam_begin, int32_t lam_end,
                         void* stream);

/*
 * rt_trace -- long-characteristic formal solution for every (direction,
 * probe) pair over the current batch (Sect. 2.3, Alg. 1 traversal; Eq.
 * RteIntegral per segment).
 *   d_dirs     device float [n_dir][dim], unit vectors (|w| - 1 within 1e-5).
 *   d_probes   device int32 [n_probes] voxel linear indices, or NULL for all
 *              probes (then n_probes must equal rt_scene_info.n_probes).  An
 *              index outside [0, nvox) is not traced: its outputs are NaN and
 *              rt_scene_device_error counts it (bad_probes); the same holds for
 *              every entry point that takes a probe list.
 *   d_I        device float [n_dir][lam_end - lam_begin][n_probes]: intensity
 *              arriving at each probe along each direction.
 * n_probes = 0 traces nothing (d_probes and d_I may then be NULL).
 * Asynchronous.  Errors: RT_E_ARG, RT_E_STATE (no batch built).
 */
rt_status rt_trace(const rt_scene* scene, const rt_trace_params* params, const float* d_dirs, int32_t n_dir,
                   const int32_t* d_probes, int64_t n_probes, float* d_I, void* stream);

/*
 * rt_trace_interval -- rt_trace over the path interval t in [t1, t2] of every
 * ray x(t) = p - t w (a radiance interval: Eq. Ray and the HDDA procedure of
 * Alg. 1 traverse [t1, t2]; Sect. 4.1 gives each cascade its own interval and
 * maximum MIP level, params->max_level).  The interval starts in the cell
 * holding x(t1) (on a cell face, the cell the ray moves into) at its block's
 * level, and its last segment ends at t2; a face crossed exactly at t2 belongs
 * to this interval.  With a distance-graded cap (params->level_dist) a block's
 * cap is still set by the path length at which the ray entered it, so
 * consecutive intervals visit the cells of the whole ray.
 *   t1, t2     0 <= t1 <= t2; t2 may be +infinity (to the grid boundary).
 *   d_I        device float [n_dir][nl][n_probes]: the interval's emission seen
 *              at p, starting from 0 at the interval's far end, or from
 *              params->I0 when the ray leaves the grid within the interval.
 *   d_T        device float [n_dir][nl][n_probes] transmittance of the
 *              interval (1 when it holds no non-empty cell), or NULL.
 * Intervals [0, t1], [t1, t2], ... compose as I = I_a + T_a I_b, T = T_a T_b.
 * Other arguments as for rt_trace.  Asynchronous.
 * Errors: RT_E_ARG (also t1 negative or not finite, t2 < t1), RT_E_STATE.
 */
rt_status rt_trace_interval(const rt_scene* scene, const rt_trace_params* params, const float* d_dirs,
                            int32_t n_dir, const int32_t* d_probes, int64_t n_probes, double t1, double t2,
                            float* d_I, float* d_T, void* stream);

/* Scene facts (host only, no device work). */
rt_status rt_scene_get_info(const rt_scene* scene, rt_scene_info* h_info);

/* Active blocks in Morton (storage) order: host int32 [n_active].  Ordered on `stream`, synchronises it. */
rt_status rt_scene_active_blocks(const rt_scene* scene, int32_t* h_blocks, void* stream);

/* VLM level of every block for the current batch, -1 = empty: host int8 [n_blocks].  Ordered on `stream`,
 * synchronises it. */
rt_status rt_scene_levels(const rt_scene* scene, int8_t* h_levels, void* stream);

/* Packed block states (state = level + 1, 0 = empty; 3 bits, 21 per word): host uint64 [n_state_words].
 * Ordered on `stream`, synchronises it. */
rt_status rt_scene_states(const rt_scene* scene, uint64_t* h_words, void* stream);

/*
 * Stored values of given cells for the current batch (parity checks).
 *   h_cells  host int32 [n][4]: x, y, z (any voxel inside the cell) and level.
 *   h_out    host float [n][RT_LAM_BATCH][2]: eta, chi per batch wavelength,
 *            decoded to float32; static emission only.
 * Ordered on `stream`, synchronises it; allocates temporary device buffers (a debugging helper).
 * Errors: RT_E_ARG (cell in an empty block, level out of range).
 */
rt_status rt_scene_cell_values(const rt_scene* scene, int32_t n, const int32_t* h_cells, float* h_out,
                               void* stream);

/*
 * Adapted-grid cells visited by one ray, using the trace kernel's own
 * traversal code on one device lane (parity of the traversal).
 *   probe_vox  voxel linear index of the probe;  h_dir host float [dim].
 *   h_cells    host int32 [cap][4]: cell origin x, y, z (multiples of 2^level) and level.
 *   h_t        host double [cap][2]: t at entry and exit of the cell.
 *   h_count    number of cells written (<= cap; RT_E_ARG if cap is too small).
 * Synchronising.
 */
rt_status rt_debug_visited(const rt_scene* scene, const rt_trace_params* params, int32_t probe_vox,
                           const float* h_dir, int32_t cap, int32_t* h_cells, double* h_t, int32_t* h_count,
                           void* stream);

/*
 * ---------------------------------------------------------------- batching
 * Many scenes of uneven size traced in one persistent launch with a
 * work-stealing queue (the batched form of the formal solution; each job is
 * exactly rt_trace over all probes of its scene's current batch).
 *
 * A job traces one scene (static emission) for n_dir directions over all of
 * its probes.  d_I is device float [n_dir][nl][n_probes] (nl = wavelengths of
 * the scene's current batch, n_probes = rt_scene_info.n_probes); params as
 * for rt_trace (d_stats is ignored).
 */
typedef struct rt_batch_job {
    const rt_scene* scene;
    const float* d_dirs;
    int32_t n_dir;
    int32_t reserved_;
    float* d_I;
    rt_trace_params params;
} rt_batch_job;

/*
 * Launch shape of the persistent kernel (0 selects the default):
 *   wg_waves       waves per workgroup: 1, 2, 4 (default) or 8;
 *   wgs_per_cu     resident workgroups per compute unit (default 2);
 *   tiles_per_pop  64-probe tiles claimed per atomic pop (default 1);
 *   order          0 (default): costliest job first (cost ~ n_dir x n_probes x
 *                  sum of grid sides); 1: the given job order.  Either way 2D jobs
 *                  come before 3D jobs: each dimension present gets one persistent
 *                  launch of its own (compiled for that dimension and, when all its
 *                  jobs share it, that storage dtype), both launches on `stream`;
 *   d_claims       optional device uint32 [total tiles], incremented once per
 *                  processed tile (lets tests check that every tile is taken
 *                  exactly once);
 *   tile_shape     which voxels of a brick one 64-probe wave tile takes:
 *                  RT_TILE_ROWS (0, default): 64 consecutive voxels in x-fastest
 *                  order (a 16 x 4 strip of a 16^2 brick, an 8 x 8 x 1 slab of an
 *                  8^3 brick); RT_TILE_CUBES (1): 8 x 8 squares in 2D, 4 x 4 x 4
 *                  cubes in 3D (bricks smaller than that tile: the whole brick).
 *                  Outputs keep the probe order of rt_trace, so every tile
 *                  shape gives the same bits.
 */
enum { RT_TILE_ROWS = 0, RT_TILE_CUBES = 1 };
typedef struct rt_batch_params {
    int32_t wg_waves;
    int32_t wgs_per_cu;
    int32_t tiles_per_pop;
    int32_t order;
    unsigned int* d_claims;
    int32_t tile_shape;
    int32_t reserved_;
} rt_batch_params;

typedef struct rt_batch rt_batch;

/* Device workspace of a batch of n_jobs jobs (job table, queue counters,
 * error counters).  Host only. */
rt_status rt_batch_workspace_bytes(int32_t n_jobs, size_t* h_bytes);

/* Validates the jobs, uploads the job table into the caller's workspace d_ws
 * (at least rt_batch_workspace_bytes(n_jobs); synchronises `stream`) and sizes
 * the queue.  The scenes must have a built batch; their storage is read at
 * every rt_batch_run, so rebuilding a scene for another batch of the same
 * size and storage dtype is picked up by the next run.  The workspace must
 * outlive the batch handle.  Errors: RT_E_ARG (also a null, misaligned or too
 * small workspace), RT_E_STATE, RT_E_UNSUPPORTED (non-static emission),
 * RT_E_HIP. */
rt_status rt_batch_create(const rt_batch_job* jobs, int32_t n_jobs, const rt_batch_params* params, void* d_ws,
                          size_t ws_bytes, void* stream, rt_batch** out);

/* Runs the batch: a queue-reset kernel and the persistent kernel.  Kernels
 * only (no allocation, copy or memset), so it can be captured in a graph. */
rt_status rt_batch_run(const rt_batch* batch, void* stream);

/* Total 64-probe tiles of the batch (the queue length). */
rt_status rt_batch_tiles(const rt_batch* batch, int64_t* h_tiles);

/* Step-cap hits of the batch's runs (ordered on `stream`, synchronises it). */
rt_status rt_batch_device_error(const rt_batch* batch, rt_device_err* h_err, void* stream);

void rt_batch_destroy(rt_batch* batch);

/*
 * Autotuner: times every launch shape of a small candidate grid (waves per
 * workgroup x workgroups per CU x tiles per pop x wave-tile shape) on the
 * given jobs, `reps` runs each after one warm-up, and returns the fastest in
 * *h_best with its mean time in *h_best_ms.  d_ws: a batch workspace for these jobs
 * (rt_batch_workspace_bytes), reused by every candidate.  Synchronises
 * `stream`; writes the jobs' outputs.
 */
rt_status rt_batch_autotune(const rt_batch_job* jobs, int32_t n_jobs, int32_t reps, void* d_ws, size_t ws_bytes,
                            void* stream, rt_batch_params* h_best, float* h_best_ms);

/*
 * Graph capture of work issued on `stream` (e.g. builds + rt_batch_run for a
 * sequence of wavelength batches), replayed with rt_graph_launch.
 */
typedef struct rt_graph rt_graph;
rt_status rt_graph_begin(void* stream);
rt_status rt_graph_end(void* stream, rt_graph** out);
rt_status rt_graph_launch(const rt_graph* graph, void* stream);
void rt_graph_destroy(rt_graph* graph);

/*
 * rt_trace_j -- angle-integrated formal solution for the current wavelength
 * batch: the mean intensity J[l][p] = sum_d w_d I_d[l][p] over the n_dir
 * directions with quadrature weights d_weights [n_dir] (device float, e.g.
 * 1/n_dir), and optionally psi[l][p] = sum_d w_d (1 - exp(-tau_1,d)) with
 * tau_1,d the optical depth of the first segment (the probe's own cell to its
 * boundary), the diagonal of the approximate operator used by accelerated
 * lambda iteration.  The march is rt_trace's (same params, same cells); I is
 * never written.  Directions are split into chunks marched by separate waves;
 * with d_work (device, work_bytes, nullable) the chunk partials are summed in a
 * fixed order (deterministic), without it every wave takes all directions.
 * rt_trace_j_workspace_bytes gives the work size for full parallelism (0 when
 * one chunk already fills the device).  d_J, d_psi: [batch][n_probes].
 * Errors as rt_trace.  Asynchronous; allocates nothing.
 */
rt_status rt_trace_j(const rt_scene* scene, const rt_trace_params* params, const float* d_dirs,
                     const float* d_weights, int32_t n_dir, const int32_t* d_probes, int64_t n_probes, float* d_J,
                     float* d_psi, float* d_work, size_t work_bytes, void* stream);
rt_status rt_trace_j_workspace_bytes(const rt_scene* scene, int32_t n_dir, int64_t n_probes, int32_t with_psi,
                                     size_t* h_bytes);

/*
 * rt_trace_j_noalloc -- rt_trace_j for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the direction-chunk partials live in a device array of
 * the library (64 MiB, one per device, held until the process ends) instead
 * of a caller workspace.  Same arguments as rt_trace_j without d_work; the
 * result equals rt_trace_j's with a workspace of rt_trace_j_workspace_bytes
 * bit for bit (same chunks, same fixed-order reduction).
 * Limit: the partials, rt_trace_j_workspace_bytes with the batch's wavelength
 * count, must fit 64 MiB (e.g. at most 16,384 probes at 64 directions with
 * psi); larger requests fail with RT_E_ARG before any device work.  Calls
 * that overlap on one device (concurrent streams or threads) share the array
 * and race; the caller serialises them.  Calls nothing that allocates.
 * Asynchronous.  Errors as rt_trace_j, RT_E_HIP if the array's address cannot
 * be looked up.
 */
rt_status rt_trace_j_noalloc(const rt_scene* scene, const rt_trace_params* params, const float* d_dirs,
                             const float* d_weights, int32_t n_dir, const int32_t* d_probes, int64_t n_probes,
                             float* d_J, float* d_psi, void* stream);

/*
 * ------------------------------------------------- neural radiance cache
 * Truncated march: every ray is marched to path length t_trunc (index units);
 * the part beyond is the far field, to be supplied by a learned cache (the
 * neural radiance cache form of the formal solution).  Outputs, for rays
 * (dir, probe) and batch wavelengths l:
 *   d_I_near [n_dir][nl][n_probes]  near-field intensity (for rays that need no
 *                                   query, the complete intensity incl. I0)
 *   d_T_near [n_dir][nl][n_probes]  transmittance to the truncation point (0 when
 *                                   no query is needed)
 *   d_I_far  [n_dir][nl][n_probes]  gen != 0 only: exact far-field intensity
 *                                   arriving at the truncation point (incl. I0)
 *   d_feat   [n_dir][n_probes][4]   truncation point x, y, z (index space; z = 0.5
 *                                   in 2D) and q: 0 if the ray needs no query,
 *                                   else 1 + the index of the block whose cell
 *                                   holds the truncation point (the block the
 *                                   fallback map is indexed by)
 *   d_fstat  [n_dir][nl][n_probes][4] level statistics of the cell there: mean
 *                                   and variance of ln(chi ds0), of ln(eta ds0)
 * The complete intensity is I = I_near + T_near I_far.  The truncation point
 * is t_trunc, moved to the entry of the next non-empty cell when t_trunc lies
 * in empty space (the far field is the same).  Rays that leave the grid
 * before it need no query.  In inference mode (gen = 0) a ray whose
 * truncation block is flagged in d_fallback (uint8 [n_blocks], nullable)
 * keeps marching to the boundary and needs no query.  Grids of 2^24 blocks or
 * more are rejected (q must stay exact in FP32).  Asynchronous.
 */
rt_status rt_trace_truncated(const rt_scene* scene, const rt_trace_params* params, float t_trunc, int32_t gen,
                             const uint8_t* d_fallback, const float* d_dirs, int32_t n_dir, const int32_t* d_probes,
                             int64_t n_probes, float* d_I_near, float* d_T_near, float* d_I_far, float* d_feat,
                             float* d_fstat, void* stream);

/*
 * The cache: an MLP 256 -> 4 x 64 (SiLU) -> 1 on BF16 matrix cores with FP32
 * accumulation, FP32 master weights and Adam.  Input: 16 log-spaced
 * frequencies from 1 to freq_max cycles per domain (sin, cos) of the
 * normalised truncation point, the direction and the wavelength offset within
 * the scene's wavelength range, plus the 4 level statistics; output
 * ln(I_far) / 10.
 *   max_batch  largest training batch (multiple of 256, at most 2^19); sizes the workspace.
 *   freq_max   highest frequency (grid side / 2 in the default set-up).
 *   seed       weight initialisation (uniform +-1/sqrt(fan_in)) and batch sampling.
 * Training rows are 12 floats: x/n_x, y/n_y, z/n_z, w_x, w_y, w_z, wavelength
 * offset, mean ln chi / 10, ln(1 + var ln chi), (mean ln eta - mean ln chi) / 10,
 * ln(1 + var ln eta), weight (0 ignores the row); target ln(I_far) / 10.
 */
typedef struct rt_nrc_desc {
    int32_t max_batch;
    float freq_max;
    uint64_t seed;
} rt_nrc_desc;

typedef struct rt_nrc rt_nrc;

/* Device workspace of the cache for this descriptor: weights, Adam moments,
 * gradients and the training activations of max_batch rows (host only, no
 * device work). */
rt_status rt_nrc_workspace_bytes(const rt_nrc_desc* desc, size_t* h_bytes);
rt_status rt_nrc_num_params(int32_t* h_n);
/* Lays the cache out in the caller's workspace d_ws (at least
 * rt_nrc_workspace_bytes, 256-byte aligned, outliving the handle) and
 * initialises the weights (synchronises `stream`).  Errors: RT_E_ARG (also a
 * null, misaligned or too small workspace), RT_E_HIP. */
rt_status rt_nrc_create(const rt_nrc_desc* desc, void* d_ws, size_t ws_bytes, void* stream, rt_nrc** out);
/* Releases the host handle (the workspace is the caller's).  NULL is ignored. */
void rt_nrc_destroy(rt_nrc* nrc);
/* FP32 master weights, host float [num_params] (checkpoint / restore); ordered on `stream`, synchronises it. */
rt_status rt_nrc_get_weights(const rt_nrc* nrc, float* h_w, void* stream);
rt_status rt_nrc_set_weights(rt_nrc* nrc, const float* h_w, void* stream);
/* Whole training state, for resuming training: FP32 master weights, Adam's first
 * and second moments (host float [num_params] each) and the step count (which
 * also keys the counter-based batch sampling).  Training is deterministic, so
 * steps run after rt_nrc_set_state on a cache created with the same descriptor
 * repeat those run after the matching rt_nrc_get_state bit for bit.
 * Both are ordered on `stream` and synchronise it.
 * Errors: RT_E_ARG (null pointer, negative step), RT_E_HIP. */
rt_status rt_nrc_get_state(const rt_nrc* nrc, float* h_w, float* h_m, float* h_v, int32_t* h_step, void* stream);
rt_status rt_nrc_set_state(rt_nrc* nrc, const float* h_w, const float* h_m, const float* h_v, int32_t step,
                           void* stream);
/* Packs generation-mode outputs of one batch into training rows starting at row0
 * (rows ordered (dir, lam, probe)); d_raw [.][12], d_target [.]. */
rt_status rt_nrc_pack(const rt_scene* scene, const float* d_dirs, int32_t n_dir, int64_t n_probes,
                      const float* d_feat, const float* d_fstat, const float* d_I_far, float* d_raw, float* d_target,
                      int64_t row0, void* stream);
/* `steps` Adam steps (lr, beta 0.9 / 0.999) on batches of `batch` rows sampled
 * from the n rows (mean squared error on the target). */
rt_status rt_nrc_train(rt_nrc* nrc, const float* d_raw, const float* d_target, int64_t n, int32_t steps, int32_t batch,
                       float lr, void* stream);
/* Mean loss of the last training batch (ordered on `stream`, synchronises it). */
rt_status rt_nrc_loss(const rt_nrc* nrc, float* h_loss, void* stream);
/* Gradients of the mean squared error over the first n rows (n multiple of 256,
 * <= max_batch) into d_grad [num_params]; for checking the backward pass. */
rt_status rt_nrc_gradients(rt_nrc* nrc, const float* d_raw, const float* d_target, int64_t n, float* d_grad,
                           void* stream);
/* Network outputs for n training-form rows into d_y [n]. */
rt_status rt_nrc_predict(const rt_nrc* nrc, const float* d_raw, int64_t n, float* d_y, void* stream);
/* I = I_near + T_near exp(10 y) for every query of a truncated trace of the
 * scene's current batch (rays needing no query copy I_near). */
rt_status rt_nrc_compose(const rt_nrc* nrc, const rt_scene* scene, const float* d_dirs, int32_t n_dir,
                         int64_t n_probes, const float* d_feat, const float* d_fstat, const float* d_I_near,
                         const float* d_T_near, float* d_I, void* stream);
/* Held-out check on a generation-mode trace: composed prediction into d_I_pred,
 * relative error against I_near + T_near I_far into d_err (nullable), and
 * d_fallback[block of the truncation point] = 1 wherever it exceeds thresh
 * (the map is not cleared first); d_count (uint32 [n_blocks], nullable, not
 * cleared) counts the checked (query, wavelength) pairs per block.  The map
 * drives rt_trace_truncated's per-ray fallback (nonzero = march on). */
rt_status rt_nrc_validate(const rt_nrc* nrc, const rt_scene* scene, const float* d_dirs, int32_t n_dir,
                          int64_t n_probes, const float* d_feat, const float* d_fstat, const float* d_I_near,
                          const float* d_T_near, const float* d_I_far, float thresh, float* d_I_pred,
                          uint8_t* d_fallback, uint32_t* d_count, float* d_err, void* stream);
/* Flags in d_fallback every block with fewer than min_queries checked pairs in
 * d_count (from rt_nrc_validate calls): the cache is then used only where the
 * held-out check has evidence that it passes.  Asynchronous. */
rt_status rt_nrc_fallback_unverified(const rt_scene* scene, const uint32_t* d_count, int32_t min_queries,
                                     uint8_t* d_fallback, void* stream);

/* Device error counters accumulated by traces of this scene (ordered on `stream`, synchronises it); reset
 * clears them. */
rt_status rt_scene_device_error(const rt_scene* scene, rt_device_err* h_err, void* stream);
rt_status rt_scene_reset_device_error(rt_scene* scene, void* stream);

/* Releases the scene's host handle (its device storage is the caller's workspace).  NULL is ignored. */
void rt_scene_destroy(rt_scene* scene);

/* Thread-local description of the last failure in this thread ("" if none). */
const char* rt_last_error(void);

/* Library version string. */
const char* rt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RT_H */
