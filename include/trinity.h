/*
 * trinity.h -- C-ABI of the MI355X (gfx950) time-dependent radiative-transfer
 * step of TRINITY (Yajima et al., "TRINITY: a three-dimensional time-dependent
 * radiative transfer code for in-vivo near-infrared imaging").
 *
 * The library advances the photon field N[d][v] (voxel v, HEALPix direction
 * d) of a voxelised medium step by step:
 *   inject   a collimated Gaussian pulse at a surface point (Sec. 3.1);
 *   collide  N_c[:,v] = a_v N[:,v] + b_v (P N)[:,v] -- Eq. (10) with the
 *            explicit source of Eq. (2)/(12), P the discrete Henyey-Greenstein
 *            matrix of Eq. (11) on HEALPix directions (Sec. 2.1);
 *   sweep    move every direction's photons one plane along long
 *            characteristics that cross the box from face to face (Sec. 2.1,
 *            Fig. 1), absorb what leaves the box (Sec. 3.1), reflect and
 *            refract at refractive-index jumps (Eq. 13-14, Sec. 3.3);
 *   tally    per-step light leaving through each detector patch (Fig. 9) and
 *            a photon budget (injected, absorbed, escaped, in the box).
 *
 * Conventions that hold for every call:
 *  - Every call returns a tr_status; nothing else crosses the ABI on error.
 *    tr_last_error() gives a message for the calling thread's last failure.
 *  - A medium whose device work failed (TR_EDEVICE, TR_ENUMERIC) is poisoned:
 *    every later call on it except tr_destroy_medium returns TR_ESTATE.
 *  - Inputs are copied during the call; the caller may free them on return.
 *  - Outputs are caller-allocated.  The library owns all of its device memory
 *    and frees it in tr_destroy_medium.
 *  - Voxel arrays are float32, indexed v = (z*ny + y)*nx + x, x fastest.  z is
 *    depth; the top face z = 0 carries source and detectors.  Lengths are mm,
 *    coefficients 1/mm, times ps.
 *  - Faces are numbered face = 2*axis + side: axis 0 = x, 1 = y, 2 = z; side 0
 *    is the low-index face, side 1 the high-index face (face 4 = top).
 *  - Device work is queued on the HIP stream given at creation and is
 *    asynchronous unless a call says it synchronises.
 *  - Calls on one medium must not overlap (one thread at a time per medium).
 */
#ifndef TRINITY_H
#define TRINITY_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tr_medium tr_medium;   /* opaque, library-owned */

typedef enum {
  TR_OK = 0,
  TR_EINVAL = -1,     /* bad argument; nothing was changed */
  TR_ENOMEM = -2,     /* device or host allocation failed; nothing was changed */
  TR_EDEVICE = -3,    /* a HIP call failed; the medium is poisoned */
  TR_ENUMERIC = -4,   /* NaN or Inf in the photon budget; the medium is poisoned */
  TR_ESTATE = -5      /* call on a poisoned medium, or out of order */
} tr_status;

enum { TR_HG_SINKHORN = 0, TR_HG_ROW = 1 };
enum { TR_COEF_PAPER = 0, TR_COEF_ABS_EXACT = 1 };
enum { TR_ADVANCE_AUTO = 0, TR_ADVANCE_PHASE = 1, TR_ADVANCE_SPLIT = 2, TR_ADVANCE_RETARDED = 3 };
enum { TR_PREC_FP32 = 0, TR_PREC_BF16SPLIT = 1 };
enum { TR_SOURCE_EXPLICIT = 0, TR_SOURCE_IMPLICIT = 1 };
enum { TR_TRANSPORT_AUTO = 0, TR_TRANSPORT_SWEEP = 1 };
enum { TR_RSRC_TARGET = 0, TR_RSRC_FLUX = 1 };

typedef struct {
  int nx, ny, nz;     /* voxels per axis, each >= 1 and <= 4096, and at most 107374080
                         voxels in all (the collision kernels address the field with
                         32-bit offsets spanning five rows) */
  double dx_mm;       /* voxel edge */
  int nside;          /* HEALPix resolution: N = 12 nside^2 directions, RING order, 1..16 */
  double g;           /* Henyey-Greenstein anisotropy, Eq. (11); -1 < g < 1 */
  double dt_ps;       /* time step; 0 => dx * min(n) / c0 (light at c0/min(n) crosses one voxel) */
  int hg_norm;        /* TR_HG_SINKHORN: P = D K D, rows and columns sum to 1 (default);
                         TR_HG_ROW: rows of K divided by their sums */
  int coef;           /* TR_COEF_PAPER: b = (mu_s/mu_t)(1 - e^{-mu_t l}), Eq. (9)-(10) with
                         S1 = S0; TR_COEF_ABS_EXACT: b = e^{-mu_a l}(1 - e^{-mu_s l}) */
  int advance;        /* TR_ADVANCE_AUTO: phase if n is uniform, else split;
                         TR_ADVANCE_PHASE: all photons of a direction move one plane on the
                         steps the direction's phase selects (n must be uniform);
                         TR_ADVANCE_SPLIT: the fraction nu_d * min(n)/n_v moves each step;
                         TR_ADVANCE_RETARDED: time steps below the crossing time (Sec. 2.1,
                         the retarded formal solution; Sec. 2.2 and 3.1 run at a tenth and
                         a fifth of it).  The hop between planes of direction d,
                         dr_d = dx/|Omega_a|, takes D_d = dr_d n/(c0 dt) >= 1 steps; every
                         step collides the field with the hop's coefficients
                         a = e^{-mu_t dr_d}, b = omega (1 - a) into a history of the last
                         floor(max D_d) + 1 collided fields, and a voxel takes its upwind
                         voxel's collided value at the retarded step m + 1 - D_d (linear
                         between the two nearest steps).  A voxel's photons cross a plane at
                         1/D_d of them per step: the source puts D_d times its per-step
                         photons into its voxels, and escape, detector and absorption
                         tallies count 1/D_d of the content per step.  A varying n makes
                         the hop from voxel u last D_d n_u / min(n) steps, and a hop into a
                         voxel of another index is intercepted (Eq. 13-14, Sec. 3.3): of
                         the flux that reaches the interface, R returns along the mirror
                         direction and 1 - R enters along Snell's direction, each turned
                         into content with its new hop's duration (at most 127 distinct
                         values of n).  Needs FP32, the explicit source, TR_COEF_PAPER, and
                         at most 192 directions unless nside_scatter puts the source on a
                         coarser grid (then a = e^{-mu_t dr_d} per fine direction and
                         b (P N) comes from the coarse bins; uniform n only); see also
                         retarded_source; tr_set_state, the adjoint and the server refuse
                         it */
  int precision;      /* TR_PREC_FP32 or TR_PREC_BF16SPLIT (P and N split into bf16 hi+lo,
                         the four bf16 MFMA products, fp32 accumulation; each value
                         off by at most 2^-16 of itself) */
  int source;         /* TR_SOURCE_EXPLICIT: S1 := S0 in Eq. (10) (default);
                         TR_SOURCE_IMPLICIT: S1 is the source of the outgoing intensity,
                         the fixed point of Sec. 2.4 Steps 3-6, solved per voxel in
                         closed form through P = V diag(lambda) V^T:
                         N_c = V diag((a + w0 lambda)/(1 - w1 lambda)) V^T N,
                         w0 = omega f0, w1 = omega f1 (Eq. 9).  Needs TR_HG_SINKHORN,
                         TR_COEF_PAPER, TR_PREC_FP32 and at most 192 directions. */
  int nside_scatter;  /* 0 (or nside): scatter on the transport directions.  Else the
                         source is computed on the coarser HEALPix grid of this nside
                         (nside / nside_scatter a power of two, at most 192 coarse
                         directions; Sec. 2.1, 3072 transport and 192 scattering bins):
                         the photons of a coarse bin are the sum over its fine
                         children, are scattered by the coarse phase matrix, and each
                         child of the target bin gets an equal share.  Needs the
                         explicit source and FP32. */
  int transport;      /* TR_TRANSPORT_AUTO (0): in phase advance with the explicit source on
                         one angular grid and at most 192 directions (and both fields
                         within 2 GiB, each extent <= 1023), the collision kernel moves
                         each collided value straight to its downwind voxel: one kernel
                         per step instead of a collision and a sweep, same field values.
                         TR_TRANSPORT_SWEEP (1): always the separate sweep kernel. */
  int retarded_source;  /* TR_ADVANCE_RETARDED only.  TR_RSRC_TARGET (0): the source of
                         direction i weighted by its own hop's 1 - e^{-dtau_i} (the formal
                         solution of Eq. 10 along the target's hop, as the paper prints it;
                         with hops of unequal length scattering conserves light only to
                         O(dtau)).  TR_RSRC_FLUX (1): C_i = a_i N_i + D_i omega
                         sum_j P_ij (1 - a_j) N_j / D_j -- what each direction scatters per
                         step is what the others gain, so light is conserved exactly; it
                         agrees with TR_RSRC_TARGET to first order in dtau.  With
                         nside_scatter the coarse sums weight fine direction j by
                         (1 - a_j) / D_j and fine direction i takes D_i times its share
                         of the coarse source. */
} tr_grid_desc;

typedef struct {
  int ndir;           /* N = 12 nside^2 */
  int nvox;           /* nx*ny*nz */
  int mode;           /* TR_ADVANCE_PHASE, TR_ADVANCE_SPLIT or TR_ADVANCE_RETARDED as resolved */
  int ninterceptions; /* (direction, voxel) pairs whose move crosses an index jump */
  double dt_ps;       /* time step as resolved */
  long long steps_done;
  size_t device_bytes;  /* device memory the medium holds */
  int history;        /* TR_ADVANCE_RETARDED: collided fields kept (floor(max D_d) + 1); else 0 */
  int moves_fused;    /* 1 if the collision kernel also does the moves (see transport) */
} tr_info;

/* ---- medium life cycle ------------------------------------------------- */

/* Build a medium from per-voxel mu_a, mu_s (1/mm) and refractive index n
 * (Table 1 quantities; c = c0/n, Sec. 2.1).  The arrays hold nx*ny*nz floats
 * each, on the host (arrays_on_device = 0) or on the current device
 * (arrays_on_device = 1).  hip_stream is a hipStream_t (NULL = the null
 * stream) on which all of this medium's work is queued.  The host set-up
 * (directions, phase matrix, ray lattice, coefficients, interface lists) runs
 * in FP64 before the call returns; the state starts at zero with step 0 next.
 * TR_EINVAL: bad sizes, nside, g, negative coefficients, n < 1, a time step that
 * moves light more than one plane per step, phase mode with non-uniform n.
 * TR_ENOMEM: device memory exhausted.  On error *out is NULL. */
tr_status tr_create_medium(const tr_grid_desc* desc, const float* mua, const float* mus,
                           const float* n, int arrays_on_device, void* hip_stream,
                           tr_medium** out);

/* Device bytes tr_create_medium would allocate for this descriptor with
 * ndet detectors and room for max_steps steps (for admission by HBM budget),
 * for a uniform refractive index: an upper bound, within a few per cent.
 * Returns 0 for an invalid descriptor, and for TR_ADVANCE_RETARDED, whose
 * history length depends on n (tr_bytes_required_n covers it). */
size_t tr_bytes_required(const tr_grid_desc* desc, int ndet, int max_steps);

/* The same for the given refractive index n (nx*ny*nz floats, host memory):
 * adds what n decides -- the mode TR_ADVANCE_AUTO resolves to, the interface
 * and gather tables of index jumps, the index classes, and with
 * TR_ADVANCE_RETARDED the history of floor(max D) + 1 fields.  Runs the host
 * set-up of the time step and the interceptions (FP64, no device work).
 * Returns 0 for an invalid descriptor or n, or phase advance with a
 * non-uniform n. */
size_t tr_bytes_required_n(const tr_grid_desc* desc, const float* n, int ndet, int max_steps);

/* Release every resource of the medium; waits for its queued work. NULL is OK. */
tr_status tr_destroy_medium(tr_medium* m);

/* Message for the calling thread's last failed call ("" if none). */
const char* tr_last_error(void);

/* ---- problem statement (Sec. 3.1) ------------------------------------- */

/* Collimated pulse (Sec. 3.1: pulse collimated within 15 degrees at a surface
 * point).  Photons enter the top-face voxel (ix, iy) (w = 1) or the 2x2 block
 * (ix..ix+1, iy..iy+1) (w = 2) in the directions whose centres lie within
 * cone_deg of +z (or the 4 nearest when none does).  The pulse is a Gaussian
 * of the given FWHM centred at t0; step m receives its integral over
 * [m dt, (m+1) dt), scaled so the pulse after t = 0 holds total_photons.
 * Replaces any earlier source; takes effect from the next step.
 * TR_EINVAL: voxels outside the top face, w not 1 or 2, fwhm <= 0. */
tr_status tr_set_source(tr_medium* m, int ix, int iy, int w, double cone_deg, double t0_ps,
                        double fwhm_ps, double total_photons);

/* Detector patches (Sec. 3.1: detectors with the source's opening angle).
 * Detector k is the voxel on face face[k] at in-face indices (i[k], j[k]) --
 * the voxel indices along the two other axes in increasing axis order.  It
 * records, each step, the light leaving through that face from that voxel in
 * directions within cone_deg of the face's outward normal (4 nearest when
 * none; every direction when cone_deg <= 0).  tr_read_detectors bins the
 * per-step records into nbins bins of bin_ps.  1 <= ndet <= 64.  Clears the
 * detector records of steps already run.  TR_EINVAL: bad face or indices. */
tr_status tr_set_detectors(tr_medium* m, int ndet, const int* face, const int* i, const int* j,
                           double cone_deg, double bin_ps, int nbins);

/* ---- stepping (Sec. 2.4, Steps 3-7) ------------------------------------ */

/* Queue nsteps steps (inject, collide, sweep, tally) on the medium's stream
 * and return without waiting.  Steps run from the medium's step counter
 * onward.  TR_EINVAL: nsteps < 0. */
tr_status tr_step(tr_medium* m, int nsteps);

/* tr_step, then wait for the stream and check the photon budget of the new
 * steps for NaN/Inf (TR_ENUMERIC). */
tr_status tr_solve(tr_medium* m, int nsteps);

/* tr_step for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same steps with the same kernels, queued kernel by kernel, with no device
 * or host allocation of any kind: the per-step records are not grown and no
 * graph is instantiated.  The kernels' per-workgroup partial sums and the
 * tally kernel's per-step sums and counter live in a workspace of 4 MiB per
 * GPU (a file-scope device array the library holds until the process ends)
 * instead of the medium's own buffers.  Every call on one GPU shares that
 * workspace and the call clears only the counter, so calls that overlap on
 * one GPU race: serialise them (one stream, or wait between them).  Needs
 * steps_done + nsteps <= the record capacity (1024 steps from tr_create_medium
 * and tr_set_detectors; tr_step and tr_solve grow it).  Asynchronous on the
 * medium's stream, like tr_step; tr_synchronize reports the budget check.
 * TR_EINVAL: nsteps < 0, steps beyond the record capacity, or a medium whose
 * step needs more workspace than 4 MiB (2 x collision workgroups + 7 x the
 * larger of the sweep and collision workgroup counts + 9 doubles). */
tr_status tr_step_noalloc(tr_medium* m, int nsteps);

/* Wait for the medium's queued work; report a device error if one occurred. */
tr_status tr_synchronize(tr_medium* m);

/* Zero the state, the detector records and the budget; the next step is 0. */
tr_status tr_reset(tr_medium* m);

/* ---- read-out (Fig. 9; synchronises) ------------------------------------ */

/* Detector signals binned in time: out[k*nbins + j] = light recorded by
 * detector k in [j bin_ps, (j+1) bin_ps), the light of step m spread evenly
 * over [m dt, (m+1) dt).  n_out must be >= ndet*nbins.  FP64. */
tr_status tr_read_detectors(tr_medium* m, double* out, size_t n_out);

/* Per-step detector records: out[k*steps_done + s].  n_out >= ndet*steps_done. */
tr_status tr_read_detector_steps(tr_medium* m, double* out, size_t n_out);

/* Photon budget per step: out[s*9 + q], q = 0 injected, 1 absorbed, 2 in the
 * box after the step, 3..8 escaped through faces 0..5.  n_out >= 9*steps_done. */
tr_status tr_read_budget(tr_medium* m, double* out, size_t n_out);

/* Energy density proxy E[v] = sum_d N[d][v] (Figs. 7-8), nvox floats, written
 * to host memory (on_device = 0) or device memory (on_device = 1). */
tr_status tr_read_energy(tr_medium* m, float* out, int on_device);

/* Copy the photon field N[d][v] (ndir*nvox floats, direction-major) out of
 * or into the medium, in host or device memory.  For tests and restarts.  The
 * copy is queued on the medium's stream after its earlier work and waited for;
 * device data that the caller wrote on another stream must be complete
 * before the call.  With TR_ADVANCE_RETARDED the state also holds the history
 * of collided fields, so tr_set_state returns TR_EINVAL. */
tr_status tr_get_state(tr_medium* m, float* out, int on_device);
tr_status tr_set_state(tr_medium* m, const float* in, int on_device);

tr_status tr_get_info(tr_medium* m, tr_info* out);

/* ---- resuming a solve ----------------------------------------------------- */

/* Save and restore everything a solve carries from step to step, so that a
 * solve can stop and resume (in this process or another) with the same
 * results as an uninterrupted one: the photon field N, with TR_ADVANCE_RETARDED
 * also the history of collided fields, the step index, and the per-step
 * detector records and budget rows of the steps done.  A saved state is a
 * block of host memory laid out as a 64-byte header (magic "TRSTATE1", a
 * 64-bit fingerprint of the medium, then steps, ndir, nvox, ndet, history and
 * the total size as 64-bit integers), the field [ndir][nvox] float32, the
 * history [history][ndir][nvox] float32, the budget rows [steps][9] FP64 and
 * the detector records [ndet][steps] FP64, in the host's byte order.
 *
 * tr_state_bytes: the size of a saved state of the medium as it stands.
 * tr_save_state: waits for the medium's queued work (reporting its errors as
 *   tr_synchronize does) and writes the state to out (host memory,
 *   n_out >= tr_state_bytes).  TR_EINVAL: null or short output.
 * tr_load_state: restores a saved state into a medium built with the same
 *   description, the same mu_a, mu_s and n, the same source and the same
 *   detectors (the fingerprint checks all of them); the next step is the saved
 *   step index.  Checkpoints of an earlier tr_solve_checkpointed are dropped.
 *   Synchronises.  TR_EINVAL: not a saved state, truncated, of another shape,
 *   or saved from a medium that differs in any of the above (nothing changed);
 *   TR_ENOMEM: no room for the records. */
tr_status tr_state_bytes(tr_medium* m, size_t* bytes);
tr_status tr_save_state(tr_medium* m, void* out, size_t n_out);
tr_status tr_load_state(tr_medium* m, const void* in, size_t n_in);

/* ---- gradients (adjoint) ------------------------------------------------- */

/* Reset the medium, then solve nsteps steps from step 0 keeping a copy of the
 * field every ckpt_every steps (memory: ceil(nsteps/ckpt_every) fields) for
 * tr_backward.  Synchronises.  TR_EINVAL: nsteps or ckpt_every < 1. */
tr_status tr_solve_checkpointed(tr_medium* m, int nsteps, int ckpt_every);

/* Gradient of a loss of the binned detector signals with respect to the
 * per-voxel mu_a and mu_s, by the exact adjoint of the steps run by
 * tr_solve_checkpointed: the transposed sweep, detector read-out and collision
 * run backwards through time, segment by segment, each segment's fields
 * recomputed from its checkpoint.  dL_dbins[k*nbins + j] = dL/d(binned signal
 * of detector k in bin j) (host, FP64).  dmua, dmus: nvox floats each (host).
 * The medium's field, step counter and records are as before the call.
 * Supported for phase advance, FP32, up to 192 directions.  TR_ESTATE: no
 * checkpointed solve to differentiate; TR_EINVAL: unsupported configuration;
 * TR_ENOMEM: no room for ckpt_every recomputed fields. */
tr_status tr_backward(tr_medium* m, const double* dL_dbins, float* dmua, float* dmus);

/* ---- kernel timing ------------------------------------------------------ */

/* Kernel kinds reported by tr_profile_end.  With a two-level angular grid,
 * TR_K_COLLIDE is the contraction on the coarse directions alone; the sums
 * over children and the return to the fine directions are TR_K_COARSE_SUM and
 * TR_K_APPLY (no launches otherwise). */
enum { TR_K_INJECT = 0, TR_K_COLLIDE = 1, TR_K_SWEEP = 2, TR_K_GATHER = 3, TR_K_REDUCE = 4,
       TR_K_COARSE_SUM = 5, TR_K_APPLY = 6, TR_K_COUNT = 7 };

/* Start timing: the next steps (up to max_steps of them) are queued one kernel
 * at a time with a pair of HIP events on the medium's stream around every
 * kernel (no graph replay while timing).  TR_EINVAL: max_steps < 1. */
tr_status tr_profile_begin(tr_medium* m, int max_steps);

/* Stop timing, wait for the stream, and return per kernel kind the summed
 * device time in ms (kernel_ms[TR_K_COUNT]) and the number of launches timed
 * (launches[TR_K_COUNT]).  TR_ESTATE if timing was not started. */
tr_status tr_profile_end(tr_medium* m, double* kernel_ms, int* launches);

/* ---- continuous-batching server ----------------------------------------- */
/*
 * Serves many forward solves, as a diffuse-optical-tomography reconstruction
 * issues them (Sec. 1, Sec. 4), on one device at once.  All requests share the
 * angular set-up (nside, g, normalisation, coefficient form) and run in phase
 * mode (uniform refractive index per request), FP32; grids, media, sources,
 * detectors and step counts differ per request.  Requests are admitted in
 * submission order whenever a slot is free and their device memory fits in
 * the remaining budget; every server step advances all admitted requests by
 * one step in batched kernels, so requests that arrive while others run join
 * the batch as soon as memory frees up.  A request's result is the same bits
 * whether it runs alone or in a batch.
 */
typedef struct tr_server tr_server;   /* opaque, library-owned */

typedef struct {
  int nside;            /* 1..4 (up to 192 directions) */
  double g;             /* Henyey-Greenstein anisotropy */
  int hg_norm;          /* as tr_grid_desc */
  int coef;             /* as tr_grid_desc */
  size_t budget_bytes;  /* device memory the server may hold for requests */
  int max_slots;        /* requests on the device at once, 1..256 */
} tr_server_desc;

typedef struct {
  int nx, ny, nz;       /* voxels per axis */
  double dx_mm;
  double dt_ps;         /* 0 => dx * n / c0 */
  const float* mua;     /* host arrays of nx*ny*nz values, copied at submit */
  const float* mus;
  const float* n;       /* must be uniform */
  int src_ix, src_iy, src_w;   /* as tr_set_source */
  double src_cone_deg, t0_ps, fwhm_ps, total_photons;
  int ndet;             /* as tr_set_detectors */
  const int* det_face;
  const int* det_i;
  const int* det_j;
  double det_cone_deg, bin_ps;
  int nbins;
  int nsteps;           /* steps the solve runs, >= 1 */
} tr_request;

enum { TR_REQ_QUEUED = 0, TR_REQ_RUNNING = 1, TR_REQ_DONE = 2, TR_REQ_FAILED = 3,
       TR_REQ_CANCELLED = 4 };

typedef struct {
  int status;           /* TR_REQ_* */
  long long steps_done;
  double queued_ms;     /* submit to admission (or to now / cancellation) */
  double run_ms;        /* admission to completion (or to now) */
  size_t bytes;         /* device memory the request holds while admitted */
} tr_request_info;

/* Create a server whose work is queued on hip_stream.  TR_EINVAL: bad
 * descriptor; TR_ENOMEM: device set-up failed. */
tr_status tr_server_create(const tr_server_desc* desc, void* hip_stream, tr_server** out);

/* Release the server and every request it holds; waits for its queued work. */
tr_status tr_server_destroy(tr_server* s);

/* Device bytes a request would hold while admitted (validates it). */
tr_status tr_server_request_bytes(const tr_server* s, const tr_request* req, size_t* bytes);

/* Validate and queue a request (inputs are copied); *id identifies it.
 * TR_EINVAL: invalid request (bad sizes, non-finite or negative coefficients,
 * non-uniform n, ...); TR_ENOMEM: the request alone exceeds the budget. */
tr_status tr_server_submit(tr_server* s, const tr_request* req, long long* id);

/* Retire finished and cancelled requests, admit queued ones while slots and
 * budget allow, then run up to max_steps server steps (fewer when an admitted
 * request finishes earlier) and retire what finished.  Synchronises when a
 * request finishes.  *running / *queued (may be NULL) receive the counts. */
tr_status tr_server_advance(tr_server* s, int max_steps, int* running, int* queued);

/* State and timing of a request.  TR_EINVAL: unknown id. */
tr_status tr_server_info(tr_server* s, long long id, tr_request_info* out);

/* Results of a finished request: binned detector signals (ndet*nbins, as
 * tr_read_detectors) and per-step budget (nsteps*9, as tr_read_budget); either
 * pointer may be NULL.  TR_ESTATE: not done; TR_ENUMERIC: the request failed
 * (its budget went non-finite) -- other requests are unaffected. */
tr_status tr_server_result(tr_server* s, long long id, double* det, size_t n_det, double* budget,
                           size_t n_budget);

/* Cancel a queued or running request; a running one leaves at the next advance. */
tr_status tr_server_cancel(tr_server* s, long long id);

/* ---- host set-up tables (no device needed; for checking the set-up) ---- */

/* HEALPix RING centres (Sec. 2.1), out[3*N]. */
tr_status tr_host_directions(int nside, double* out);

/* For every direction of nside, the direction of the coarser grid nside_c
 * (nside / nside_c a power of two) whose pixel contains it, out[12 nside^2]. */
tr_status tr_host_parents(int nside, int nside_c, int* out);

/* Discrete phase matrix P[i*N + j] (Eq. 11-12) for directions of nside. */
tr_status tr_host_phase_matrix(int nside, double g, int hg_norm, double* out);

/* Ray lattice of the grid: axis[d], sign[d] and offset[(d*2 + q)*(maxext+1) + k]
 * = transverse offset of the ray at plane k for transverse axis q (0 = b, 1 = c),
 * maxext = max(nx, ny, nz). */
tr_status tr_host_lattice(int nside, int nx, int ny, int nz, int* axis, int* sign, int* offset);

/* Move tables of phase advance with the moves in the collision kernel (the
 * lattice's plane-to-plane moves, Sec. 2.1 and Fig. 1), NP = 12 nside^2
 * rounded up to a multiple of 32, maxext = max(nx, ny, nz) <= 1023.
 * tab[d*maxext + p] (NP + 1 rows): for a voxel at coordinate p along direction
 * d's dominant axis, 64 times the flat offset of its move plus the mask of the
 * faces (2 axis + side) the move may leave through; row NP and rows of padding
 * directions are zero.  dir[d] = 10 axis | 3 << (2 axis + 8).  reverse = 1:
 * the inverse moves of the adjoint (each voxel back to the voxel whose photons
 * moved into it, on the box taken periodically along the dominant axis).
 * TR_EINVAL: a direction whose transverse shifts are not -1, 0, +1 of one sign
 * (such grids step with the separate sweep). */
tr_status tr_host_move_tables(int nside, int nx, int ny, int nz, int reverse, int* tab, int* dir);

/* Per-voxel collision coefficients a, b and relative path r (split-mode move
 * fraction factor), and the resolved time step. */
tr_status tr_host_coefficients(const tr_grid_desc* desc, const float* mua, const float* mus,
                               const float* n, double* a, double* b, double* r, double* dt_ps);

/* Directions within cone_deg of the unit vector (ax, ay, az), 4 nearest when
 * none: indices written to out (capacity cap), count to *count. */
tr_status tr_host_cone_set(int nside, double ax, double ay, double az, double cone_deg,
                           int* out, int cap, int* count);

/* Pulse weights q_m for m = m0 .. m0+count-1 (see tr_set_source). */
tr_status tr_host_pulse(double dt_ps, double t0_ps, double fwhm_ps, double total, int m0,
                        int count, double* out);

/* Interface interceptions (Eq. 13-14) of the grid: arrays of capacity cap,
 * count written to *count (also when it exceeds cap, in which case nothing
 * else is written). */
tr_status tr_host_interceptions(const tr_grid_desc* desc, const float* n, int* d, int* v,
                                int* w, double* R, int* d_refl, int* d_refr, int cap,
                                int* count);

/* ---- Measurement --------------------------------------------------------
 * Not part of the method: a probe of what the matrix cores deliver on the GPU
 * at hand, the ceiling beside the datasheet peak for the collision kernels'
 * rates. */
enum { TR_PROBE_MFMA_F32 = 0, TR_PROBE_MFMA_BF16 = 1 };

/* Runs `blocks` workgroups of 512 threads on the current device, each
 * wavefront issuing iters x 8 independent MFMAs from registers (kind
 * TR_PROBE_MFMA_F32: 32x32x2 FP32, the FP32 collision's instruction;
 * TR_PROBE_MFMA_BF16: 32x32x16 bf16, the BF16-split one), once to warm up and
 * once timed with HIP events on a stream of its own.  Writes the achieved
 * TFLOP/s (2 M N K per MFMA) to *tflops and the timed launch's duration to
 * *ms.  Allocates and frees a small device buffer (blocks x 2 KiB).
 * TR_EINVAL: unknown kind, iters outside 1..2^20, blocks outside 1..2^16
 * (bounds that keep a launch to about two minutes at most), or a null output;
 * TR_EDEVICE: a HIP call failed. */
tr_status tr_probe_mfma(int kind, int iters, int blocks, double* tflops, double* ms);

#ifdef __cplusplus
}
#endif
#endif /* TRINITY_H */
