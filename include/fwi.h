/*
 * fwi.h -- C ABI of libfwi.so, the MI355X (gfx950) hot path of acoustic
 * full-waveform inversion.
 *
 * Method (Huot et al., "High-resolution imaging on TPUs"):
 *   Eq. 2  constant-density acoustic wave equation  P_tt = v^2 lap P + s;
 *   Eq. 3  leapfrog  P^{n+1} = -P^{n-1} + 2P^n + v^2 dt^2 lap P^n + dt^2 s^n,
 *          here with a sponge layer (damping 2 eta P_t, centred in time):
 *            P^{n+1} = alpha (2P^n + kappa lap P^n + dt^2 s^n) - beta P^{n-1},
 *            kappa = v^2 dt^2, alpha = 1/(1+eta dt), beta = (1-eta dt)/(1+eta dt);
 *          eta = 0 on the whole model grid, so there the update is Eq. 3.
 *   Fig. 3 / Section 3  central star Laplacian of order >= 8 (8th and 16th
 *          order in Section 4); orders 2, 4, 8, 16 are accepted.
 *   Eq. 1  least-squares misfit phi = ||d_mod - d_obs||^2 (summed over shots),
 *          and its exact gradient with respect to the model velocity
 *          (Section 1 names the misfit and its gradient as the costly part of
 *          every FWI iteration).
 *
 * Conventions shared by every entry point
 *   - All array pointers are DEVICE pointers owned by the caller, unless the
 *     name starts with h_ (host pointer).  float is IEEE fp32, int32_t indices.
 *   - Arrays are C-contiguous, slowest axis first: a 2-D model is [nz][nx], a
 *     3-D model [nz][ny][nx] (x fastest).  Positions are integer model-grid
 *     cells in the same axis order: [D] per source, [D] per receiver.
 *   - The sponge is OUTSIDE the model grid: the library pads the model by
 *     nsponge cells on every face, copying edge velocities, and holds the
 *     wavefield at zero beyond the padded grid.
 *   - Source: one point source per shot; at step n the library adds
 *     alpha dt^2 src[s][n] / dx^D at the source cell (a discrete delta).
 *   - Traces: traces[s][n][r] = P^{n+1} at receiver r of shot s, i.e. the
 *     field at time (n+1) dt; the initial state is P^0 = P^{-1} = 0.
 *   - dv is d(phi)/d(v) on the model grid, summed over shots, with the sponge
 *     damping held fixed.  Outputs are overwritten, never accumulated.
 *   - Work is enqueued on `stream` (a hipStream_t, NULL = default stream);
 *     results are valid once the stream is synchronised.  A propagating call
 *     first copies the (small) position arrays to the host and measures the
 *     velocity range with one reduction kernel into the workspace, then
 *     synchronises `stream` to validate them; fwi_forward, fwi_forward_ckpt,
 *     fwi_backward and fwi_gradient also synchronise it at the end, for the
 *     non-finite check below.  The time loop itself runs without host
 *     synchronisation.
 *   - Workspaces: the caller allocates `ws` (>= the size reported by
 *     fwi_workspace_bytes, 256-byte aligned) and keeps it alive until the
 *     stream has finished the call's work.  The library allocates no device
 *     memory and keeps none between calls.  Calls on distinct workspaces are
 *     independent.
 *
 * Errors: every entry point returns an int status (FWI_OK == 0, negative on
 * error).  Shapes, sizes and pointers are checked on the host before any
 * kernel is launched; positions, velocities and the stability limit right
 * after the velocity-range kernel (which writes only the workspace) and
 * before any step.  On those errors no output is written.  FWI_ENONFINITE is
 * the exception: it is detected after the outputs were written (a non-finite
 * last wavefield, misfit or gradient), and the outputs then hold whatever the
 * run produced.  Asynchronous device faults surface as FWI_EHIP on a later
 * call.  No C++ exception crosses the ABI.
 */
#ifndef FWI_H
#define FWI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum fwi_status {
    FWI_OK = 0,
    FWI_EINVAL = -1,      /* malformed problem description or argument */
    FWI_ECFL = -2,        /* v_max dt / dx above the stability limit of the order */
    FWI_EBOUNDS = -3,     /* a source or receiver position outside the model grid */
    FWI_ENOMEM = -4,      /* workspace (or checkpoint buffer) smaller than required */
    FWI_EHIP = -5,        /* a HIP runtime call failed (message: fwi_last_error) */
    FWI_ENONFINITE = -6,  /* the last wavefield, the misfit or the gradient is not finite */
    FWI_EUNSUPPORTED = -7 /* valid request this build does not implement */
};

enum fwi_mode {
    FWI_MODE_FORWARD = 0,      /* fwi_forward */
    FWI_MODE_GRADIENT = 1,     /* fwi_gradient */
    FWI_MODE_FORWARD_CKPT = 2, /* workspace of fwi_forward_ckpt (excluding ckpt_buf) */
    FWI_MODE_BACKWARD = 3,     /* workspace of fwi_backward (excluding ckpt_buf) */
    FWI_MODE_CKPT_BUF = 4      /* the checkpoint buffer of forward_ckpt / backward */
};

enum fwi_ckpt_kind {
    FWI_CKPT_ALL = 0,     /* keep every time level (small problems, tests) */
    FWI_CKPT_EVERY = 1,   /* snapshot every `every` steps, recompute segments */
    FWI_CKPT_REVOLVE = 2  /* binomial (revolve) schedule over `slots` snapshots */
};

/* eta_max value that asks the library for the default sponge strength. */
#define FWI_ETA_AUTO (-1.0f)

/* One propagation problem: model grid, discretisation and acquisition size. */
typedef struct fwi_problem {
    int32_t ndim;       /* 2 or 3 */
    int32_t shape[3];   /* model grid, slowest axis first ({nz, nx} or {nz, ny, nx}) */
    float dx;           /* grid spacing (m), the same on every axis, > 0 */
    float dt;           /* time step (s), > 0 */
    int32_t nt;         /* number of time steps, >= 1 */
    int32_t order;      /* spatial order 2M: 2, 4, 8 or 16 */
    int32_t nsponge;    /* sponge width nb in cells (>= 0), added on every face */
    float eta_max;      /* peak sponge damping rate (1/s), finite; < 0 (FWI_ETA_AUTO):
                           3 v_max ln(10^3) / (2 nsponge dx), v_max the model's largest
                           velocity (a 10^-3 round-trip decay through the sponge) */
    int32_t nshots;     /* shots, >= 1 */
    int32_t nrec;       /* receivers per shot, >= 0 */
} fwi_problem;

/* Checkpointing policy of the gradient. */
typedef struct fwi_ckpt {
    int32_t kind;          /* enum fwi_ckpt_kind */
    int32_t every;         /* FWI_CKPT_EVERY: interval k >= 1 */
    int32_t slots;         /* FWI_CKPT_REVOLVE: snapshot slots (0: from budget) */
    int32_t reserved;      /* must be 0 */
    uint64_t budget_bytes; /* FWI_CKPT_REVOLVE with slots == 0: snapshot budget */
} fwi_ckpt;

/* Human-readable name of a status code (static string, never NULL). */
const char *fwi_strerror(int status);

/* Detail of the last error raised on the calling thread (static per thread). */
const char *fwi_last_error(void);

/* Largest v_max dt / dx the leapfrog of this order tolerates in ndim
 * dimensions: sqrt(4 / (ndim * S)), S the largest symbol of one axis of the
 * central stencil (Section 3 stencils).  Host-only. */
int fwi_cfl_limit(int32_t ndim, int32_t order, double *h_cfl_max);

/* Workspace bytes needed by an entry point (enum fwi_mode) for `prob`;
 * `ckpt` is read by the gradient modes and may be NULL otherwise.  Host-only. */
int fwi_workspace_bytes(const fwi_problem *prob, int32_t mode, const fwi_ckpt *ckpt,
                        uint64_t *h_bytes);

/*
 * Forward modelling (Eq. 3 with sponge, Fig. 3 stencil): every shot is
 * propagated nt steps through the padded model and sampled at its receivers.
 *   v        [model grid] velocity (m/s), > 0
 *   src      [nshots][nt] source wavelet samples, src[s][n] = w_s(n dt)
 *   src_pos  [nshots][ndim]
 *   rec_pos  [nshots][nrec][ndim]
 *   traces   [nshots][nt][nrec] output
 */
int fwi_forward(const fwi_problem *prob, const float *v, const float *src,
                const int32_t *src_pos, const int32_t *rec_pos, float *traces,
                void *ws, uint64_t ws_bytes, void *stream);

/*
 * fwi_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, bitwise the same traces, with the workspace taken
 * from a fixed array the library holds on each GPU it runs on (128 MiB,
 * kept until the process ends) instead of a caller's `ws`.  The caller
 * passes only inputs and outputs.  Calls no hipMalloc or hipFree.  The
 * array is shared by every call on the same GPU: calls that overlap on one
 * GPU (other streams, other host threads) race; serialise them.  Each call
 * initialises every part of the array it reads.  FWI_ENOMEM if the problem
 * needs more workspace than the array holds (fwi_workspace_bytes, mode
 * FWI_MODE_FORWARD); otherwise the errors of fwi_forward.
 */
int fwi_forward_noalloc(const fwi_problem *prob, const float *v, const float *src,
                        const int32_t *src_pos, const int32_t *rec_pos, float *traces,
                        void *stream);

/*
 * Misfit (Eq. 1) and its gradient with respect to v: forward with
 * checkpoints, residual 2 (d - d_obs), adjoint propagation and the
 * imaging-condition gradient, recomputing the forward field as `ckpt` says.
 *   obs            [nshots][nt][nrec] observed traces
 *   h_misfit       host double: sum over shots, steps, receivers of (d - obs)^2
 *   dv             [model grid] output, sum over shots
 *   traces_or_null [nshots][nt][nrec] modelled traces, or NULL
 */
int fwi_gradient(const fwi_problem *prob, const float *v, const float *src,
                 const int32_t *src_pos, const int32_t *rec_pos, const float *obs,
                 const fwi_ckpt *ckpt, double *h_misfit, float *dv, float *traces_or_null,
                 void *ws, uint64_t ws_bytes, void *stream);

/*
 * The forward half of a differentiable forward: as fwi_forward, and also
 * stores into ckpt_buf (size: FWI_MODE_CKPT_BUF) what fwi_backward needs to
 * recompute the wavefield under policy `ckpt`.
 */
int fwi_forward_ckpt(const fwi_problem *prob, const float *v, const float *src,
                     const int32_t *src_pos, const int32_t *rec_pos, const fwi_ckpt *ckpt,
                     float *traces, void *ckpt_buf, uint64_t ckpt_bytes,
                     void *ws, uint64_t ws_bytes, void *stream);

/*
 * Vector-Jacobian product of fwi_forward with respect to v: given
 * grad_traces = d(loss)/d(traces) [nshots][nt][nrec], writes
 * dv = d(loss)/d(v) [model grid] (sum over shots).  ckpt_buf must hold what
 * fwi_forward_ckpt stored for the same prob, v, src, positions and ckpt; the
 * call recomputes wavefields inside it, so it is consumed (its contents are
 * undefined afterwards and a second backward needs a new forward_ckpt).
 */
int fwi_backward(const fwi_problem *prob, const float *v, const float *src,
                 const int32_t *src_pos, const int32_t *rec_pos, const fwi_ckpt *ckpt,
                 void *ckpt_buf, uint64_t ckpt_bytes, const float *grad_traces,
                 float *dv, void *ws, uint64_t ws_bytes, void *stream);

/*
 * Smallest and largest velocity of a model of n cells (device array v), e.g.
 * to choose dt and the sponge's eta_max.  ws: device scratch of at least
 * 4096 bytes.  Synchronises `stream`.  FWI_EINVAL if a value is not finite.
 */
int fwi_velocity_range(const float *v, int64_t n, float *h_vmin, float *h_vmax, void *ws,
                       uint64_t ws_bytes, void *stream);

/*
 * Diagnostic bandwidth ceiling: out[i] = a[i] + b[i] * c[i] for i < n, a
 * pointwise stream with the forward step's memory mix (three fields read,
 * one written, each once), which bounds the rate any step kernel reading
 * p^n, p^{n-1} and kappa and writing p^{n+1} can reach.  Not part of the
 * method.  variant: bits 0-1 load width (0: 32-bit, 1: 64-bit, 2: 128-bit
 * per lane), bit 2 non-temporal loads and stores, bit 3 a grid of at most
 * 2048 blocks striding over the arrays (else one lane per vector).  n is a
 * positive multiple of 4, arrays 16-byte aligned, out distinct from the
 * inputs.  Asynchronous on `stream`.  FWI_EINVAL on a bad argument.
 */
int fwi_stream_probe(const float *a, const float *b, const float *c, float *out, int64_t n,
                     int32_t variant, void *stream);

/*
 * Diagnostic: the 8th-order forward step's memory pattern with the stencil
 * taken out, to separate what the pattern costs from what the stencil
 * costs.  Not part of the method.  The four device fields are laid out as
 * the 3-D step's (each nz + 8 planes of ny + 8 rows of pitch floats, pitch =
 * nx + 8 rounded up to a multiple of 64, the 4-cell frame included; fields
 * 16-byte aligned).  Blocks of 4 wavefronts march 64 x 16 column tiles
 * through z chunks of zc planes in the step's block order, read cur, prv and
 * kap once per cell one plane ahead and write out = 2 cur + kap * prv at
 * the nz x ny x nx cells inside the frame; nothing else is written.  Mode
 * bits add the step's other work one at a time: 1 the tile's halo rows and
 * columns of cur, 2 the plane staged in LDS with one barrier per plane, 4
 * the 4 + 4 planes of cur around each chunk that the step's z-queue reads;
 * modes 8 and 9 are modes 0 and 1 with 64-bit loads and stores (each lane
 * two adjacent columns).  The output is the same in every mode for finite
 * inputs.  zc = 0 takes
 * the chunk length the forward step picks for this grid; *h_zc (may be
 * NULL) receives the length used.  Asynchronous on `stream`.  FWI_EINVAL on
 * a bad argument (NULL field, out equal to an input, a grid dimension out
 * of 1 .. 2^20, a plane of 2^31 bytes or more, zc < 0, mode outside 0..9).
 */
int fwi_tile_probe(const float *cur, const float *prv, const float *kap, float *out, int nz,
                   int ny, int nx, int zc, int32_t mode, int32_t *h_zc, void *stream);

/*
 * Binomial checkpointing schedule (revolve, Griewank & Walther) for
 * reversing `nsteps` forward steps with `slots` snapshot slots, the initial
 * state being free (it is zero).  Host-only.  Writes up to `cap` actions as
 * (opcode, argument) pairs into h_actions (may be NULL with cap 0), their
 * count into h_count, and the number of forward steps the schedule performs
 * (initial sweep included) into h_forward_steps.
 *   opcodes: 1 ADVANCE(to time), 2 TAKESHOT(slot), 3 RESTORE(slot, time is the
 *            slot's), 4 ADJOINT(time k: consume state k), 5 RESTART (state 0).
 */
int fwi_revolve_schedule(int32_t nsteps, int32_t slots, int32_t *h_actions, int64_t cap,
                         int64_t *h_count, int64_t *h_forward_steps);

/*
 * The launches a gradient with binomial checkpointing issues, for one shot
 * of `nsteps` steps and `slots` snapshot slots, computed on the host without
 * a device: the forward sweep and then the backward sweep, in order.  It
 * exposes the placement of levels in the ring and in snapshot slots for
 * verification.  Writes up to `cap` launches of ten int32 each into h_ops
 * (may be NULL with cap 0) and their count into h_count:
 *   {kind, a, b, c, lev0, fld0, lev1, fld1, lev2, fld2}
 *   kind 1: forward step from level a (reads a and a-1, writes a+1);
 *   kind 2: adjoint step at level a (reads forward level a);
 *   kind 3: snapshot copy for slot a at time b; c & 3 is the direction (0:
 *           levels b, b-1 into fields 2a, 2a+1; 1: fields into the ring; 2:
 *           zero levels 0, -1 in the ring) and c >> 2 a mask (bit w: level
 *           b - w).
 * (lev_i, fld_i) are the launch's level map: level lev_i is read or written
 * in snapshot field fld_i instead of the ring (lev_i = INT32_MIN: unused).
 * Every other level L is ring entry L mod 2.  Errors: FWI_EINVAL for
 * nsteps < 1, slots < 0 or NULL outputs.
 */
int fwi_revolve_plan(int32_t nsteps, int32_t slots, int32_t *h_ops, int64_t cap,
                     int64_t *h_count);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent one-shot jobs.
 *
 * A job is one shot (forward, or misfit + gradient) of its own problem (any
 * grid, 2-D or 3-D, nshots == 1) living in caller-owned device memory `mem`
 * of fwi_job_bytes bytes, which is the HBM footprint used for admission.
 * fwi_jobs_advance moves every job of a set forward by one chunk of
 * `ksteps` time steps of its current phase (forward, checkpoint recompute or
 * adjoint), putting the steps of all the jobs into shared launches: one
 * launch per time step per (dimension, order, direction), blocks indexed
 * over all the jobs' tiles.  Jobs join and leave between chunks.  Each job's
 * arithmetic is independent of which other jobs share its launches, so its
 * results are bitwise the same alone and in a mix.
 * ------------------------------------------------------------------------ */
typedef struct fwi_job fwi_job;

enum fwi_job_kind { FWI_JOB_FORWARD = 0, FWI_JOB_GRADIENT = 1 };

/* Device bytes one job needs (kind FWI_JOB_*).  A gradient job checkpoints
 * by `ckpt` (FWI_CKPT_EVERY or FWI_CKPT_REVOLVE, as for fwi_gradient), or
 * every `chunk` steps when ckpt is NULL; forward jobs ignore it.  Host-only.
 * Errors: FWI_EINVAL for a bad kind, chunk < 1, nshots != 1 or a bad ckpt. */
int fwi_job_bytes(const fwi_problem *prob, int32_t kind, int32_t chunk, const fwi_ckpt *ckpt,
                  uint64_t *h_bytes);

/* Validates and stages a job (synchronises `stream`): as fwi_forward (kind
 * FORWARD: traces required) or fwi_gradient (kind GRADIENT: obs and dv
 * required, traces optional) with the checkpoint policy `ckpt` (NULL: every
 * `chunk` steps).  The job's traces, misfit and gradient are bitwise those of
 * the stand-alone call with the same policy.  A binomial (revolve) job moves
 * between forward recomputation and adjoint steps within one chunk; its
 * snapshots are copies of two consecutive levels, and a restore copies them
 * back into the two-level ring.  All arrays, and `mem`, must stay alive until the job is
 * done and the stream has passed its last advance.  *h_job receives a host
 * handle (fwi_job_destroy). */
int fwi_job_create(const fwi_problem *prob, int32_t kind, int32_t chunk, const fwi_ckpt *ckpt,
                   const float *v, const float *src, const int32_t *src_pos,
                   const int32_t *rec_pos, const float *obs, float *traces, float *dv, void *mem,
                   uint64_t mem_bytes, void *stream, fwi_job **h_job);

/* Workspace (device, 256-byte aligned) of one fwi_jobs_advance over up to
 * njobs jobs and ksteps steps (launch tables and per-step level lists).
 * Host-only.  Errors: FWI_EINVAL for njobs < 0, ksteps < 1 or NULL output. */
int fwi_jobs_ws_bytes(int32_t njobs, int32_t ksteps, uint64_t *h_bytes);

/* Advances every job by up to ksteps steps of its current phase, in shared
 * launches on `stream`, and enqueues the per-job operations due around them
 * (snapshots, final sampling, residual, gradient fold).  Finished jobs are
 * skipped.  Does not synchronise: the launch tables reach the device as
 * kernel arguments of a small assembly kernel that writes them into `ws`, so
 * a caller can enqueue the next chunk while this one runs.  `ws` may be
 * reused by the next call on the same stream (stream order protects it).
 * Errors: FWI_EINVAL for njobs < 0, ksteps < 1 or a NULL job; FWI_ENOMEM if
 * ws_bytes is below fwi_jobs_ws_bytes(njobs, ksteps). */
int fwi_jobs_advance(fwi_job *const *jobs, int32_t njobs, int32_t ksteps, void *ws,
                     uint64_t ws_bytes, void *stream);

/* Host-side state: *h_done = 1 once all of the job's work has been enqueued
 * (results are valid after the stream has finished it); *h_steps_left (if
 * not NULL) = the time steps, forward, recomputation and adjoint, still to
 * enqueue.  Host-only. */
int fwi_job_query(const fwi_job *job, int32_t *h_done, int64_t *h_steps_left);

/* Misfit of a finished gradient job (synchronises `stream`). */
int fwi_job_misfit(const fwi_job *job, double *h_misfit, void *stream);

/* Device address of a gradient job's misfit (one double in the job's memory,
 * valid once the stream has passed the job's last advance), for callers that
 * copy it asynchronously instead of synchronising.  Host-only. */
int fwi_job_misfit_device(const fwi_job *job, const double **d_misfit);

/* Frees the host handle (not `mem`). */
void fwi_job_destroy(fwi_job *job);

#ifdef __cplusplus
}
#endif

#endif /* FWI_H */
