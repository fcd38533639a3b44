/*
 * pat.h -- C ABI of libpat, a gfx950 (MI355X) solver for the forward and
 * adjoint operators of photoacoustic tomography in lossy heterogeneous media
 * (Javaherian & Holman, "A Multi-Grid Iterative Method for Photoacoustic
 * Tomography"), and of the auxiliary operators of its multi-grid ISTA/FISTA.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Arrays are row-major with x fastest: [ny][nx] in 2D, [nz][ny][nx] in 3D.
 *    Per-axis descriptor fields are listed in physical order (x, y, z).
 *  - Sensor data are time-major: data[n][s], n = 0..nt-1 (sample n at t = n dt),
 *    s = 0..n_sensors-1, float32.
 *  - Every float array argument is a caller-owned *device* pointer (e.g. the
 *    data_ptr() of a torch tensor on the HIP device).  Only sensor_pos and
 *    the scalar out-parameters are host memory.  Pointers must stay valid
 *    until the work enqueued on the stream has finished.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *    Calls enqueue work and return without waiting unless stated otherwise.
 *  - Output arrays are overwritten, never accumulated into.
 *  - No C++ exception crosses the ABI; every int-returning call returns one of
 *    the PAT_* codes below.  On a non-zero return nothing was enqueued.
 *  - A plan may be used by one stream at a time.
 */
#ifndef PAT_H
#define PAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
#define PAT_OK          0
#define PAT_EINVAL      1  /* bad descriptor, size, pointer or sensor position   */
#define PAT_EUNSTABLE   2  /* dt above the stability bound c_max dt/dx <= 1/sqrt(d) */
#define PAT_ENOMEM      3  /* device or host allocation failed                    */
#define PAT_EHIP        4  /* a HIP runtime call failed                           */
#define PAT_ENONFINITE  5  /* a non-finite pressure was seen (PAT_CHECK_FINITE)   */
#define PAT_ENOSYS      6  /* combination not supported by this library           */
#define PAT_ETOOBIG     7  /* larger than the fixed scratch of pat_tv_prox_noalloc */

/* ------------------------------------------------------------------ flags */
#define PAT_NO_PML        0x1u  /* switch the PML off: periodic grid             */
#define PAT_CHECK_FINITE  0x2u  /* record non-finite pressure; see pat_plan_sync */
#define PAT_SMOOTH_P0     0x8u  /* filter the initial pressure inside the operators
                                   (section VI-A: a self-adjoint smoothing of p0 in
                                   every forward, included in the adjoint):
                                   H = H0 S, H^T = S H0^T with S = F^-1 w F and w the
                                   product over the axes of the Blackman window centred
                                   on k = 0, 0.42 + 0.5 cos(2 pi m/n) + 0.08 cos(4 pi m/n)
                                   (1 at k = 0, 0 at the Nyquist bin; real and even, so S
                                   is symmetric); pat_adjoint_atd also ends with S */
#define PAT_EOS_INIT      0x10u /* lossy plans: start the density from the equation of
                                   state at t = 0 (section III: with u(0) = 0 the tau term
                                   vanishes, c0^2 (1 - eta L2) rho(0) = p0) instead of
                                   rho(0) = p0 / c0^2; solved by six fixed-point steps
                                   x <- p0/c0^2 + eta L2 x, and pat_adjoint applies their
                                   exact transpose.  pat_plan_create returns PAT_EINVAL
                                   when max |eta| |k|^(y-1) over the medium and the grid
                                   exceeds 0.05 (six steps then no longer reach float
                                   rounding).  Ignored for lossless plans and N_t = 1. */

/* pat_batch_create_ex flags */
#define PAT_BATCH_NO_FUSE 0x1u  /* keep every size class in launches of its own */
#define PAT_BATCH_NO_STAGGER 0x2u  /* start every group's time loop at once */

/*
 * Grid, time axis and physics of one solver instance (one multi-grid level).
 *
 *  ndim         2 or 3.
 *  n[j]         points per axis, including the PML: a power of two in
 *               [16, 1024] (3D: [16, 256]).  n[2] is ignored in 2D.
 *  dx[j]        spacing [m]; node i of axis j sits at origin[j] + i*dx[j].
 *  nt           number of time samples (>= 1): data[n] is recorded at t = n dt.
 *  dt, cfl      time step [s]; dt <= 0 selects dt = cfl * min_j dx[j] / c_max.
 *  pml_size[j]  PML points on each side of axis j, inside the grid (0 = none);
 *               2*pml_size[j] < n[j].
 *  pml_alpha    PML absorption at full depth, nepers per grid point
 *               (section VI-A uses 2).
 *  alpha_power  power-law exponent y of the absorption (section II-A-2);
 *               0 < y < 3, y != 1.  Ignored when alpha0_db is NULL.
 *  n_sensors    number of point detectors (>= 1).
 *  flags        PAT_NO_PML | PAT_CHECK_FINITE | PAT_SMOOTH_P0 | PAT_EOS_INIT.
 */
typedef struct {
  int32_t ndim;
  int32_t n[3];
  double dx[3];
  double origin[3];
  int32_t nt;
  double dt;
  double cfl;
  int32_t pml_size[3];
  double pml_alpha;
  double alpha_power;
  int32_t n_sensors;
  uint32_t flags;
} pat_desc;

/* Derived quantities of a plan (filled by pat_plan_info). */
typedef struct {
  double dt;            /* time step actually used [s]                        */
  double c_ref;         /* reference speed of the k-space correction = max c0  */
  int64_t npoints;      /* grid points                                        */
  int32_t lossy;        /* 1 when alpha0_db was given                          */
  int32_t n_slots;      /* partial-sum slots of the sensor gather              */
  size_t device_bytes;  /* device memory owned by the plan                     */
  size_t state_bytes;   /* size of a forward-state snapshot (pat_forward_range) */
} pat_info;

typedef struct pat_plan pat_plan;
typedef struct pat_batch pat_batch;

/*
 * pat_plan_create -- derive everything the time loop needs, once per level.
 *
 * Implements the set-up of the forward model of section II-A: the medium
 * coefficients of equations mom, mass, state and Twelve (tau, eta from
 * alpha0 and c0), the k-space operators, the per-axis PML (section VI-A) and
 * the linear-interpolation sensor operator M w of section III.
 *
 *  c0, rho0    device, N floats each, sound speed [m/s] and ambient density
 *              [kg/m^3], both > 0 and finite.
 *  alpha0_db   device, N floats, absorption in dB/(MHz^y cm), or NULL for a
 *              lossless medium (then tau = eta = 0 and no absorption pass runs).
 *  sensor_pos  host, n_sensors*ndim doubles, physical (x, y[, z]) per sensor;
 *              each grid coordinate (pos - origin)/dx must lie in [0, n-1].
 *
 * The plan copies what it needs: the caller may free the inputs afterwards.
 * The call synchronises `stream` (it reads back c_max to fix dt).
 * Errors: PAT_EINVAL (descriptor, NULL pointer, sensor outside the grid,
 * non-positive or non-finite medium), PAT_EUNSTABLE, PAT_ENOMEM, PAT_EHIP.
 */
int pat_plan_create(pat_plan** out, const pat_desc* desc, const float* c0, const float* rho0,
                    const float* alpha0_db, const double* sensor_pos, void* stream);

/*
 * pat_desc_check -- the host-side checks of pat_plan_create, without a device.
 *
 * Runs the descriptor validation, the stability bound of the scheme and the
 * construction of the linear-interpolation sensor operator (section III,
 * M w) on the host only: no HIP call is made, so it can run where no GPU is
 * present.
 *
 *  desc        descriptor as for pat_plan_create.
 *  lossy       non-zero when the plan will be given alpha0_db (checks
 *              alpha_power).
 *  sensor_pos  host, n_sensors*ndim doubles, as for pat_plan_create.
 *  c_max       largest sound speed of the medium [m/s]; > 0 also checks the
 *              stability bound c_max dt / min dx <= 1/sqrt(ndim) with the
 *              dt the plan would use; <= 0 skips that check.
 *
 * Returns PAT_OK, PAT_EINVAL (descriptor, NULL sensor_pos, sensor outside
 * the grid or not finite) or PAT_EUNSTABLE.
 */
int pat_desc_check(const pat_desc* desc, int32_t lossy, const double* sensor_pos, double c_max);

/* Release a plan and its device memory (NULL is accepted). */
void pat_plan_destroy(pat_plan* plan);

/* Copy the derived quantities of `plan` into *info (host). */
int pat_plan_info(const pat_plan* plan, pat_info* info);

/*
 * pat_forward -- the forward operator H of section III: data = H p0.
 *
 * Runs the k-space scheme for nt-1 steps from p(0) = p0, u(0) = 0
 * (equation initial) and samples the pressure at the sensors by linear
 * interpolation at every step, t = 0 included.  With PAT_SMOOTH_P0 the
 * scheme starts from S p0 instead (S: the flag's window filter).
 *
 *  p0    device, N floats (initial pressure, the image x).
 *  data  device, nt*n_sensors floats, written as data[n][s].
 */
int pat_forward(pat_plan* plan, const float* p0, float* data, void* stream);

/*
 * pat_adjoint -- the adjoint H^* = P^* M^* of section III as the exact
 * transpose of pat_forward: for every p0 and h,
 *   <pat_forward(p0), h> = <p0, pat_adjoint(h)>   (equation adj2),
 * up to float32 rounding.  It steps the time-reversed system of equations
 * moma/massa/statea with the data injected as a mass source and returns
 * the transposed initial condition (the discrete rho*(T)/rho0 of adjj),
 * filtered by S when the plan has PAT_SMOOTH_P0.
 *
 *  data  device, nt*n_sensors floats, [n][s].
 *  img   device, N floats, overwritten.
 */
int pat_adjoint(pat_plan* plan, const float* data, float* img, void* stream);

/*
 * pat_forward_range -- the forward operator in time segments, for
 * checkpointing: records samples n_begin .. n_end-1 into data[n][s] (the rows
 * of `data` outside that range are not touched).
 *
 *  n_begin == 0  starts from p0 (state_io is only written);
 *  n_begin  > 0  resumes from the snapshot in state_io, which must be the one
 *                written by an earlier call that ended at n_end == n_begin
 *                (p0 is then ignored and may be NULL).
 *  state_io      device, info.state_bytes bytes; on return it holds the
 *                scheme's state after sample n_end-1 (velocities, split
 *                densities and the x-spectrum of the pressure).
 *
 * Running [0, k) then [k, nt) gives bitwise the same data as pat_forward.
 */
int pat_forward_range(pat_plan* plan, const float* p0, float* data, int32_t n_begin, int32_t n_end,
                      void* state_io, void* stream);

/*
 * pat_adjoint_atd -- the paper's "adjoint-then-discretize" operator, for
 * comparison with the exact transpose pat_adjoint (which is what gradients
 * need).  The adjoint system of section III (eq. moma, massa, statea, with
 * eq. initial2 and the image rho*(T) / rho0 of eq. adjj) is discretized with
 * the forward's scheme and PML: leapfrog from p* = u* = rho* = 0, the
 * time-reversed data entering eq. massa as a mass source -- over step n the
 * density gains rho0 (W^T h[nt-1-n] + W^T h[nt-2-n]) / 2, split equally over
 * the axis components -- and p* = c0^2 rho* - rho0 L1[c0^2 tau (sigma / dt -
 * div u*)] - rho0 L2[c0^2 eta / rho0 rho*] (statea's order).  data: nt x ns
 * (device), img: N floats (device, overwritten).  For data that vanish at
 * the first and the last sample it agrees with pat_adjoint to rounding in a
 * homogeneous lossless or absorption-only medium without PML, and converges
 * to it at first order in dt in a heterogeneous one; the end samples enter
 * differently (the t = 0 sample with the trapezoid's half weight), and the
 * dispersion term and data taken inside the PML give differences that do
 * not vanish with dt.  nt = 1 gives a zero image.
 * The plan's state is clobbered as by pat_forward.
 */
int pat_adjoint_atd(pat_plan* plan, const float* data, float* img, void* stream);

/*
 * Batched execution of many plans (uneven sizes and nt allowed: instances
 * retire when their own time axis ends).  Each pass of the scheme runs as one
 * launch over a work table that holds the tiles of every active instance; the
 * time loop is captured into HIP graphs of `chunk` steps and replayed.
 * The plans must outlive the batch; a batch is used by one stream at a time.
 *
 *  pat_batch_create   plans: host array of nb plan pointers; chunk >= 1
 *                     (0 selects the default, 64).  All plans must have the
 *                     same ndim.
 *  pat_batch_forward  p0[i], data[i]: host arrays of nb device pointers.
 *  pat_batch_adjoint  data[i], img[i]: host arrays of nb device pointers.
 *
 * Results equal pat_forward / pat_adjoint per instance bitwise.
 */
int pat_batch_create(pat_batch** out, pat_plan* const* plans, int32_t nb, int32_t chunk);
/*
 * pat_batch_create_ex  as pat_batch_create, with the grouping explicit: the
 *   instances of one size class (same grid, nt and physics) are split into
 *   `parts` equal groups (0: the default, 2), each launched as its own work
 *   tables, and the groups run on `lanes` streams (0: one per group; with
 *   fewer streams than groups, the groups are placed heaviest first, by grid
 *   points x time steps, on the least-loaded stream).  Groups on different
 *   streams overlap on the GPU.  The streams come from a per-device pool
 *   that every batch shares (created by the first batch, two at a time, and
 *   kept until the process ends), so batches created later do not add
 *   hardware-queue mappings of their own; the work of batches called on
 *   different caller streams may interleave on them.
 *   Fusion (default; flags PAT_BATCH_NO_FUSE turns it off): 2D size classes
 *   whose axes are 128, 256 or 512 points long, with the same physics and
 *   nt >= 2, share their launches -- part k of each such class joins fused
 *   group k, whose every pass is one launch over the tiles of all its
 *   instances.  The group's time loop has as many steps as its longest
 *   instance (max nt - 1); an instance with S = nt - 1 steps runs its step
 *   floor(n S / span) at the loop steps n where that value advances, so
 *   each of its steps runs once and in order, spread evenly over the loop.
 *   Short classes then ride in the launches of the long ones instead of
 *   queueing short launches of their own beside them.
 *   Staggered start (default; PAT_BATCH_NO_STAGGER turns it off): with
 *   several groups, the groups at odd positions start their time loop once
 *   the first group has finished one pass, so that concurrent groups tend
 *   to pair a column pass (arithmetic-bound) with a row pass (memory-bound).
 *   pat_batch_create(out, plans, nb, chunk) is pat_batch_create_ex(out,
 *   plans, nb, chunk, 0, 0, 0).  parts = 1, lanes = 1 runs one launch per
 *   pass and group, one launch at a time.  PAT_EINVAL for unknown flags.
 */
int pat_batch_create_ex(pat_batch** out, pat_plan* const* plans, int32_t nb, int32_t chunk, int32_t parts,
                        int32_t lanes, uint32_t flags);
void pat_batch_destroy(pat_batch* batch);
int pat_batch_forward(pat_batch* batch, const float* const* p0, float* const* data, void* stream);
int pat_batch_adjoint(pat_batch* batch, const float* const* data, float* const* img, void* stream);

/*
 * pat_forward_batched / pat_adjoint_batched -- H and H^T (section III) of
 * many plans in one call: plans, p0 / data and data / img are host arrays of
 * nb plan and device pointers, as for pat_batch_forward / pat_batch_adjoint.
 * The first call with a given list of plans (same pointers, same order)
 * builds a batch with the default settings (pat_batch_create_ex(..., 0, 0,
 * 0, 0)) and keeps it for later calls with that list; destroying any of its
 * plans frees it.  Results equal pat_forward / pat_adjoint per instance
 * bitwise.  A list is used by one stream at a time, and a plan by one list
 * at a time.  PAT_EINVAL for NULL arrays or entries, nb < 1, or plans of
 * different ndim.
 */
int pat_forward_batched(pat_plan* const* plans, int32_t nb, const float* const* p0, float* const* data,
                        void* stream);
int pat_adjoint_batched(pat_plan* const* plans, int32_t nb, const float* const* data, float* const* img,
                        void* stream);

/*
 * Tile-shape autotuner of the batched executor: how many columns of the
 * column FFTs inside the k-space derivative and fractional-Laplacian
 * operators (section Forward Problem, lossless and lossy media) one
 * workgroup transforms, and whether a workgroup takes one or both fields
 * of a two-field pass.  For every column pass of the batch that has several
 * compiled variants (multiplier passes over one or two fields per launch
 * with columns of 128, 256 or 512 points: 16, 8 or 4 columns per
 * workgroup; 2D passes applying one multiplier per field: one or two fields
 * per workgroup), each variant is launched reps times on the batch's own
 * device buffers and timed with HIP events.  A batch of several groups
 * then runs its groups at the same time, where a variant that wins alone can
 * lose (a wide workgroup needs a whole CU's worth of LDS), so a second phase
 * times width policies in context: each policy (width 8 with one field per
 * workgroup; the fastest variant; the fastest of width <= 8; of width <= 4;
 * of width 8) is applied to every tuned pass and timed on a short concurrent
 * run of forward steps of all groups (the longest time axis 4 x chunk steps,
 * the others in proportion), the policies taking turns over three rounds,
 * the best run of each counting.  The first policy is kept unless another
 * runs at least 0.5 % faster; the policy kept is used from then on.
 * Results stay bitwise equal to
 * pat_forward / pat_adjoint: a variant only changes how columns and fields
 * are grouped into workgroups.
 *
 *  pat_batch_autotune  reps >= 1 timed launches per candidate.  Waits for the
 *                      batch and `stream` to be idle, runs on `stream`,
 *                      returns after the timing; clobbers the batch's
 *                      internal state buffers (never the caller's arrays) and
 *                      drops its captured graphs (re-captured on next use).
 *  pat_tuning_report   JSON array, one object per tuned pass: class shape
 *                      n, nt, lossy, instances, direction (0 forward, 1 adjoint), pass
 *                      index, mode, nfield, axis_len, candidates
 *                      [{tile, fpb, us}] (fpb: fields per workgroup), the
 *                      chosen tile and fpb, and for a batch of several groups
 *                      the chosen width policy and the microseconds of each
 *                      policy timed ("policy", "policy_us").  Writes at most cap bytes
 *                      including a terminating NUL into buf (buf may be NULL
 *                      when cap is 0) and the full length without the NUL to
 *                      *needed.  Empty array "[]" before any autotune.
 */
int pat_batch_autotune(pat_batch* batch, int32_t reps, void* stream);
int pat_tuning_report(const pat_batch* batch, char* buf, size_t cap, size_t* needed);

/*
 * pat_batch_time_pass  diagnostics: `reps` back-to-back launches of pass
 *   `pass` of direction dir (0 forward, 1 adjoint; the pass order of one
 *   time step) over every class of the batch with grid width nx (0: every
 *   class), one class at a time, each burst timed with HIP events on
 *   `stream` after one untimed launch.  Writes the mean microseconds per
 *   launch and the mean algorithmic bytes per launch (the full-grid arrays
 *   the pass must read and write, float32).  The launches run a generic time
 *   step on whatever the batch's state holds and clobber it, like
 *   pat_batch_autotune.  PAT_EINVAL when no class matches, the pass index
 *   is out of range, or the pass reads the caller's arrays (the first pass
 *   of the adjoint, which scatters the data).
 */
int pat_batch_time_pass(pat_batch* batch, int32_t dir, int32_t pass, int32_t nx, int32_t reps, void* stream,
                        double* us_per_launch, double* bytes_per_launch);

/*
 * pat_batch_set_tile  applies a stored choice (as reported above) without
 * timing: every class of grid n (nx, ny, nz; nz = 1 in 2D) with nt time
 * samples and physics `lossy` (0/1), direction dir, pass index `pass`, tile
 * width `tile` and fields per workgroup (tile 0 with 1 restores the
 * default).  Returns PAT_EINVAL when no class matches, the pass is not a
 * column pass or the variant is not compiled for it.  Drops the matching
 * classes' captured graphs.
 */
int pat_batch_set_tile(pat_batch* batch, const int32_t n[3], int32_t nt, int32_t lossy, int32_t dir, int32_t pass,
                       int32_t tile, int32_t fields_per_block);

/*
 * pat_tv_prox -- the proximal map of equation proxmal for
 * g = lambda_eff * TV + indicator(x >= lower), section IV:
 *   x = argmin  lambda_eff * TV_iso(x) + 1/2 ||x - z||^2   s.t. x >= lower,
 * by n_iter iterations of the fast gradient projection on the dual field of
 * Beck and Teboulle (the dual approach the paper uses), with forward
 * differences, Neumann boundary and dual step 1/(4 d lambda_eff).
 * lambda_eff = 0 returns max(z, lower) (the coarse-level projection).
 *
 *  ndim, n     grid (2 or 3 axes, any sizes >= 1, physical order x, y, z).
 *  z, x        device, N floats each (may not alias).
 *  lower       device, N floats, or NULL for the bound 0.
 *  work        device scratch of at least pat_tv_prox_work_bytes(ndim, n) bytes.
 */
size_t pat_tv_prox_work_bytes(int32_t ndim, const int32_t n[3]);

/*
 * pat_tv_prox_noalloc -- pat_tv_prox without a workspace argument and
 * without any allocation, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, arithmetic and result as pat_tv_prox (bitwise
 * equal), except that the FGP workspace is a fixed array in the library's
 * device memory instead of `work`:
 *   PAT_TV_PROX_NOALLOC_FLOATS floats (16 MiB) per device, held by every GPU
 *   the library runs on until the process ends.  (2 ndim + 1) * N must not
 *   exceed it (2D up to 838,860 points, e.g. 1024 x 512; 3D up to 599,186,
 *   e.g. 128 x 128 x 32); larger grids return PAT_ETOOBIG before anything
 *   is enqueued.
 * Every call on one GPU uses that GPU's one array: calls that overlap on a
 * GPU (two streams, or two host threads) race on it and give wrong results;
 * serialise them (one stream, or events).  The call clears the part of the
 * array it reads before writing it (a fill kernel, no hipMemset), so the
 * array's contents from an earlier call never matter.  Enqueues kernels
 * only: nothing synchronises, so the call can be captured into a graph.
 * Errors: PAT_EINVAL as pat_tv_prox, PAT_ETOOBIG, PAT_EHIP.
 */
#define PAT_TV_PROX_NOALLOC_FLOATS (1L << 22)
int pat_tv_prox_noalloc(int32_t ndim, const int32_t n[3], const float* z, float* x, double lambda_eff,
                        int32_t n_iter, const float* lower, void* stream);
int pat_tv_prox(int32_t ndim, const int32_t n[3], const float* z, float* x, double lambda_eff,
                int32_t n_iter, const float* lower, void* work, size_t work_bytes, void* stream);
/*
 * pat_tv_prox_batched -- pat_tv_prox for `count` images of one ndim at once
 *   (the prox step of many reconstructions in one iteration): every FGP
 *   iteration is one launch over all the images (24 per launch) instead of
 *   one per image.  n: host array count x 3; z, x, work: host arrays of
 *   count device pointers; lambda_eff, work_bytes: host arrays of count;
 *   lower: NULL or a host array of count device pointers (each may be NULL);
 *   n_iter common.  Each image's result equals pat_tv_prox's bitwise.
 *   Everything is validated before anything is enqueued.
 */
int pat_tv_prox_batched(int32_t count, int32_t ndim, const int32_t* n, const float* const* z, float* const* x,
                        const double* lambda_eff, int32_t n_iter, const float* const* lower, void* const* work,
                        const size_t* work_bytes, void* stream);

/*
 * pat_restrict / pat_prolong -- the transfer operators I_h^{h-1} and
 * I_{h-1}^h of section V (which the paper leaves undefined): the coarse grid
 * is cell-centred over 2^d blocks of fine points;
 *   restrict: coarse[I] = 2^-d * sum_{delta in {0,1}^d} fine[2I + delta]
 *   prolong:  fine[i]   = coarse[floor(i/2)]   (= 2^d * restrict^T)
 * n_fine / n_coarse: per-axis sizes (n_fine even).  Arrays are device floats.
 */
int pat_restrict(int32_t ndim, const int32_t n_fine[3], const float* fine, float* coarse, void* stream);
int pat_prolong(int32_t ndim, const int32_t n_coarse[3], const float* coarse, float* fine, void* stream);

/*
 * pat_dot_f64 -- sum_i a[i]*b[i] of float32 device arrays accumulated in
 * float64 with a fixed reduction order (deterministic), for the objective
 * 1/2 ||Hx - p||^2 and the norms of the multi-grid decision rule (sections
 * IV, V).  Synchronises `stream` and writes the result to *out_host.
 * b == a gives the squared norm.  n may be 0 (result 0).
 * Scratch: 4 KB of device memory per (device, stream), allocated by the
 * first reduction on that stream (this call, pat_residual_f64 or
 * pat_tv_smooth) and kept until the process ends; reductions on different
 * streams, or from different host threads on different streams, may run
 * concurrently.
 */
int pat_dot_f64(const float* a, const float* b, int64_t n, double* out_host, void* stream);

/*
 * pat_residual_f64 -- r = a - b written to device `r` (float32) and
 * 1/2 ||a - b||^2 accumulated in float64 (deterministic), in one pass.
 * Synchronises `stream`; *half_sq_host receives the value.  Scratch as
 * pat_dot_f64.
 */
int pat_residual_f64(const float* a, const float* b, float* r, int64_t n, double* half_sq_host,
                     void* stream);

/*
 * pat_residual_f64_batched -- the residuals of `count` pairs at once, with
 * nothing returned to the host and no synchronisation: the gradient-step
 * residuals H_i x_i - p_i of a batch of problems (section IV, eq. Six) and
 * their objective, left on the device for the adjoint that follows.
 *   count      1 .. 4096 pairs.
 *   a, b, r    host arrays of `count` device pointers: r_i = a_i - b_i
 *              (float32, n[i] elements each; r_i may alias a_i or b_i).
 *   n          host array of `count` element counts (>= 0; pointers may be
 *              NULL where n[i] = 0).
 *   work_dev   device scratch of pat_residual_batched_work_bytes(count)
 *              bytes, owned by the caller; calls that overlap on the GPU
 *              need their own.
 *   out_dev    device, count + 1 doubles: out_dev[i] = 1/2 ||a_i - b_i||^2,
 *              accumulated in float64 with pat_residual_f64's fixed
 *              partition (equal to that call's value bitwise), and
 *              out_dev[count] = their sum in index order.
 * Returns PAT_EINVAL for a bad count, a NULL array or a negative count.
 */
size_t pat_residual_batched_work_bytes(int32_t count);
int pat_residual_f64_batched(int32_t count, const float* const* a, const float* const* b, float* const* r,
                             const int64_t* n, double* work_dev, double* out_dev, void* stream);

/*
 * Operators of the two-level iteration (section V, Alg. FISTAMG).
 *
 * pat_tv_smooth -- the smoothed TV of equation Thirty-two,
 *   J_rho(x) = sum_j sqrt(|D x|_j^2 + rho^2) - rho,
 * D x the forward differences of pat_tv_prox (zero across each axis' last
 * face), and its gradient D^T (D x / sqrt(|D x|^2 + rho^2)), the TV term of
 * equation Twentyone.  rho = 0 gives the isotropic TV (the gradient then
 * takes 0 where D x = 0).
 *   ndim, n    grid (2 or 3 axes, physical order x, y, z).
 *   x          device, N floats.
 *   grad       device, N floats, or NULL: grad += scale * grad J_rho(x)
 *              (may not alias x).
 *   value_host host double, or NULL: J_rho(x), accumulated in float64 with a
 *              fixed partition (deterministic); the call then synchronizes
 *              `stream`.  At least one of grad, value_host.
 *
 * pat_restrict_lower -- the restricted bound constraint of equation
 *   constraint: lower[I] = (R y)[I] - min over the 2^d block of I of
 *   (y - l), so that y + P(x_c - R y) >= l for every coarse x_c >= lower
 *   (R, P as in pat_restrict / pat_prolong).  fine_lower: the fine level's
 *   bound l (N_fine floats, device), or NULL for l = 0 (the target level's
 *   nonnegativity); a bound at an intermediate level arises with more than
 *   two levels.  n_fine as in pat_restrict.
 *
 * pat_axpby -- out = a x + b y over n floats (device; out may alias x or y):
 *   the extrapolation and correction steps of Alg. FISTA / FISTAMG.
 * pat_project -- out = max(x, lower) over n floats, lower NULL meaning 0:
 *   the coarse level's proximal map, a projection (section V-E).
 */
int pat_tv_smooth(int32_t ndim, const int32_t n[3], const float* x, double rho, double scale, float* grad,
                  double* value_host, void* stream);
int pat_restrict_lower(int32_t ndim, const int32_t n_fine[3], const float* fine, const float* fine_lower,
                       float* lower, void* stream);
int pat_axpby(int64_t n, double a, const float* x, double b, const float* y, float* out, void* stream);
int pat_project(int64_t n, const float* x, const float* lower, float* out, void* stream);

/*
 * pat_plan_sync -- wait for `plan`'s work on `stream` and report deferred
 * device errors: PAT_ENONFINITE if PAT_CHECK_FINITE was set and a non-finite
 * pressure value was produced since the last sync (the flag is then cleared).
 */
int pat_plan_sync(pat_plan* plan, void* stream);

/*
 * Diagnostics: HIP-event timing of one pass of the time step.
 *
 * pat_timing_begin selects pass `pass_index` (0-based position in the step's
 * launch sequence) of direction 0 (forward) or 1 (adjoint), for grids with
 * row length nx (0: any); every later eager launch of that pass -- by
 * pat_forward, pat_adjoint, pat_forward_range, or the eager steps of a batch
 * (all of them with chunk = 1, else the nt-1 mod chunk steps run before the
 * graph-captured chunks) -- is bracketed by HIP events on its stream.  pat_timing_end waits for those events and returns their summed
 * duration [ms], the number of launches and the algorithmic bytes they moved
 * (full-grid float32 arrays each pass must read and write, per grid point,
 * times the points the launch covers).  Not thread-safe against concurrent
 * begin/end calls; launches captured into graphs are not timed.
 *
 * Forward lossy 2D sequence: 0 gradient (column), 1 velocity (row),
 * 2 divergence (column), 3 density (row), 4 absorption (column),
 * 5 equation of state + sensors (row).  Adjoint lossy 2D: 0 transposed state
 * (row), 1 absorption (column), 2 density (row), 3 gradient (column),
 * 4 velocity (row), 5 divergence sum (column).
 */
int pat_timing_begin(int32_t direction, int32_t pass_index, int32_t nx);
int pat_timing_end(double* total_ms, int64_t* launches, double* alg_bytes);

/* Static description of a return code. */
const char* pat_strerror(int code);

/*
 * pat_diag_sync_costs -- diagnostic: what one pass boundary costs in each
 * launch structure the batched executor could use (its per-pass launches
 * rest on this comparison).  On the current device, with a grid of
 * blocks_per_cu x (compute units) blocks of 256 threads each doing
 * floats_per_block floats of streaming read-modify-write:
 *   *us_grid_barrier   time per iteration of one cooperative launch whose
 *                      blocks repeat (work, grid-wide barrier) iters times,
 *                      the barrier being HIP's cooperative-groups grid sync;
 *   *us_atomic_barrier the same with a hand-written barrier (one atomic add
 *                      per block and a generation word); every wait is
 *                      bounded, and a wait that gives up yields -1;
 *   *us_stream_launch  time per launch of iters back-to-back launches;
 *   *us_graph_launch   the same launches replayed from a captured graph.
 * Synchronous.  Allocates and frees its own buffer, stream and graph.
 * Errors: PAT_EINVAL (blocks_per_cu above what can be co-resident, bad
 * sizes, NULL outputs), PAT_ENOSYS (no cooperative launch), PAT_EHIP.
 */
int pat_diag_sync_costs(int32_t blocks_per_cu, int32_t floats_per_block, int32_t iters, double* us_grid_barrier,
                        double* us_atomic_barrier, double* us_stream_launch, double* us_graph_launch);

#ifdef __cplusplus
}
#endif
#endif /* PAT_H */
