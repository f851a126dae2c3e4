/*
 * ssd.h -- C ABI of the sliding-mesh spectral difference (SSD) library.
 *
 * The library evaluates the per-stage residual of the 2-D compressible
 * Euler / Navier-Stokes equations on quadrilateral meshes whose rotating
 * and stationary zones meet at a circular sliding interface, and advances
 * it with an explicit SSP Runge-Kutta method, on one AMD Instinct GPU
 * (Zhang & Liang, arXiv:1503.02198).
 *
 * Conventions shared by every entry point
 *  - Every function returns ssd_status: 0 on success, a negative code on
 *    failure.  No C++ exception crosses the ABI.  After a failure
 *    ssd_last_error() returns a message for the calling thread.
 *  - A failing call has no side effect on the mesh handle.
 *  - Device arrays (q, r, work) are caller-owned device pointers of 32-bit
 *    floats; the library never frees or retains them beyond the call.
 *  - State layout (cell-blocked): value (v, j, i) of element e is Q[v], v =
 *    0..3 the conservative variables rho, rho u, rho v, E (Sec. 2.1, eq. Q),
 *    at solution point (X_i, X_j); its plane is p = (v N + j) N + i.
 *    Elements go in blocks of 64 consecutive elements, the last block holding
 *    the remaining n_elem mod 64; block b = e / 64 stores plane after plane,
 *    each plane as a row of its nb = min(64, n_elem - 64 b) elements:
 *      index(e, p) = 64 * 4 N^2 * b + p * nb + (e - 64 b).
 *    state_len = 4 N^2 n_elem floats (no padding).  For full blocks this is
 *    q[b][v][j][i][e mod 64].
 *    The state holds the physical Q at the solution points; since the
 *    Jacobian of a fixed or rigidly rotating cell does not change in time,
 *    d(|J| Q)/dt = |J| dQ/dt and the residual is returned as dQ/dt.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls that enqueue work return before it completes.
 *  - One handle is used by one host thread and one stream at a time.
 */
#ifndef SSD_H
#define SSD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssd_mesh ssd_mesh;

typedef enum {
  SSD_OK = 0,
  SSD_ERR_INVALID_ARG = -1, /* null pointer, out-of-range size or value   */
  SSD_ERR_MESH = -2,        /* the mesh description is inconsistent        */
  SSD_ERR_STATE = -3,       /* call out of order (e.g. stale mortars)      */
  SSD_ERR_DEVICE = -4,      /* a HIP runtime call failed                   */
  SSD_ERR_NOMEM = -5,       /* device or host allocation failed            */
  SSD_ERR_NUMERIC = -6      /* a stage produced rho <= 0, p <= 0 or NaN    */
} ssd_status;

/* Face tags of ssd_mesh_desc.face_kind. */
enum {
  SSD_FACE_INTERIOR = 0,        /* conforming neighbour, Rusanov flux (Sec. 3.1)   */
  SSD_FACE_PERIODIC = 1,        /* conforming neighbour across a periodic cut      */
  SSD_FACE_SLIDING = 2,         /* on the circular rotor/stator interface (Sec. 3.2) */
  SSD_FACE_WALL_ISOTHERMAL = 3, /* no-slip wall at T_wall moving with its zone      */
  SSD_FACE_WALL_SLIP = 4,       /* impermeable slip wall moving with its zone       */
  SSD_FACE_FARFIELD = 5         /* Rusanov flux against the far-field state         */
};

/* Element maps of ssd_mesh_desc.elem_geom (Sec. 3.1: 4-node linear cells,
 * 12-node cubic cells along curved boundaries). */
enum { SSD_GEOM_LINEAR = 0, SSD_GEOM_CUBIC = 1 };

/* Explicit SSP Runge-Kutta time integrators (Sec. 3: an explicit SSP
 * scheme; Sec. 4: the five-stage fourth-order one for every test case).
 *  SSD_RK3_SSP    three-stage third order, Shu-Osher form, stage times
 *                 t, t + dt, t + dt/2; work: 2 state_len floats.
 *  SSD_RK54_SSP   five-stage fourth order (SSPRK(5,4), the published
 *                 coefficients of Spiteri and Ruuth), each stage at the
 *                 time of its stage value; work: 3 state_len floats. */
typedef enum { SSD_RK3_SSP = 0, SSD_RK54_SSP = 1 } ssd_rk;

/*
 * Mesh and case description.  All arrays are host memory, read during
 * ssd_create_mesh and copied; the caller may free them afterwards.
 *
 *  N          solution points per direction = order of accuracy, 2..6
 *             (Sec. 3.1: N Chebyshev-Gauss SPs, N+1 FPs per direction).
 *  n_elem     number of elements; one handle needs its state array
 *             (16 N^2 n_elem bytes) and trace array (64 N n_elem bytes)
 *             below 4 GiB (n_elem < 16.7 million at N = 4); with mu > 0
 *             the gradient arrays, twice those sizes, as well.
 *  elem_xy    [n_elem][12][2] node coordinates, counter-clockwise around
 *             the reference square [0,1]^2: (0,0) (1/3,0) (2/3,0) (1,0)
 *             (1,1/3) (1,2/3) (1,1) (2/3,1) (1/3,1) (0,1) (0,2/3) (0,1/3).
 *             Linear cells use only nodes 0, 3, 6, 9.
 *  elem_geom  [n_elem] SSD_GEOM_LINEAR (bilinear) or SSD_GEOM_CUBIC
 *             (12-node cubic serendipity).
 *  elem_zone  [n_elem] 0 stationary, 1 rotating about rot_center.
 *  nbr_elem, nbr_face, face_kind   [n_elem][4] for the local faces
 *             0: eta=0, 1: xi=1, 2: eta=1, 3: xi=0.  INTERIOR and PERIODIC
 *             faces name their neighbour element and its local face; other
 *             kinds set nbr_elem = -1.
 *  rot_center, iface_radius   centre of rotation and radius of the sliding
 *             circle (ignored without SLIDING faces).
 *  omega, theta0   rotation rate of zone 1 and its angle at t = 0; the
 *             rotor angle used by ssd_rk_step is theta0 + omega t.
 *  gamma, gas_R, mu, prandtl   gas properties; mu = 0 selects the Euler
 *             equations (Sec. 2.1), constant mu otherwise.
 *  T_wall     temperature of isothermal walls.
 *  farfield   rho, u, v, p of far-field faces.
 */
typedef struct {
  int32_t N;
  int32_t n_elem;
  const double *elem_xy;
  const int32_t *elem_geom;
  const int32_t *elem_zone;
  const int32_t *nbr_elem;
  const int32_t *nbr_face;
  const int32_t *face_kind;
  double rot_center[2];
  double iface_radius;
  double omega;
  double theta0;
  double gamma;
  double gas_R;
  double mu;
  double prandtl;
  double T_wall;
  double farfield[4];
} ssd_mesh_desc;

typedef struct {
  int32_t N;          /* solution points per direction                  */
  int32_t n_elem;     /* elements                                       */
  int32_t K;          /* sliding-interface faces on the larger side (0: none) */
  int32_t n_cubic;    /* cubic elements                                 */
  int32_t viscous;    /* 1 when mu > 0                                  */
  int32_t device;     /* HIP device the handle lives on                 */
  int64_t state_len;  /* floats in one state array: 4 N^2 n_elem        */
  int64_t work_len;   /* floats ssd_rk_step needs in `work` for any scheme: 3 state_len */
} ssd_info;

/*
 * Validates the description, builds FP64 geometry and operator tables and
 * uploads them to `device`.  Fails with SSD_ERR_MESH when a neighbour link is
 * not mutual, a face tag is unknown, |J| <= 0 at a solution or flux point,
 * or the faces of a side of the sliding interface do not tile the circle.
 *
 * Sliding interface: when both sides hold K faces that are uniform arcs
 * (Sec. 3.2), each face meets two mortars placed by (m, delta).  Otherwise
 * (general rings: different face counts, non-uniform arcs; the extension
 * named at the end of Sec. 3.2) the sides' face end points, merged in
 * angular order at each rotor angle, bound the mortars, and a face meets as
 * many as fall on it.  *out receives the handle.
 */
ssd_status ssd_create_mesh(const ssd_mesh_desc *desc, int device, ssd_mesh **out);

/* Frees every device and host resource of the handle (synchronises). */
ssd_status ssd_destroy_mesh(ssd_mesh *m);

/* Sizes of the handle; synchronous, no device work. */
ssd_status ssd_query(const ssd_mesh *m, ssd_info *info);

/*
 * Sets the rotor angle theta and rate omega used by the next
 * ssd_mortar_rebuild and ssd_residual (Sec. 2.2: grid velocity
 * omega x r, coordinates rotated analytically).  Marks the mortars stale.
 */
ssd_status ssd_set_rotation(ssd_mesh *m, double theta, double omega);

/*
 * Rebuilds the sliding-interface connectivity and projection matrices for
 * the current angle on the device in FP64 (Sec. 3.2: each face meets two
 * mortars whose offset o and scale s follow the rotor, eq. xz; the
 * face-to-mortar matrices M^-1 S and mortar-to-face matrices s M^-1 S^T of
 * eqs. prjQ2 and prjF2).  Enqueued on `stream`; a no-op without an
 * interface.
 */
ssd_status ssd_mortar_rebuild(ssd_mesh *m, void *stream);

/*
 * r = dQ/dt for state q at the current angle and rate: interpolation to
 * the flux points (eq. Qt), transformed fluxes (eq. transform_relation)
 * with the ALE terms, common fluxes on conforming, boundary and sliding
 * faces (Sec. 3.1, Sec. 3.2), and the flux-polynomial derivative (eqs. Ft,
 * Gt).  q and r: device float arrays of state_len, must not overlap.
 * SSD_ERR_STATE if the mortars are stale (ssd_set_rotation without a later
 * ssd_mortar_rebuild).
 */
ssd_status ssd_residual(ssd_mesh *m, const float *q, float *r, void *stream);

/*
 * One step of `scheme` (ssd_rk) from t to t + dt in place on q (device,
 * state_len floats), using `work` (device, at least the floats the scheme
 * needs, work_len covers all) as scratch.  Before each stage it sets the
 * angle theta0 + omega t_stage and rebuilds the mortars (Sec. 3.2: the
 * connectivity is updated at every Runge-Kutta stage).
 * SSD_ERR_INVALID_ARG for dt <= 0, a non-finite t or an unknown scheme;
 * work must not overlap q.
 */
ssd_status ssd_rk_step(ssd_mesh *m, float *q, float *work, double t, double dt, ssd_rk scheme,
                       void *stream);

/*
 * nsteps >= 1 consecutive steps of `scheme` from t (step n starts at t + n dt),
 * with the same effect as nsteps calls of ssd_rk_step.  The face traces the
 * last stage of a step leaves behind serve the first stage of the next one,
 * so the separate trace pass runs once per call instead of once per step.
 */
ssd_status ssd_rk_steps(ssd_mesh *m, float *q, float *work, double t, double dt, int32_t nsteps,
                        ssd_rk scheme, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * steps as ssd_rk_steps, with the work arrays taken from a fixed array of
 * SSD_SCRATCH_BYTES per GPU that the library holds until the process ends
 * (set up by ssd_create_mesh on its device).  The call allocates nothing.
 * Limits and sharing:
 *   - the scheme's work arrays (2 state_len floats for SSP-RK3, 3 for
 *     SSPRK54) must fit in SSD_SCRATCH_BYTES, else SSD_ERR_INVALID_ARG with
 *     no work enqueued;
 *   - kernel timing must be off (ssd_timing_enable(m, 0)), else
 *     SSD_ERR_STATE: the timers may create events;
 *   - every call on one GPU uses that GPU's one array, which keeps the
 *     last call's contents (nothing in it needs to start at zero): calls
 *     that overlap on one GPU (other streams, other threads, other meshes)
 *     race and must be serialised by the caller.
 */
#define SSD_SCRATCH_BYTES (64u << 20)
ssd_status ssd_rk_steps_noalloc(ssd_mesh *m, float *q, double t, double dt, int32_t nsteps,
                                ssd_rk scheme, void *stream);

/*
 * Synchronises `stream` and reports SSD_ERR_NUMERIC if any stage since the
 * last check produced a non-finite value, rho <= 0 or p <= 0; clears the
 * flag.
 */
ssd_status ssd_check(ssd_mesh *m, void *stream);

/* Message of the calling thread's last failure ("" if none). */
const char *ssd_last_error(void);

/*
 * Batches: many meshes of one device stepped together.  A batch groups its
 * meshes by (N, viscous); per RK stage every group runs one mortar launch,
 * (viscous) one gradient and one viscous-mortar launch, and one stage
 * launch, each with one block per item of a device table of (mesh, 64-cell
 * tile or interface chunk) pairs.  A mesh with general sliding rings (see
 * ssd_create_mesh) has its own mortar merge, flux and back-projection
 * launches inside its group's chain, its rotor angle likewise read from the
 * group's step counter.  Groups share no data, so each group's
 * whole chain of launches runs on one of up to SSD_BATCH_MAX_STREAMS
 * streams, forked from and joined back to the caller's stream.  On the
 * first call an autotuner picks, per group, the tile shape of the stage
 * launch (one or, for N <= 4, two 64-cell tiles per block: the faster by at
 * least 3 %, remembered for the process by (N, viscous, log2 of the
 * group's tile count) and reused by later batches), then times the stage of
 * the whole batch with 1, 2, ... streams (groups dealt to streams longest
 * first by their measured times) and keeps the most streams within 3 % of
 * the fastest (the trials are eager launches, whose per-stream fork and
 * join a replayed graph does not pay); every time is the median of 5
 * trials.  With
 * use_graph, one and two steps are captured as HIP graphs on the first call
 * for a scheme and replayed; the stage time is read from a device step
 * counter per group, so the graphs do not depend on t.
 *
 * The batch references the meshes: they must outlive it, and no other call
 * may use them while a batch call runs.  Calls on one batch must not
 * overlap.
 */
typedef struct ssd_batch ssd_batch;

#define SSD_BATCH_MAX_STREAMS 4

typedef struct {
  int32_t n_groups;     /* groups in the batch                                 */
  int32_t N;            /* solution points per direction of this group         */
  int32_t viscous;
  int32_t tiles;        /* 64-cell tiles over all meshes of the group          */
  int32_t stream;       /* stream index of the group's launches                */
  int32_t n_streams;    /* streams the batch uses (1..SSD_BATCH_MAX_STREAMS)   */
  int32_t tuned;        /* 1 once the autotuner has run                        */
  float stage_us;       /* the group's stage alone, as timed by the autotuner  */
  int32_t tiles_per_block;   /* 64-cell tiles per block of the stage launch */
  float stage_us_tpb[2];     /* the stage alone with 1 and 2 tiles per block
                                (0: not timed; the choice was known)        */
} ssd_batch_group;

/* n >= 1 distinct meshes, all on one device, none with a learned correction
 * attached (ssd_subgrid_attach): the batched stage has no correction input.
 * Errors: SSD_ERR_INVALID_ARG. */
ssd_status ssd_batch_create(ssd_mesh *const *meshes, int32_t n, ssd_batch **out);
ssd_status ssd_batch_destroy(ssd_batch *b);

/*
 * nsteps steps of `scheme` for every mesh c of the batch, mesh c from t[c]
 * with step dt[c], in place on q[c] (device, its state_len floats) with
 * work[c] (device, its work_len floats).  Same arithmetic as ssd_rk_steps
 * per mesh; the rotor angle is formed on the device from t[c] + (n + c_k)
 * dt[c], so results agree with ssd_rk_steps to rounding.  Host arrays q,
 * work, t, dt have one entry per mesh in creation order.  Afterwards each
 * mesh is at the rotor angle of t[c] + nsteps dt[c] with stale mortars, as
 * after ssd_rk_steps, with or without graphs.  A mesh that has had a learned
 * correction attached since the batch was created gives
 * SSD_ERR_INVALID_ARG, with no work enqueued.
 */
ssd_status ssd_batch_rk_steps(ssd_batch *b, float *const *q, float *const *work, const double *t,
                              const double *dt, int32_t nsteps, ssd_rk scheme, int32_t use_graph,
                              void *stream);

/* Shape of group `group` (0 <= group < n_groups). */
ssd_status ssd_batch_query(const ssd_batch *b, int32_t group, ssd_batch_group *info);

/*
 * Kernel timing.  ssd_timing_enable selects the kernel classes whose
 * launches are timed with HIP events on their stream: `classes` is a bit
 * mask, bit SSD_KERNEL_x for class x (SSD_TIMING_ALL: every class, 0: off).
 * The stage kernel's events are attached to its dispatch and record the
 * kernel's own start and end; the other classes are bracketed by two event
 * records in the stream, which adds a few microseconds per launch, so time
 * only the classes of interest in a throughput run.  Classes: the stage kernel
 * (residual or fused RK stage), the face-trace kernel, the mortar kernels
 * (the rebuild fused with the inviscid mortar, and with mu > 0 the viscous
 * mortar), the stand-alone mortar rebuild (ssd_mortar_rebuild), and the
 * gradient pass of viscous meshes.  ssd_timing_read synchronises and
 * returns the summed milliseconds and the launch count of one kernel class
 * (SSD_KERNEL_*) since the last reset; ssd_timing_reset clears them.
 */
enum { SSD_KERNEL_STAGE = 0, SSD_KERNEL_TRACES = 1, SSD_KERNEL_MORTAR = 2, SSD_KERNEL_REBUILD = 3,
       SSD_KERNEL_GRAD = 4, SSD_KERNEL_COUNT = 5 };
enum { SSD_TIMING_ALL = (1 << SSD_KERNEL_COUNT) - 1 };
ssd_status ssd_timing_enable(ssd_mesh *m, int classes);
ssd_status ssd_timing_reset(ssd_mesh *m);
ssd_status ssd_timing_read(ssd_mesh *m, int kernel, double *total_ms, int64_t *launches);
/* The same launches one by one: ms[i] (host, cap entries) receives the
 * duration of the i-th timed launch of class `kernel` since the last reset,
 * in launch order, for i < min(cap, launches); *launches receives their
 * count.  Synchronises the device.  Errors: SSD_ERR_INVALID_ARG for a bad
 * class, cap < 0, or a null ms with cap > 0. */
ssd_status ssd_timing_samples(ssd_mesh *m, int kernel, float *ms, int64_t cap, int64_t *launches);
/*
 * Measurement probe for the choice between vector ALUs and matrix cores
 * for the per-cell contractions of the flux-point method (Sec. 3.1 eqs. Qt,
 * Ft, Gt), on the stage kernel's data layout (64 cells per wave, one line
 * per wave): `reps` rounds of interpolation to the flux points of a line
 * (the mesh's N = 4 operator I), the pointwise flux q^2, and the derivative
 * back to the solution points (operator D), per cell and variable.
 * variant 0 runs them as fused multiply-adds per lane, variant 1 on
 * v_mfma_f32_16x16x4_f32 with 16 cells per matrix.  q and out (device) are
 * [4][4 lines][4 points][n_cells] floats, cell index fastest; n_cells is a
 * positive multiple of 64.  Not part of the method: its result is only
 * compared between the variants.  Errors: SSD_ERR_INVALID_ARG (mesh N != 4,
 * bad variant, n_cells or reps).
 */
ssd_status ssd_probe_contraction(ssd_mesh *m, int32_t variant, int32_t n_cells, int32_t reps,
                                 const float *q, float *out, void *stream);
/*
 * Measurement probe for the bandwidth ceiling of the stage kernel's state
 * traffic: c[i] = 0.75 a[i] + 0.25 b[i] for i < n, two arrays read and one
 * written, as an SSP-RK stage (Sec. 3.3) reads Q and Qn and writes the new
 * state.  variant 0: 16-byte accesses per lane, default cache policy;
 * 1: the same, non-temporal; 2: the stage kernel's own access, 4-byte
 * non-temporal buffer loads and stores per lane, 256 bytes per wave and
 * instruction.  a, b, c: device arrays of n floats on the mesh's device,
 * 16-byte aligned, c overlapping neither a nor b; n a positive multiple of
 * 1024 with 4 n < 2^32.  Asynchronous on `stream`.  Not part of the method.
 * Errors: SSD_ERR_INVALID_ARG (bad variant, n or null array).
 */
ssd_status ssd_probe_stream(ssd_mesh *m, int32_t variant, int64_t n, const float *a,
                            const float *b, float *c, void *stream);


/*
 * Learned per-element subgrid correction (an extension of the method; not
 * in the paper).  A coarse run of N = 2..4 solution points per direction
 * adds, in every SSP-RK3 stage, a correction C(Q) to dQ/dt: per element, a
 * small MLP maps the element's 4 N^2 solution-point values and its
 * neighbours' face traces (16 N values) to 4 N^2 corrections.  The network
 * is trained on fine runs of the solver: a nested fine mesh (every coarse
 * cell split 2 x 2 in its reference square) is restricted to the coarse
 * one, and the target is the restricted fine dQ/dt minus the coarse
 * residual of the restricted state.
 *
 * Network: xn = (x - mu_x) / sig_x, h1 = tanh(W1 xn + b1), h2 = tanh(W2 h1
 * + b2), yn = W3 h2 + b3, y = yn sig_y + mu_y; hidden width
 * SSD_MLP_HIDDEN.  Products run on the BF16 matrix cores (operands rounded
 * to bfloat16, FP32 accumulation); biases, tanh and the update are FP32.
 *
 * Feature layout of element e, n_in = 4 N^2 + 16 N values per row:
 *   [v N^2 + j N + i]            Q[v][j][i] of the element
 *   [4 N^2 + (f N + p) 4 + v]    variable v of the neighbour's trace at
 *                                point p of local face f (in the face's own
 *                                parameter order); boundary and sliding
 *                                faces use the element's own trace.
 * Outputs (n_out = 4 N^2 per row) are one element's values, index (v N + j) N + i.
 */
#define SSD_MLP_HIDDEN 64

typedef struct ssd_mlp ssd_mlp;

/* A network for meshes of N = 2..4 solution points per direction, on
 * `device`, all parameters zero and the normalisation the identity.
 * Errors: SSD_ERR_INVALID_ARG, SSD_ERR_NOMEM, SSD_ERR_DEVICE. */
ssd_status ssd_mlp_create(int32_t N, int32_t device, ssd_mlp **out);
ssd_status ssd_mlp_destroy(ssd_mlp *net);
/* n_in and n_out of the network. */
ssd_status ssd_mlp_dims(const ssd_mlp *net, int32_t *n_in, int32_t *n_out);

/*
 * Parameters as host FP32 arrays, row-major: W1 [H][n_in], b1 [H],
 * W2 [H][H], b2 [H], W3 [n_out][H], b3 [n_out] (H = SSD_MLP_HIDDEN).
 * Setting them also clears the optimiser state.  Both calls synchronise
 * the device.
 */
ssd_status ssd_mlp_set_params(ssd_mlp *net, const float *W1, const float *b1, const float *W2,
                              const float *b2, const float *W3, const float *b3);
ssd_status ssd_mlp_get_params(const ssd_mlp *net, float *W1, float *b1, float *W2, float *b2,
                              float *W3, float *b3);

/* Normalisation as host FP32 arrays mu_x, sig_x [n_in], mu_y, sig_y [n_out];
 * every sig > 0.  Errors: SSD_ERR_INVALID_ARG. */
ssd_status ssd_mlp_set_normalization(ssd_mlp *net, const float *mu_x, const float *sig_x,
                                     const float *mu_y, const float *sig_y);
/* Fits the normalisation to n >= 2 rows of X [n][n_in] and T [n][n_out]
 * (device): per-column mean and standard deviation, the deviation floored
 * at min_rel times the column's root mean square (min_rel >= 0); a column
 * that is zero throughout gets sig = 1.  Synchronises. */
ssd_status ssd_mlp_fit_normalization(ssd_mlp *net, const float *X, const float *T, int64_t n,
                                     float min_rel, void *stream);

/* Y [n][n_out] = the network of the rows X [n][n_in] (device, n >= 0). */
ssd_status ssd_mlp_forward(ssd_mlp *net, const float *X, int64_t n, float *Y, void *stream);

/*
 * Loss gradient of the minibatch of rows idx[0..batch) of X [n_rows][n_in]
 * and T [n_rows][n_out] (device; idx device int32, batch >= 1; an index
 * outside [0, n_rows) contributes nothing).  The loss is the mean
 * over the batch and the outputs of (yn - (t - mu_y) / sig_y)^2.  The
 * gradient goes to host arrays laid out as ssd_mlp_get_params, the loss to
 * *loss.  Parameters are not changed.  Synchronises.
 *
 * Input noise (noise > 0, training only): the normalised input i of
 * minibatch position s gets noise * eps added before the first layer, eps
 * = (2u - 1) sqrt(3) with u the top 24 bits (times 2^-24) of the SplitMix64
 * output of stream noise_seed at counter (step << 32) + s n_in + i, where
 * step is the number of Adam steps taken since the parameters were set,
 * plus one.
 */
ssd_status ssd_mlp_gradient(ssd_mlp *net, const float *X, const float *T, int64_t n_rows,
                            const int32_t *idx, int32_t batch, float noise, uint64_t noise_seed,
                            float *gW1, float *gb1, float *gW2, float *gb2, float *gW3, float *gb3,
                            double *loss, void *stream);
/*
 * One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * loss of the minibatch idx[0..batch).  The minibatch losses are summed on
 * the device; ssd_mlp_loss returns the sum and the number of steps since
 * the last call (and synchronises).
 */
ssd_status ssd_mlp_train_step(ssd_mlp *net, const float *X, const float *T, int64_t n_rows,
                              const int32_t *idx, int32_t batch, float lr, float noise,
                              uint64_t noise_seed, void *stream);
ssd_status ssd_mlp_loss(ssd_mlp *net, double *loss_sum, int64_t *steps);

/* Features of every element of state q (device, state layout) into the rows
 * X [E][n_in] (device). */
ssd_status ssd_subgrid_features(ssd_mesh *m, const float *q, float *X, void *stream);

/*
 * Restriction of a state qf of the nested fine mesh `fine` to its coarse
 * parent mesh `coarse`: the L2 projection, in each coarse cell's reference
 * square, of the fine piecewise polynomial onto the coarse polynomials,
 * at the coarse solution points.  children [E_coarse][4] (device int32):
 * the fine element of child (a, b) at index a + 2 b, child (a, b) covering
 * [a/2, (a+1)/2] x [b/2, (b+1)/2] of the parent's reference square.
 * qc is in the coarse state layout.  Supported (N coarse, N fine): (2, 2),
 * (2, 4), (2, 6), (3, 3), (3, 4), (3, 5), (3, 6), (4, 6).  The child table
 * is read back and checked (every entry in [0, E_fine)) before the launch,
 * so the call synchronises with the device.
 *
 * children = NULL: `fine` and `coarse` are the same mesh and qc is the L2
 * projection of qf onto the lower order of `coarse`, element by element
 * (N pairs with 2 <= N coarse < N fine <= 6).
 */
ssd_status ssd_restrict(const ssd_mesh *fine, const ssd_mesh *coarse, const int32_t *children,
                        const float *qf, float *qc, void *stream);
/* Training targets T [E_coarse][4 N^2] = restriction of Rf (a fine dQ/dt)
 * minus Rc (a coarse dQ/dt, state layout). */
ssd_status ssd_subgrid_targets(const ssd_mesh *fine, const ssd_mesh *coarse,
                               const int32_t *children, const float *Rf, const float *Rc, float *T,
                               void *stream);

/* Relaxation term of training targets taken along a corrected coarse run
 * (a posteriori training): T [E][4 N^2] (rows as in ssd_subgrid_targets)
 * += rate (q_ref - q), with q_ref (the restricted fine state) and q (the
 * coarse run's state) device arrays in the state layout of `coarse`.  With
 * T = restrict(Rf) - Rc(q) the target is the correction that also pulls q
 * back to q_ref at the given rate.  Errors: SSD_ERR_INVALID_ARG (null
 * array, non-finite rate). */
ssd_status ssd_subgrid_nudge(const ssd_mesh *coarse, const float *q_ref, const float *q, float rate,
                             float *T, void *stream);

/* Attaches `net` (same N and device) to mesh m with weight w (finite): from
 * then on ssd_rk_step(s) with SSD_RK3_SSP adds w C(Q) to dQ/dt in every
 * stage (other schemes return SSD_ERR_INVALID_ARG), C evaluated at each
 * stage's input, or, with per_step != 0, once per step at Q^n and held for
 * the step's three stages (a third of the network's cost).  net = NULL
 * detaches (plain SSD).  The network must outlive the attachment. */
ssd_status ssd_subgrid_attach(ssd_mesh *m, ssd_mlp *net, float w, int32_t per_step);

#ifdef __cplusplus
}
#endif

#endif /* SSD_H */
