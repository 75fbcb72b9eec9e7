/*
 * rrlbm.h -- C-ABI of the MI355X (gfx950) recursive-regularized lattice
 * Boltzmann library (librrlbm.so).
 *
 * Method: Coreixas, Wissocq, Puigt, Boussuge, Sagaut, "Recursive
 * regularization step for high-order lattice Boltzmann methods".  One time
 * step is the explicit stream-and-collide scheme of Sec. III.A, with the
 * regularized collision of Eq. (RegularizedCollision) / Eq. (GenRegCollision)
 * at a single relaxation time: the non-equilibrium populations are rebuilt
 * from Hermite coefficients, a1^(2) by projection (Eq. a12Proj) and the higher
 * orders by the recursive formula (Malaspinas' isothermal form,
 * Eq. MalaspinasRecursiveRelation; the thermal extension,
 * Eq. RecursiveRelation_ThermalCase, with a1^(3) rebuilt through
 * Eq. TempGradLBM as App. C describes).  Lattices are those of Table I.
 *
 * Conventions shared by every entry point
 *   - Grids are periodic, nx by ny nodes, lattice units (dx = dt = 1).
 *   - Velocities are integers in canonical order: ascending c_y, then
 *     ascending c_x (lbm_lattice_velocities lists them).
 *   - Field arrays (rho, ux, uy, theta, vorticity) are FP64, row-major [y][x],
 *     nx*ny elements.  Population arrays exchanged with the caller are FP64,
 *     [i][y][x], Q*nx*ny elements.
 *   - "device" pointers are HIP device allocations (e.g. torch tensors on
 *     cuda:0); "host" pointers are ordinary memory.  The library never frees
 *     caller memory.
 *   - Every launch goes on the HIP stream given to lbm_init (a hipStream_t
 *     passed as void*; NULL is the default stream).  Calls are asynchronous
 *     unless stated otherwise.
 *   - Return value: 0 on success or a negative LBM_E* code; the calling
 *     thread's message is then available from lbm_last_error().
 *
 * Storage (population precision)
 *   LBM_STORE_FP64 (default) keeps the plain populations f_i in double and does
 *   all arithmetic in double.  LBM_STORE_FP32 / LBM_STORE_BF16 keep the
 *   weight-shifted populations g_i = f_i - w_i in float / bfloat16 and do all
 *   arithmetic in float.  LBM_STORE_MOMENTS (recursive regularization only)
 *   keeps, per node, the six values (rho, u_x, u_y, a1^(2)_xx, a1^(2)_xy,
 *   a1^(2)_yy) of the pre-collision populations in double: with the
 *   recursion the post-collision populations are a function of these alone
 *   (Eq. GenRegCollision, Eq. MalaspinasRecursiveRelation), so a step
 *   rebuilds each pulled population from its source node's moments.  With
 *   LBM_THERMAL (D2V37, App. C) the collision reads the populations only
 *   through their raw moments of order <= 3, and the state is the eleven
 *   values they give before rank 4: rho, u_x, u_y, sig = (theta - 1) c_s^2,
 *   a1^(2)_xx, a1^(2)_xy, a1^(2)_yy, a1^(3)_xxx, a1^(3)_xxy, a1^(3)_xyy,
 *   a1^(3)_yyy (planes in that order).
 *   The sequence of states equals that of LBM_STORE_FP64 up to rounding.
 *   LBM_STORE_FP32 | LBM_MATH_FP64 keeps the float storage of g_i and does
 *   the collision in double, so each value is rounded to float once per step
 *   (at the store); batches take it, the closure does not.
 *
 * Scheme (population storage only)
 *   By default a step gathers from one buffer into the other (f_a, f_b
 *   alternate).  LBM_SCHEME_AA keeps the state in f_a alone and updates it in
 *   place (the AA pattern; 2D and 3D contexts): after an even number of
 *   steps the post-collision value f_i(x) sits in plane opp(i) at x (opp(i):
 *   the velocity -c_i), after an odd number in plane i at x + c_i
 *   (periodic); a step from an even count reads plane opp(i) at x - c_i and
 *   writes plane i at x + c_i, one from an odd count reads and writes node
 *   x's own planes.  Each node's update reads and then writes the same
 *   slots, so steps are race-free.  The states (and what lbm_populations,
 *   lbm_moments, lbm_moments_3d and the checkpoints give) are those of the
 *   two-buffer scheme bit for bit; a checkpoint holds f_a as it sits, so it
 *   loads only into an LBM_SCHEME_AA context.  It halves the state memory
 *   and the working set, which the 256 MiB memory-side cache then serves
 *   better: on D2V37 FP64 it is 32% faster at 768^2 and 6% at 1024^2, on
 *   D2V17 FP64 14% at 2048^2, on D3Q19 and D3Q27 13-15% and on D3V39 9% at
 *   128^3; it is level with the two-buffer step at D2V37 FP64 2048^2
 *   (1.2 GB), 9% slower at D3Q103 128^3 and 7-20% slower on D3Q19, D3Q27
 *   and D3V39 at 256^3.
 *   Not with LBM_STORE_MOMENTS, batches or the closure.
 *
 * Environment (read when a context is created; none changes any result)
 *   RRLBM_CACHE_POLICY=0/1/2  forces the cache policy of the step: 0 ordinary
 *     loads and non-temporal stores, 1 ordinary loads and stores with the tile
 *     order reversed every other step, 2 non-temporal loads and ordinary
 *     stores.  By default the policy follows the size of one state buffer
 *     (1 up to 128 MiB, 2 from 256 to 320 MiB, 0 otherwise; 3D: RR and BGK).
 *     With LBM_SCHEME_AA: 1 ordinary stores, 0 non-temporal stores, 2
 *     non-temporal stores in the steps that write a node's own slots and
 *     ordinary ones in the others; the tile order is reversed every other
 *     step with 1 and 2 in 2D and with every policy in 3D.  The default is 1
 *     at every size in 2D, and in 3D 0 for buffers above 512 MiB up to 2 GiB
 *     and 1 otherwise.
 *   RRLBM_XCD_REMAP=0  keeps the hardware's round-robin order of blocks over
 *     the 8 XCDs instead of giving each XCD a contiguous band of tiles.
 *   RRLBM_BATCH_SPLIT=1/2  (read by lbm_batch_create) gives each lattice of a
 *     batch its own work list and persistent kernel, recorded as concurrent
 *     graph branches (1) or one after another (2); by default one kernel walks
 *     a single mixed list.
 */
#ifndef RRLBM_H
#define RRLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

/* Lattices (Table I). */
#define LBM_D2Q9 0  /* E^9_{2,5},  c_s^2 = 1/3, basis 1,x,y,xx,xy,yy,xxy,xyy,xxyy */
#define LBM_D2V17 1 /* E^17_{2,7}, all Hermite tensors of rank <= 3           */
#define LBM_D2V37 2 /* E^37_{2,9}, all Hermite tensors of rank <= 4           */
/* 3D lattices (Table II); isothermal, FP64 (or FP32 with FP64 arithmetic) populations, lbm_*_3d entry points. */
#define LBM_D3Q19 3 /* E^19_{3,5}, c_s^2 = 1/3, ranks <= 2 and the six xxy-type rank-3 tensors */
#define LBM_D3Q27 4 /* E^27_{3,5}, c_s^2 = 1/3, the 27 products with each exponent <= 2 */
#define LBM_D3V39 5 /* E^39_{3,7}, c_s^2 = 2/3, all Hermite tensors of rank <= 3 */
#define LBM_D3Q103 6 /* E^103_{3,9}, c_s = 1/1.19697977..., all Hermite tensors of rank <= 4 */

/* Flags for lbm_init (bitwise OR). */
#define LBM_THERMAL 0x1u        /* thermal/compressible form; D2V37 only          */
#define LBM_STORE_FP32 0x2u     /* store f - w in float, float arithmetic          */
#define LBM_STORE_BF16 0x4u     /* store f - w in bfloat16, float arithmetic       */
#define LBM_STORE_MOMENTS 0x8u  /* store the collision's moments in double; RR     */
#define LBM_COLL_PR 0x10u       /* projection-based regularization (Sec. II.E)     */
#define LBM_COLL_BGK 0x20u      /* BGK collision (Sec. III.A)                      */
#define LBM_EQ_INIT_ORDER2 0x100u /* initial f^(0) truncated at Hermite order 2    */
#define LBM_A13_PROJECTED 0x200u  /* thermal RR: keep the projected a1^(3)         */
#define LBM_MATH_FP64 0x400u      /* with LBM_STORE_FP32: double arithmetic        */
#define LBM_SCHEME_AA 0x800u      /* one population buffer, in-place steps          */

/* Error codes. */
#define LBM_OK 0
#define LBM_EINVAL (-1)   /* invalid argument (lattice, size, order, flags, NULL) */
#define LBM_ETAU (-2)     /* tau <= 1/2 or not finite                             */
#define LBM_EDEVICE (-3)  /* a HIP call failed                                    */
#define LBM_ENOMEM (-4)   /* the context could not allocate its scratch           */

/* Lattice constants (Tables I and II).  Any output pointer may be NULL.
 * q: number of velocities; reach: largest velocity component; n_eq: highest
 * Hermite rank of the basis (the order the equilibrium is expanded to);
 * cs2: c_s^2 in lattice units.  Returns LBM_EINVAL for an unknown lattice. */
int lbm_lattice_info(int lattice, int* q, int* reach, int* n_eq, double* cs2);

/* Velocities and weights in canonical order; host arrays of q entries each
 * (any may be NULL). */
int lbm_lattice_velocities(int lattice, int* cx, int* cy, double* w);

/* Elements (of the storage type) one state buffer must hold for an nx by ny
 * grid with the given LBM_STORE_* flags (other flag bits are ignored):
 * q * nx * (ny rounded up to a multiple of 4) for populations, the library's
 * row-tiled layout; 6 * nx * ny doubles for LBM_STORE_MOMENTS (six planes
 * [m][y][x]).  Negative on error. */
int64_t lbm_buffer_elems(int lattice, int nx, int ny, uint32_t flags);

/* Creates a context and writes the initial state.
 *   lattice    LBM_D2Q9, LBM_D2V17 or LBM_D2V37.
 *   nx, ny     grid size; each must be >= the lattice reach and
 *              lbm_buffer_elems() must stay below 2^31.
 *   tau        discrete relaxation time (tau-bar of Sec. III.A, > 1/2):
 *              nu = c_s^2 theta (tau - 1/2).
 *   reg_order  regularization order N, 2 <= N <= n_eq; the non-equilibrium
 *              part keeps Hermite ranks 2..N of the basis while the
 *              equilibrium always uses the full basis.  Ignored for BGK.
 *   flags      LBM_* flags above.  LBM_THERMAL requires LBM_D2V37.
 *   f_a, f_b   two device buffers of lbm_buffer_elems() elements of the
 *              storage type (double, float or bfloat16), caller-owned; they
 *              must stay valid until lbm_destroy.  With LBM_SCHEME_AA only
 *              f_a is used and f_b must be NULL.
 *   rho,ux,uy  device FP64 fields of the initial state.
 *   theta      device FP64 field of theta = T/T_0 (thermal), or NULL (= 1).
 *   grad       device FP64 array [4][y][x] of the velocity gradients
 *              (du_x/dx, du_x/dy, du_y/dx, du_y/dy) in lattice units, or NULL.
 *              When given (isothermal only, else LBM_EINVAL) the initial
 *              state is f^(0) + f^(1) (Sec. III.B): f^(1) expands
 *              a1^(2) = -rho c_s^2 tau (grad u + grad u^T) and the recursive
 *              a1^(3), a1^(4) over the same Hermite terms as f^(0).
 *   noise      device FP64 array [i][y][x] or NULL; the initial populations are
 *              f^(0)(rho, u, theta) [+ f^(1)] + noise_amp * w_i * noise.
 *   stream     hipStream_t for every launch of this context.
 * The buffer then holds the post-collision populations of step 0.  *out is
 * set only on success. */
int lbm_init(lbm_ctx** out, int lattice, int nx, int ny, double tau, int reg_order, uint32_t flags,
             void* f_a, void* f_b, const double* rho, const double* ux, const double* uy,
             const double* theta, const double* grad, const double* noise, double noise_amp, void* stream);

/* Advances nsteps (>= 0) time steps: each is one fused launch that gathers
 * f_i(x - c_i) (periodic pull), regularizes, relaxes and stores (in place
 * with LBM_SCHEME_AA).  Returns
 * LBM_EDEVICE if a launch fails.  A blow-up is not an error (lbm_moments
 * counts non-finite nodes). */
int lbm_step(lbm_ctx* ctx, int nsteps);

/* Number of steps taken since lbm_init. */
int64_t lbm_step_count(const lbm_ctx* ctx);

/* Relaxation times of the rank-3 and rank-4 non-equilibrium coefficients
 * (Eq. GenRegCollision with one time per Hermite order, the MRT form of
 * Sec. II.C; rank 2 keeps the tau of lbm_init).  Both default to tau.  In
 * the thermal form tau3 sets the thermal diffusivity c_s^2 theta (tau3 - 1/2),
 * so Pr = (tau - 1/2) / (tau3 - 1/2).  On 3D contexts tau4 relaxes every
 * rank >= 4 (D3Q27 reaches rank 6).  Applies from the next step; ranks
 * above the regularization order stay equilibrium.  LBM_EINVAL for a NULL
 * context or BGK, LBM_ETAU unless both are finite and > 1/2. */
int lbm_set_relaxation(lbm_ctx* ctx, double tau3, double tau4);

/* Macroscopic fields of the current step (rho, u and theta are collision
 * invariants, so they are the fields before and after the collision).
 * rho, ux, uy, theta, vort: device FP64 fields or NULL.  vort is
 * d(uy)/dx - d(ux)/dy from the periodic fourth-order centred difference.
 * sums: host array of LBM_NSUMS doubles or NULL; when given the call
 * synchronizes the stream and fills, over all nodes,
 *   [0] sum rho          [1] sum rho ux        [2] sum rho uy
 *   [3] sum rho E = sum_i f_i |c_i|^2 / 2      [4] sum |u|^2   [5] sum |u|^4
 *   [6] sum omega^2      [7] sum omega^4       [8] non-finite nodes
 *   [9] sum theta */
#define LBM_NSUMS 10
int lbm_moments(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* theta, double* vort,
                double* sums);

/* Allocation-free lbm_moments, for callers that cannot allocate memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments and results (bit for bit) as lbm_moments, which
 * allocates device and pinned scratch on its first call; this variant
 * allocates nothing and uses instead a device array the library holds on
 * every GPU it runs on until the process ends (LBM_NOALLOC_MAX_NODES / 256 *
 * 10 + 10 doubles, about 5 MiB).  Limits:
 *   - nx * ny <= LBM_NOALLOC_MAX_NODES (LBM_EINVAL beyond);
 *   - ux and uy are required whenever vort or sums is (the vorticity reads
 *     them); rho, theta, vort may be NULL (that field is not written);
 *   - calls that overlap on one GPU (other streams, other threads) share that
 *     array and race: serialize them;
 *   - with sums = NULL the call only launches kernels on the context's
 *     stream; with sums it synchronizes that stream.
 * 2D contexts only (LBM_EINVAL for a 3D one). */
#define LBM_NOALLOC_MAX_NODES (1 << 24)
int lbm_moments_noalloc(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* theta, double* vort,
                        double* sums);

/* Copies the current post-collision populations into the device FP64 array
 * f_out[i][y][x] (shifted storage is converted back to f = g + w). */
int lbm_populations(lbm_ctx* ctx, double* f_out);

/* ---- Checkpoints ---------------------------------------------------------
 * The state of the explicit scheme of Sec. III.A between two steps is the
 * post-collision population field (or, with LBM_STORE_MOMENTS, the moments it
 * is built from) together with the step counter, which also keys the BF16
 * stochastic rounding.  A checkpoint holds both, plus the relaxation times of
 * lbm_set_relaxation: a 64-byte header (magic "RRLBMCK1", lattice, nx, ny,
 * nz, flags, step count, tau, tau3, tau4) followed by the current state buffer
 * exactly as it sits in device memory (storage type, library layout).  So
 * k steps, lbm_save, lbm_load into a fresh context and n - k more steps give
 * bit for bit the state of n steps.  Works for 2D and 3D contexts. */
#define LBM_CHECKPOINT_HEADER_BYTES 64

/* Bytes of a checkpoint of ctx (header + one state buffer); negative on error. */
int64_t lbm_checkpoint_bytes(const lbm_ctx* ctx);

/* Writes the checkpoint of the current step to dst, host or device memory
 * owned by the caller, of dst_bytes >= lbm_checkpoint_bytes(ctx) bytes.
 * Synchronizes the context's stream.  LBM_EINVAL for a NULL pointer or a
 * short buffer, LBM_EDEVICE if a copy fails. */
int lbm_save(lbm_ctx* ctx, void* dst, int64_t dst_bytes);

/* Restores a checkpoint (host or device memory, src_bytes long) into ctx,
 * which must have been created with the same lattice, grid, tau and flags as
 * the context that wrote it (LBM_EINVAL otherwise, and for a short or foreign
 * buffer; ctx is then unchanged).  The state goes to the first of ctx's
 * buffers; the step count and tau3, tau4 are those of the checkpoint.
 * Synchronizes the context's stream. */
int lbm_load(lbm_ctx* ctx, const void* src, int64_t src_bytes);

/* Frees the context's own scratch (not the caller's buffers).  NULL is a no-op. */
void lbm_destroy(lbm_ctx* ctx);

/* Message describing the last error on the calling thread ("" if none). */
const char* lbm_last_error(void);

/* ---- 3D lattices (Table II) ---------------------------------------------
 * Isothermal recursive regularization (the 3D forms of the recursion in
 * App. C, Eq. MalaspinasRecursiveRelation at theta = 1), projection-based
 * regularization or BGK on D3Q19, D3Q27, D3V39 and D3Q103, FP64 populations, or
 * (LBM_STORE_FP32 | LBM_MATH_FP64) the 2D form's weight-shifted floats
 * g = f - w with every operation in double, rounded once per value at the
 * store.  Grids
 * are periodic nx by ny by nz; fields are [z][y][x] (nx*ny*nz doubles) and
 * populations exchanged with the caller are [i][z][y][x].  The layout is the
 * 2D one over the ny*nz rows r = z*ny + y.  A 3D context works with
 * lbm_step, lbm_step_count, lbm_set_relaxation, lbm_populations and
 * lbm_destroy; lbm_moments, batches and the closure reject it. */

/* Velocities (ascending c_z, then c_y, then c_x) and weights of a 3D lattice;
 * host arrays of q entries (any may be NULL).  LBM_EINVAL for a 2D id. */
int lbm_lattice_velocities_3d(int lattice, int* cx, int* cy, int* cz, double* w);

/* Elements (double, or float with LBM_STORE_FP32) one state buffer holds:
 * q * nx * (ny*nz rounded up to a multiple of 4).  flags must carry no
 * LBM_STORE_BF16 or LBM_STORE_MOMENTS bit.  Negative on error. */
int64_t lbm_buffer_elems_3d(int lattice, int nx, int ny, int nz, uint32_t flags);

/* Creates a 3D context and writes the initial state, the equilibrium of
 * (rho, u) over the lattice's basis (LBM_EQ_INIT_ORDER2: ranks <= 2) plus
 * noise_amp * w_i * noise[i][z][y][x], collided once (the kept state is
 * post-collision, as in 2D).
 *   lattice    LBM_D3Q19, LBM_D3Q27, LBM_D3V39 or LBM_D3Q103.
 *   nx, ny, nz each >= the lattice reach; lbm_buffer_elems_3d() < 2^31.
 *   tau        discrete relaxation time (> 1/2), nu = c_s^2 (tau - 1/2).
 *   reg_order  2 <= N <= n_eq (3, 6, 3, 4); ignored with LBM_COLL_BGK.
 *   flags      LBM_COLL_PR, LBM_COLL_BGK, LBM_EQ_INIT_ORDER2, LBM_SCHEME_AA,
 *              and LBM_STORE_FP32 together with LBM_MATH_FP64, only.
 *   f_a, f_b   two distinct device buffers of lbm_buffer_elems_3d() elements,
 *              owned by the caller for the context's lifetime; with
 *              LBM_SCHEME_AA (the single-buffer scheme of the 2D contexts,
 *              with c_i and opp(i) in 3D) only f_a, and f_b must be NULL.
 *   rho, ux, uy, uz  device fields; noise device [q][z][y][x] or NULL.
 * Same errors as lbm_init. */
int lbm_init_3d(lbm_ctx** out, int lattice, int nx, int ny, int nz, double tau, int reg_order, uint32_t flags,
                void* f_a, void* f_b, const double* rho, const double* ux, const double* uy, const double* uz,
                const double* noise, double noise_amp, void* stream);

/* Fields of the current step of a 3D context: rho, ux, uy, uz device FP64
 * arrays or NULL.  sums: host array of LBM_NSUMS_3D doubles or NULL; when
 * given the call synchronizes the stream and fills, over all nodes,
 *   [0] sum rho  [1] sum rho ux  [2] sum rho uy  [3] sum rho uz
 *   [4] sum_i f_i |c_i|^2 / 2    [5] sum |u|^2   [6] sum |u|^4
 *   [7] non-finite nodes
 * LBM_EINVAL for a 2D context. */
#define LBM_NSUMS_3D 8
int lbm_moments_3d(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* uz, double* sums);

/* ---- Batched stepping ----------------------------------------------------
 * Many independent contexts (any lattice and grid size) advanced together:
 * one persistent launch per step walks a work list of tiles that spans
 * every member, and lbm_batch_step replays a HIP graph holding two such
 * launches (the two buffer parities).  Members keep working with
 * lbm_moments / lbm_populations / lbm_destroy; the batch never owns them. */
typedef struct lbm_batch lbm_batch;

/* ctxs: host array of n (1..4096) contexts from lbm_init.  All members must
 * use the same storage flag, the recursive-regularized isothermal collision
 * (no LBM_COLL_PR, LBM_COLL_BGK or LBM_THERMAL) and the same stream (the
 * batch launches on it).  tile_x (64, 128, 256, 512 or 1024) is the width of
 * one work item in nodes (items of 64 and 128 are four rows high, wider ones
 * one row); blocks_per_cu (1..16) sets the persistent grid to that many
 * blocks per compute unit.  Captures the graph; *out is set on success. */
int lbm_batch_create(lbm_batch** out, lbm_ctx* const* ctxs, int n, int tile_x, int blocks_per_cu);

/* Advances every member by nsteps (>= 0).  If a member was stepped on its
 * own since the last call, its buffer parity is re-read first (a small
 * host-to-device copy outside the graph). */
int lbm_batch_step(lbm_batch* b, int nsteps);

/* Autotuner: times every (tile_x, blocks_per_cu) candidate over
 * steps_per_trial graph-replayed steps (members are advanced by those
 * steps), keeps the fastest and recaptures the graph.  report (host, may be
 * NULL) receives one line per candidate, "tile_x blocks_per_cu ms_per_step",
 * truncated to report_len bytes.  Synchronizes the stream. */
int lbm_batch_autotune(lbm_batch* b, int steps_per_trial, char* report, int report_len);

/* Current (tile_x, blocks_per_cu) of the batch (either pointer may be NULL). */
int lbm_batch_config(const lbm_batch* b, int* tile_x, int* blocks_per_cu);

/* Releases the graph and the work list (not the members).  NULL is a no-op. */
void lbm_batch_destroy(lbm_batch* b);

/* ---- Learned closure (not part of the paper's method) --------------------
 * A per-node perceptron 8 -> 64 -> 64 -> 9 (tanh-form GELU), evaluated on the
 * bfloat16 matrix cores with float32 accumulation, predicts a residual added
 * to the isothermal recursive a1^(3), a1^(4) of the D2V37 collision; mass and
 * momentum are unaffected by construction.  Coefficients use the scaling
 * ahat = (1 - 1/(2 tau)) a1, comparable across grids under acoustic scaling.
 *
 * Parameter vector: LBM_MLP_NPARAM float32, row-major [in][out] matrices
 *   W1 8x64 | b1 64 | W2 64x64 | b2 64 | W3 64x16 | b3 16  (outputs 9..15 unused, keep 0)
 * Normalisation block: LBM_MLP_NNORM float32
 *   in_mean[8] in_std[8] in_lo[8] in_hi[8] out_mean[16] out_std[16] out_lo[16] out_hi[16]
 * Inputs 0..6: rho - 1, ux, uy, |u|^2 / c_s^2 (local Mach number squared),
 * ahat_xx, ahat_xy, ahat_yy; input 7 is the constant 1 (not normalised).  Outputs
 * 0..8: the ahat^(3..4) residual, order 30, 21, 12, 03, 40, 31, 22, 13, 04
 * (x and y exponents).  lo/hi bound the training data in normalised units:
 * a node whose normalised input or output leaves them keeps the plain
 * recursion (the fallback). */
#define LBM_MLP_NPARAM 5776
#define LBM_MLP_NNORM 96

/* Training samples from a fine run, restricted to a grid coarser by
 * `factor` (1..8, dividing nx and ny): for every coarse node the block
 * average of the fine nodes' rho, rho u and ahat^(2..4) (ahat computed from
 * the fine post-collision populations with the fine tau), then
 *   x[c][0..7] = raw inputs (input 7 = 1), and
 *   r[c][0..15] = ahat^(3..4) minus the recursion applied to the averaged
 *                 (rho, u, ahat^(2)) (entries 9..15 = 0).
 * Every input is tau-independent, so the coarse run's tau is not needed.
 * fine must be an isothermal RR D2V37 context; x, r are device float32
 * arrays of (nx/factor)*(ny/factor) rows.
 * Coarse node c = X + Y * (nx/factor).  Runs on fine's stream. */
int lbm_closure_samples(lbm_ctx* fine, int factor, float* x, float* r);

/* Normalisation block of n samples (x as above, r as above): mean and
 * standard deviation of inputs 0..6 and outputs 0..8 (a zero deviation is
 * replaced by 1), and their min/max in normalised units; device `norm` of
 * LBM_MLP_NNORM floats.  Synchronizes `stream`. */
int lbm_mlp_stats(const float* x, const float* r, int64_t n, float* norm, void* stream);

/* In place: x[.][0..6] and r[.][0..8] normalised with `norm`, x[.][7] = 1. */
int lbm_mlp_normalize(float* x, float* r, int64_t n, const float* norm, void* stream);

/* Training state of one network: theta (device, LBM_MLP_NPARAM float32,
 * caller-owned, updated in place) plus the library's Adam moments, gradient,
 * matrix-core weight fragments and per-wave partial sums for batches of up
 * to max_batch samples. */
typedef struct lbm_mlp lbm_mlp;
int lbm_mlp_create(lbm_mlp** out, float* theta, int64_t max_batch, void* stream);

/* Network outputs y[n][16] (normalised; 9..15 = padding) for normalised
 * inputs x[n][8], with the current theta. */
int lbm_mlp_forward(lbm_mlp* m, const float* x, int64_t n, float* y);

/* Mean squared error over `batch` samples (rows idx[0..batch) of x, t, or
 * rows 0..batch when idx is NULL; t[.][0..8] normalised targets) and its
 * gradient.  grad (device, LBM_MLP_NPARAM) may be NULL; loss (host) may be
 * NULL, otherwise the call synchronizes.  lr > 0 also applies one Adam step
 * (beta1 0.9, beta2 0.999, eps 1e-8) to theta; lr = 0 leaves theta alone. */
int lbm_mlp_step(lbm_mlp* m, const float* x, const float* t, const int* idx, int64_t batch, float lr,
                 float* grad, double* loss);

void lbm_mlp_destroy(lbm_mlp* m);

/* Attaches a trained closure to an isothermal RR D2V37 context (FP64 or FP32
 * storage): theta and norm are device float32 arrays (copied; the caller may
 * free them).  Later lbm_step calls run the fused closure kernel.  theta =
 * NULL detaches.  Resets the fallback counter. */
int lbm_closure_set(lbm_ctx* ctx, const float* theta, const float* norm);

/* Nodes (summed over steps) that kept the plain recursion since
 * lbm_closure_set.  Synchronizes the stream. */
int lbm_closure_fallbacks(lbm_ctx* ctx, int64_t* count);

#ifdef __cplusplus
}
#endif

#endif /* RRLBM_H */
