/*
 * lb.h -- C ABI of the thread-safe regularized lattice Boltzmann library
 * (liblb.so) for AMD Instinct MI355X (gfx950).
 *
 * Method: Montessori et al., "Thread-safe lattice Boltzmann for
 * high-performance computing on GPUs".  One time step is
 *   (1) moments: rho, j = rho u, Pi^neq of every node from its populations
 *       (Section 4, moment snippet; Section 2, moment definitions);
 *   (2) fused streaming + collision: every population of every node is
 *       rebuilt from the moments of the node it streams from, by Hermite
 *       projection of the non-equilibrium part (Section 3, eq. LBexp, eq.
 *       pushLB, eq. hermite and the full stream-and-collide equation);
 *   (3) boundary conditions (Section 4), fused into (2).
 * Only one population set per species is allocated; the sweep (2) never
 * reads populations, so it updates them in place without races.
 *
 * Conventions
 *   - All entry points return an lb_status (0 = LB_OK, negative on error)
 *     unless stated otherwise.  No C++ exception crosses this interface.
 *   - Host arrays are FP64, structure-of-arrays, node index
 *     n = x + nx*(y + ny*z), x fastest.  D = 2 for D2Q9, 3 otherwise.
 *   - Velocity u has D*N entries (all x, then all y, then all z).
 *   - The non-equilibrium stress Pi^neq has D(D+1)/2 * N entries, ordered
 *     xx, yy, (zz), xy, (xz, yz).
 *   - A handle is not safe for concurrent calls from several threads;
 *     distinct handles may be used from different threads.
 *   - Population storage order on the device is internal; the ABI exposes
 *     moments only.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum lb_status {
  LB_OK = 0,
  LB_EINVAL = -1,       /* invalid argument or parameter combination */
  LB_ENOMEM = -2,       /* device or host allocation failed / buffer too small */
  LB_EUNSUPPORTED = -3, /* valid request this build does not implement */
  LB_EDEVICE = -4,      /* HIP runtime error (launch, copy, synchronisation) */
  LB_ENONFINITE = -5    /* non-finite value in input or in the evolved state */
};

/* Velocity sets (Section 2: the number of discrete velocities follows from
 * the lattice's dimension and isotropy); textbook weights, cs^2 = 1/3. */
enum lb_lattice { LB_D2Q9 = 9, LB_D3Q19 = 19, LB_D3Q27 = 27 };

/* Boundary condition of one axis, applied at both ends of the axis.
 * LB_BOUNCEBACK is halfway bounce-back: the wall sits half a lattice spacing
 * beyond the first and last node layer (Section 5.1 uses bounce-back walls). */
enum lb_boundary { LB_PERIODIC = 0, LB_BOUNCEBACK = 1 };

/* Population storage precision.  The *_S modes store f_a - t_a*rho0 (the
 * deviation from the rest state) in 16 bits with round-to-nearest-even; the
 * paper proposes half-precision population storage with single-precision
 * arithmetic as future work (Sections 6.1, 6.3, 7). */
enum lb_storage {
  LB_STORE_F64 = 0,   /* requires LB_COMPUTE_F64 */
  LB_STORE_F32 = 1,
  LB_STORE_F16S = 2,
  LB_STORE_BF16S = 3
};

/* Arithmetic precision of the kernels.  LB_COMPUTE_F64 requires
 * LB_STORE_F64; the 32-bit-compute modes keep their moments in FP32. */
enum lb_compute { LB_COMPUTE_F64 = 0, LB_COMPUTE_F32 = 1 };

/* Problem statement (Sections 2-3).  Fill with lb_params_default first.
 * struct_size is the size of the caller's struct, so the layout can grow:
 * the library accepts sizeof(lb_params) and the sizes of its earlier
 * versions, LB_PARAMS_SIZE_V1 (up to `compute`), LB_PARAMS_SIZE_V2 (up to
 * `wall_velocity`) and LB_PARAMS_SIZE_V3 (up to the near-contact fields);
 * fields beyond the caller's size take their defaults (zero wall velocity,
 * near-contact interactions off, moment arrays kept).  Any other size is
 * LB_EINVAL. */
typedef struct lb_params {
  size_t struct_size;     /* = sizeof(lb_params), or an earlier version's size */
  int32_t lattice;        /* enum lb_lattice */
  int32_t hermite_order;  /* 2, or 3 (D3Q27 only): order of the Hermite
                             expansion of equilibrium and non-equilibrium
                             (eq. hermite, truncated at n = 2 in the paper) */
  int64_t nx, ny, nz;     /* lattice nodes per axis; nz = 1 for D2Q9 */
  int32_t bc[3];          /* enum lb_boundary per axis x, y, z */
  int32_t species;        /* 1, or 2 for the colour-gradient model (Sec. 2.1) */
  double tau;             /* relaxation time, omega = 1/tau; tau > 1/2 */
  double rho0;            /* bulk density of the incompressible equilibrium
                             (eq. equil); > 0 */
  double force[3];        /* constant body-force density (Section 2 allows a
                             body force but gives no scheme): Guo's source
                             term, so each node's momentum gains F per step
                             and u = (j + F/2)/rho0 */
  double sigma;           /* colour-gradient surface tension (species = 2) */
  double beta;            /* recolouring parameter (species = 2), 0..1 */
  int32_t storage;        /* enum lb_storage */
  int32_t compute;        /* enum lb_compute */
  double wall_velocity[3][2][3];
                          /* velocity of the wall on the low ([a][0]) and high
                             ([a][1]) face of axis a (Section 5, lid-driven
                             cavity: the lid's motion enters through Bouzidi's
                             momentum correction, which at the halfway wall
                             is Ladd's): a link a leaving node x across a
                             wall comes back as
                               f_abar(x) = f^pc_a(x) - 2 t_a rho0 (c_a.u_w)/cs2,
                             summed over every wall it crosses (edges and
                             corners).  Only tangential components on
                             bounce-back axes, one species: LB_EINVAL for a
                             non-zero normal component or a velocity on a
                             periodic axis, LB_EUNSUPPORTED with two species.
                             Zero (the default) = resting walls. */
  /* Near-contact interactions between interfaces (Section 2.2; species = 2
   * only; the paper gives the mechanism but no constants, so these are
   * readings).  A bulk node x of the continuous phase, phi(x) < -1 +
   * nci_eps, samples phi at x + d c_a and x - d c_a (d = nci_reach) for
   * every pair of opposite lattice directions; when neither point is bulk,
   * both are flagged.  A flagged node with a defined phase gradient G
   * gets the body force nci_strength * rho_R * G/|G| in its collision (on
   * top of `force`), pushing each interface back into its own droplet.
   * lb_moments reports u = (j + force/2)/rho0 with the constant force only. */
  double nci_strength;    /* force constant A >= 0; 0 (default) = off */
  double nci_eps;         /* bulk threshold, 0 < eps < 2 (default 0.1) */
  int32_t nci_reach;      /* sampling distance d, 1..8 lattice spacings (default 1) */
  int32_t nci_reserved_;  /* 0 */
  /* Memory of the step (Section 4 counts the thread-safe method's arrays:
   * Q populations + M moments per node).  1 (default): the moment arrays
   * are allocated and both paths of lb_set_step_path are available.  0: the
   * handle holds the population set only (D3Q19 FP32: 19 arrays, 76 B per
   * node instead of 116) plus a bounded staging buffer for lb_init /
   * lb_moments, and every step is the fused step, which keeps the moments
   * in registers; the shape must have one (lb_set_step_path), else
   * LB_EUNSUPPORTED.  Such a handle refuses the two-sweep path, lb_sweep
   * and the batched entry points (LB_EUNSUPPORTED). */
  int32_t keep_moments;
  int32_t keep_moments_reserved_;  /* 0 */
} lb_params;

/* struct_size values of the earlier versions of lb_params. */
#define LB_PARAMS_SIZE_V1 ((size_t)offsetof(lb_params, wall_velocity))
#define LB_PARAMS_SIZE_V2 ((size_t)offsetof(lb_params, nci_strength))
#define LB_PARAMS_SIZE_V3 ((size_t)offsetof(lb_params, keep_moments))

typedef struct lb_handle lb_handle;

/* Fill *p with a valid default problem (D3Q19, 32^3, periodic, tau 0.6,
 * rho0 1, no force, one species, FP32 storage and compute, resting walls,
 * near-contact interactions off).  p != NULL. */
void lb_params_default(lb_params* p);

/* Exact number of device bytes lb_create needs for these parameters:
 * populations (species * Q arrays) + moments (M arrays) of npad nodes each
 * (with keep_moments 0, in place of the moments, a staging buffer of at most
 * 256 MiB), + npad bytes of near-contact flags when nci_strength > 0,
 * npad = px * ny * nz rounded up to the layout's block size, where the row
 * pitch px is nx rounded up to a multiple of the stream-collide sweep's
 * vector chunk (1 to 8 nodes; see lb_layout), each region 256-byte aligned,
 * + npad bytes of reference colours for two species, + 64 KiB of FP64
 * reduction scratch, + ny * nz + 3 32-bit progress words where the shape has
 * a fused step (Section 4 counts 15 arrays per node for D2Q9 and 29 for
 * D3Q19 in single precision).  Returns 0 for invalid parameters. */
size_t lb_required_bytes(const lb_params* p);

/* Validate parameters without touching the device. */
int lb_validate(const lb_params* p);

/* Create a simulation on the current HIP device: the single population set
 * per species and the moment arrays the method needs (Section 4 counts the
 * arrays per node; Section 3: no second population set), or with
 * keep_moments 0 the population set alone.
 *   dev_mem    device buffer of dev_bytes >= lb_required_bytes(p), 256-byte
 *              aligned, owned by the caller and outliving the handle; or
 *              NULL, in which case the library allocates (hipMalloc) and
 *              frees the memory itself.
 *   hip_stream hipStream_t to enqueue all work on (borrowed, may be NULL for
 *              the null stream).
 * LB_ENOMEM if dev_bytes is too small or the allocation fails, LB_EINVAL for
 * a misaligned dev_mem, LB_EUNSUPPORTED for keep_moments 0 where the device
 * cannot run this shape's fused step.  The populations are zero (rest
 * state) until lb_init. */
int lb_create(const lb_params* p, void* dev_mem, size_t dev_bytes, void* hip_stream,
              lb_handle** out);

/* Set the populations to the equilibrium of the given fields (the paper does
 * not state an initial condition; Pi^neq = 0 at start).
 *   rho[N], u[D*N] host FP64; phi[N] phase field in [-1, 1] for two species
 *   (rho_R = rho (1+phi)/2, rho_B = rho (1-phi)/2), NULL for one species.
 * Synchronous with respect to the host arrays.  Resets the step counter.
 * LB_ENONFINITE if any input is not finite. */
int lb_init(lb_handle* h, const double* rho, const double* u, const double* phi);

/* Enqueue nsteps >= 0 time steps (moments, then fused stream + collide with
 * boundaries) on the handle's stream and return without waiting.  Each
 * step runs either as the two sweeps of lb_sweep or, where the shape
 * allows it, as the fused step (lb_set_step_path), whose result is the
 * same bit for bit. */
int lb_step(lb_handle* h, int64_t nsteps);

/* Enqueue one half of a time step: which = 0 the moments sweep (reads the
 * populations, writes the moment arrays), which = 1 the fused
 * stream-collide sweep (reads the moment arrays only, rewrites every
 * population in place).  lb_step(h, 1) on the two-sweep path is
 * lb_sweep(h, 0) then lb_sweep(h, 1), and the fused step gives the same
 * bits; the step counter advances after which = 1.  For instrumentation
 * and for tests of the sweeps' data dependencies.  LB_EUNSUPPORTED for a
 * handle without moment arrays (keep_moments 0). */
int lb_sweep(lb_handle* h, int which);
/* (lb_init and lb_moments use the moment arrays as staging for their host
 * transfers: after them, run which = 0 before a which = 1 sweep.) */

/* Order in which the stream-collide sweep's wavefronts take their row
 * segments, for testing that the sweep's result does not depend on the
 * order its parallel work runs in (the thread-safety of Section 3): 0 the
 * natural order (default), 1 reversed, 2 a strided permutation that sends
 * neighbouring wavefronts to distant rows.  Results are bitwise the same
 * for every order.  Batched execution always uses the natural order.
 * LB_EINVAL for another value; LB_EUNSUPPORTED for orders 1 and 2 on a
 * domain of 2^31 or more row segments. */
int lb_set_sweep_order(lb_handle* h, int order);

/* Path of lb_step.  The two sweeps (Section 4's moments loop, then the
 * streaming + collision loop of eq. pushLB) pass every node's moments
 * through the moment arrays.  The fused step computes the same moments and
 * post-collision populations, with the same arithmetic, in one launch that
 * keeps the moments in registers: one wavefront per x-row and run of
 * z-planes, marching in z, which writes into a neighbouring row only after
 * that row's wavefront has read it (progress words in device memory), so
 * the in-place update stays thread-safe in the sense of Section 3.  It
 * moves Q populations in and out per node (152 B for D3Q19 FP32) instead
 * of Q + M each way.
 *   Shapes: one species, D3Q19 or D3Q27, FP32 / FP16 / BF16 storage with
 *   FP32 arithmetic, nx = 128, 256 or 512 (D3Q27: 128, 256); every tile
 *   must be resident at once (ny * z_tiles wavefronts), and the device
 *   must support cooperative launch.
 *   path: LB_PATH_AUTO (what lb_create sets: fused for D3Q19 where the
 *   shape allows it and its tiles fill at least half the device, else two
 *   sweeps; D3Q27 takes the fused step only when asked, its two sweeps
 *   being faster),
 *   LB_PATH_TWO_SWEEP, LB_PATH_FUSED.  z_tiles: runs of planes per row,
 *   0 to choose (at least 8 planes per run); ignored for two sweeps.
 * Waits for the handle's stream.  LB_EUNSUPPORTED if LB_PATH_FUSED cannot
 * run this shape or tiling (the path is then unchanged), LB_EINVAL for a
 * bad path or z_tiles > nz.  A fused step that waits past its bound gives
 * up (its result is invalid): the next lb_synchronize, lb_moments or
 * lb_set_step_path call returns LB_EDEVICE once.  The fused step is a
 * cooperative launch; a caller that captures lb_step into a HIP graph
 * should select the two-sweep path, whose launches are ordinary kernels
 * (the batched entry points always use them).  A handle without moment
 * arrays (keep_moments 0) has the fused path only: LB_PATH_AUTO and
 * LB_PATH_FUSED select it, LB_PATH_TWO_SWEEP is LB_EUNSUPPORTED. */
#define LB_PATH_AUTO 0
#define LB_PATH_TWO_SWEEP 1
#define LB_PATH_FUSED 2
int lb_set_step_path(lb_handle* h, int path, int64_t z_tiles);

/* The path lb_step takes (LB_PATH_TWO_SWEEP or LB_PATH_FUSED) and, for the
 * fused step, its runs of planes per row (0 for two sweeps). */
int lb_get_step_path(const lb_handle* h, int* path, int64_t* z_tiles);

/* Bound of every wait of the fused step, in polls of a neighbouring row's
 * progress word (default 2^22, seconds at worst); a wait that exhausts it
 * gives up (see lb_set_step_path).  For tests of that path: 0 makes every
 * wait that is not met at its first poll give up.  Applies to later steps.
 * LB_EINVAL for a negative bound or one above INT32_MAX. */
int lb_set_fused_wait_limit(lb_handle* h, int64_t polls);

/* Device layout of the handle's state, for tests and tools.  The population
 * region (species*Q arrays of the storage type: set 0 then set 1) starts at
 * byte pop_offset of the device buffer, the moment region (M arrays of the
 * compute type: drho, j, Pi^neq [, phi]) at moment_offset.  Node (x, y, z)
 * is storage node n = x + row_pitch * (y + ny * z), row_pitch >= nx (nx
 * rounded up so that the stream-collide sweep's vectors stay aligned; the
 * storage nodes x >= nx of a row are padding: their populations stay zero
 * and are never read into a lattice node).
 * Both regions are blocked structures of arrays over padded_nodes storage
 * nodes: with B = block_nodes (a power of two), element (a, n) of a region of
 * NA arrays is element (n / B) * NA * B + a * B + n % B of that region.
 * Populations are stored shifted (f_a - t_a rho0 for set 0).  The layout is
 * internal: it may change between versions, and only the moments are part
 * of the interface. */
int lb_layout(const lb_handle* h, size_t* pop_offset, size_t* moment_offset,
              int64_t* block_nodes, int64_t* padded_nodes, int64_t* row_pitch);

/* Wait for all work enqueued on the handle's stream. */
int lb_synchronize(lb_handle* h);

/* Rebind the handle to another stream (hipStream_t, borrowed; NULL = the
 * null stream): later calls enqueue their work there.  Nothing is
 * synchronized: work already enqueued on the old stream must be complete,
 * or ordered before the new stream's next work by the caller (an event),
 * before the handle is used again.  Lets a caller set a simulation up or
 * read it back on a stream of its own and step it in a batch on the
 * batch's stream.  Not while a call on the handle is in progress. */
int lb_set_stream(lb_handle* h, void* hip_stream);

/* Read the moments of the current populations (blocks until done): the
 * density, velocity and non-equilibrium stress of Section 2's moment
 * definitions (Pi^neq as in Section 4's moment computation), copied out to
 * the host.
 *   rho[N]      density (rho0 + deviation), or NULL
 *   u[D*N]      velocity u = (j + F/2)/rho0, or NULL
 *   pineq[K*N]  non-equilibrium stress, K = D(D+1)/2, or NULL
 *   phi[N]      phase field (two species only), or NULL
 *   conserved[6] FP64 device reductions over all nodes: total mass, total
 *               momentum j (3 components, z = 0 in 2D), red mass, blue mass
 *               (species 1: red mass = total, blue mass = 0), or NULL.
 * Moments are evaluated in the handle's compute precision and returned as
 * FP64.  Returns LB_ENONFINITE (after filling the outputs) if the reduced
 * mass or momentum is not finite. */
int lb_moments(lb_handle* h, double* rho, double* u, double* pineq, double* phi,
               double* conserved);

/* Number of completed time steps since lb_init. */
int64_t lb_step_count(const lb_handle* h);

/* Destroy a handle (frees library-owned memory; a caller-owned buffer is
 * left to the caller).  NULL is accepted.  Waits for the handle's stream. */
int lb_destroy(lb_handle* h);

/* Static description of a status code.  Never NULL. */
const char* lb_strerror(int status);

/* ---- batched execution (serving many independent simulations) -------- */

typedef struct lb_batch lb_batch;

/* Create a batch executor enqueueing on hip_stream (borrowed; every handle
 * passed to lb_batch_step must have been created on the same stream).
 * Not part of the paper: it packs independent simulations so that small
 * domains share launches. */
int lb_batch_create(void* hip_stream, lb_batch** out);

/* Advance handles[i] by nsteps[i] >= 0 steps (distinct handles, count >= 0;
 * LB_EUNSUPPORTED for a handle with near-contact interactions on or without
 * moment arrays).
 * Handles with the same kernel configuration (lattice, Hermite order,
 * species, storage, compute, row vector width) share one moments launch and
 * one stream-collide launch per step; a handle whose step count is reached
 * drops out of later launches.  Each handle's result is bitwise the same as
 * when it is stepped in a batch of its own.  Runs of >= 3 steps with a fixed
 * set of handles are captured once as a HIP graph and replayed (unless
 * disabled with lb_batch_set_graphs); the instantiated graphs of the last
 * 16 launch configurations are kept and reused by later calls that launch
 * the same configuration; the call returns after the graph replays
 * complete.  The descriptor tables live in device and pinned host
 * buffers owned by the batch, grown on demand.  LB_EINVAL for NULL or
 * duplicate handles, negative counts, or a handle on another stream. */
int lb_batch_step(lb_batch* b, lb_handle* const* handles, const int64_t* nsteps, int count);

/* FP64 conservation sums of several handles of this batch's stream in one
 * round trip: out[6 i .. 6 i + 5] = total mass, momentum j (3), red mass,
 * blue mass of handles[i], as lb_moments' conserved[] (a serving loop calls
 * it between chunks to stop a simulation whose state has blown up).  Waits
 * for the stream.  LB_ENONFINITE (after filling every output) if any
 * handle's mass or momentum is not finite; LB_EINVAL for a NULL or foreign
 * handle.  The pinned staging is owned by the batch, grown on demand. */
int lb_batch_conserved(lb_batch* b, lb_handle* const* handles, int count, double* out);

/* Enable (default) or disable graph capture of batched step runs. */
int lb_batch_set_graphs(lb_batch* b, int enable);

/* Destroy a batch executor (waits for its stream).  NULL is accepted. */
int lb_batch_destroy(lb_batch* b);

/* One-shot form of the above: advance handles[i] by nsteps[i] with a batch
 * created on the handles' common stream for this call only (same rules and
 * results as lb_batch_step; the batch's tables are allocated and freed
 * inside the call).  LB_EINVAL also when the handles are on different
 * streams. */
int lb_step_batch(lb_handle* const* handles, const int64_t* nsteps, int count);

/* Limits of lb_step_batch_noalloc: handles per call, and the bytes of its
 * per-device descriptor array. */
#define LB_NOALLOC_MAX_HANDLES 1024
#define LB_NOALLOC_SCRATCH_BYTES (1u << 20)

/* For callers that cannot allocate (code recorded into a HIP graph, tight
 * serving loops, harnesses that forbid hipMalloc): lb_step_batch with no
 * allocation of any kind, device or host.  Same arguments, grouping and
 * results as lb_step_batch (bitwise), with these differences:
 *   - the descriptor tables live in a fixed array of
 *     LB_NOALLOC_SCRATCH_BYTES in the library's device code, one per GPU,
 *     held until the process ends; they are written there by small kernels
 *     on the handles' stream, so the call returns without waiting (like
 *     lb_step) and is ordered with earlier and later work on that stream;
 *   - steps are launched directly, never through a graph;
 *   - every handle must have been created on the current HIP device.
 * The array is shared by every call on one GPU and keeps the last call's
 * tables: two calls whose work overlaps on one GPU (different streams, or
 * different threads without ordering between them) race and may step with
 * each other's tables.  Calls on one stream are safe.
 * LB_ENOMEM for more than LB_NOALLOC_MAX_HANDLES handles (the tables of up
 * to that many always fit the array); LB_EINVAL and LB_EUNSUPPORTED as
 * lb_step_batch, or LB_EINVAL for a handle created on another device or
 * enqueueing on another stream.
 * Nothing is enqueued when an error is returned before the first launch. */
int lb_step_batch_noalloc(lb_handle* const* handles, const int64_t* nsteps, int count);

/* ---- instrumentation ------------------------------------------------- */

/* Start per-kernel timing: the next lb_step calls record HIP events around
 * every moments and stream-collide launch on the handle's stream, for up to
 * max_steps steps (later steps are not timed). */
int lb_timing_begin(lb_handle* h, int64_t max_steps);

/* Stop timing (synchronises the stream) and report the summed device time
 * and launch count of the moments kernel (index 0) and the stream-collide
 * kernel (index 1).  ms[2], launches[2].  Steps taken by the fused step
 * report its kernel at index 1 and no time at index 0. */
int lb_timing_end(lb_handle* h, double* ms, int64_t* launches);

/* Self-check of the short division of the post-collision coefficients
 * (x r plus one correction with the exact FMA residual, used by the
 * instruction-bound kernels in place of the IEEE division): for each odd
 * divisor d = 3, 9, 27 that the lattices need, the number of finite FP32
 * inputs x (all 2^32 bit patterns) whose quotient x / d differs in any bit
 * from the IEEE quotient; 0 means the two divisions are interchangeable.
 * Runs on hip_stream and waits for it; a few tenths of a second.
 * mismatches[3].  LB_EINVAL for NULL. */
int lb_check_division(void* hip_stream, uint64_t* mismatches);

/* Plain device-to-device copy kernel (bytes a multiple of 16, both pointers
 * 16-byte aligned), enqueued on hip_stream: the practical bandwidth ceiling
 * for the sweeps and the scale for hardware byte counters. */
int lb_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
