/*
 * libcos.h -- connected-diagram sums of the SU(N) Hubbard model (CoS / SB-CoS,
 * arXiv 2507.12349) on AMD Instinct MI355X (gfx950), FP64 throughout.
 *
 * What is computed (Results, "Theoretical Constructions"; Methods, Alg. 2/3).
 * A configuration has n interaction vertices, 1 <= n <= COS_NMAX.  Vertex k
 * carries two points, k and k+n, joined by the interaction line (the pairs
 * I = {(i, i+n)} of Alg. 1-3).  Propagator matrices are indexed by vertex:
 * G_l[k][j] is the propagator from vertex k to vertex j for flavour l, with an
 * equal-time pair read as tau = 0^- (Methods, equal-time propagators).  For
 * every permutation pi of the points (minus the shift points, below) and every
 * assignment of one flavour per cycle, the term is
 *     prod_cycles ( w * prod_{p in cycle} G_l[vertex(p)][vertex(pi(p))] )
 *   * prod_shift_points ( -sigma_{l(partner)} )
 * and the library returns the sum of the terms whose diagram is connected
 * (the graph on vertices that joins the vertices of each cycle is
 * connected).  The shift points implement the SB-CoS "shift heads": a point
 * that is not on a propagator cycle, carries the weight -sigma of the flavour
 * of the cycle through its partner, at most one per vertex (Results, SB-CoS;
 * Alg. 3).  No prefactor ((-U)^n/n!, integrals) is included.
 *
 * Variants
 *   COS_UNIFORM : one matrix G (uniform SU(N)); every closed cycle carries the
 *                 factor w * nflav (Alg. 2 closes with -N_f for w = -1).  With
 *                 COS_F_STUBS every shift point carries -sigma[0].
 *   COS_FLAVOUR : nflav matrices G_l (flavour-dependent chemical potentials or
 *                 shifts, Alg. 3); every cycle carries w; with COS_F_STUBS a
 *                 shift point carries -sigma[l].
 * The physical loop weight is w = -1.
 *
 * Memory and ownership.  The caller owns every buffer; the library keeps no
 * caller pointer beyond a call (for the asynchronous calls: beyond the
 * completion of the work queued on the stream).  "d_" arguments are device
 * pointers on the current HIP device, others are host pointers.  Matrices are
 * FP64, row-major: config c, matrix g (0 for COS_UNIFORM, the flavour
 * otherwise), entry [k][j] is at d_G[d_Goff[c] + (g*n_c + k)*n_c + j]
 * (with COS_F_SUBLATTICE the side is 2 n_c instead of n_c).
 * Shift weights: d_stub[c*nstub + g], nstub = 1 (COS_UNIFORM) or nflav.
 *
 * Errors.  Every function returns cos_status.  Arguments are validated before
 * any device work (COS_EINVAL / COS_ERANGE); a failing HIP call returns
 * COS_EDEVICE; detail text for the calling thread is in cos_last_error().
 * No exception crosses the ABI.  Calls on different streams may overlap; a
 * batch handle must not be used by two streams at once (it owns the
 * workspace its kernels write).
 */
#ifndef LIBCOS_H
#define LIBCOS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    COS_OK = 0,
    COS_EINVAL = -1,        /* null pointer, bad variant / flags / sizes */
    COS_ERANGE = -2,        /* n outside [1, COS_NMAX], nflav outside [1, COS_FMAX] */
    COS_ENOMEM = -3,        /* device or host allocation failed */
    COS_EDEVICE = -4,       /* a HIP call failed */
    COS_EUNSUPPORTED = -5   /* no usable gfx950 device */
} cos_status;

#define COS_NMAX 12
#define COS_FMAX 16
#define COS_NMAX_SUBLATTICE 8

enum { COS_UNIFORM = 0, COS_FLAVOUR = 1 };
/* COS_F_SUBLATTICE: bipartite lattices (Results, four-state interaction mask
 * {0, (1,A), (1,B), 2}; Alg. 1/2; Methods, strategy (i): the sum over every
 * sublattice assignment).  Every vertex k also carries a label s_k in {A, B}
 * shared by its two points, and the sum runs over all 2^n labellings in one
 * pass.  Matrices are then 2n x 2n per configuration and flavour, row-major,
 * index 2k + s (s = 0 for A, 1 for B): entry [2k+s][2j+t] is the propagator
 * from vertex k on sublattice s to vertex j on sublattice t.  Orders up to
 * COS_NMAX_SUBLATTICE; forward sums and the reverse sweep (d_G_bar in the
 * same 2n x 2n layout); not combinable with COS_F_STUBS (shifts enter through
 * the matrices' diagonals). */
/* COS_F_MASK_ONLY: the SU(2) mask-only variant (Results, the variant for
 * cycles without extra factors; Methods, Alg. 1).  The DP works on points
 * (each vertex k has an up point and a down point, one per spin block) and
 * tracks only the interaction masks: an extension goes from the current point
 * to any point of its spin block other than the head, onto an interaction not
 * yet visited twice (a point may thus be visited twice: these non-physical
 * clows are kept and cancel through the cycle sign); a closed cycle carries
 * w and the next one opens on the lowest interaction visited once, at either
 * end except the current head.  Requires COS_FLAVOUR with nflav = 2 (matrix 0
 * = the up block, matrix 1 = the down block) and cycle_weight = -1 (the
 * cancellation needs the fermion sign; other weights return COS_EINVAL);
 * not combinable with COS_F_STUBS.  The result is the SU(2) connected sum,
 * 2^-n times the COS_FLAVOUR two-flavour sum of the same matrices.  With
 * COS_F_SUBLATTICE it is Alg. 1 with its sublattice labels.  Forward sums
 * and the reverse sweep. */
/* COS_F_DETERMINISTIC: gradients that are the same bit for bit on every run,
 * whatever the launch shapes, the chunking of the groups or the reverse
 * variant: the reverse sweep cuts each level's masks into a fixed number of
 * parts, sums the dS/dG and dS/dsigma terms of a part in a fixed order in
 * registers (one wavefront per matrix row) and the parts in a fixed order
 * afterwards, with no atomics.  Slower than the default reverse (the child
 * adjoints are read once per row of G, from the caches); the forward and S
 * are unchanged (they are deterministic anyway).  Not combinable with
 * COS_F_SUBLATTICE. */
enum { COS_F_STUBS = 1, COS_F_SUBLATTICE = 2, COS_F_MASK_ONLY = 4, COS_F_DETERMINISTIC = 8 };

typedef struct cos_batch_s *cos_batch_t;

/* Plan a batch of nconf configurations with orders n[c] (host array, read
 * during the call only).  Builds (or reuses) the per-order state tables,
 * uploads the schedule (configurations ordered by decreasing work) and
 * allocates the workspace on the current device.  The handle can then be
 * used for any number of asynchronous calls, including under stream capture,
 * each made with that same device current (COS_EINVAL otherwise).
 * Returns COS_ERANGE for an order outside [1, COS_NMAX], COS_EINVAL for
 * nconf < 1 or a bad variant / flag. */
cos_status cos_batch_create(int32_t nconf, const int32_t *n, int32_t nflav,
                            int32_t variant, int32_t flags, cos_batch_t *out);
/* Upper bound, in bytes, on each of the two level workspaces of batches
 * planned from now on in this process (the forward's two level windows, made
 * at cos_batch_create; the reverse sweep's stored forward levels, made at the
 * first reverse call).  A batch of several orders may take up to half of the
 * bound again for the windows of the orders its forward runs on a second
 * stream (cos_connected_sum_batched), only if that fits, else it runs every
 * order on the caller's stream.  A batch whose groups of 64 configurations do not all
 * fit runs them in chunks of as many groups as fit (at least one), one after
 * the other; results do not depend on the chunking (S bitwise).  0 (the
 * initial setting) bounds the windows by 45% of the device memory free at
 * cos_batch_create and the stored levels by 90% of the memory free at the
 * first reverse call.  Whatever the bound, an allocation that fails is
 * retried with every chunk halved, down to one group per chunk (then
 * COS_ENOMEM).  COS_EINVAL for bytes < 0.  Batches already planned keep
 * their bound. */
cos_status cos_set_workspace_limit(int64_t bytes);
cos_status cos_batch_destroy(cos_batch_t b);

/* Forward sum for every configuration of the batch (the connected sum of
 * Results, "Theoretical Constructions", computed by the dynamic programme of
 * Methods, Alg. 2/3: extensions, closes with the per-cycle weight, heads
 * opened on the lowest once-visited vertex, SB-CoS shift heads), asynchronous
 * on `stream` (a hipStream_t, NULL = default stream).  Configurations are packed 64 to a
 * group (one per lane) by order, largest order first; for each order there is
 * one launch per level of the state space (level = number of visited points,
 * 2n levels), each covering every group of that order.  With two or more
 * orders, the orders after the largest (after the two largest when the
 * others' windows would not fit) run on a second stream of the batch (made
 * at cos_batch_create, default priority, with level windows of their own,
 * up to half of the workspace bound on top of the forward's windows; see
 * cos_set_workspace_limit), forked from `stream` at the call's start and
 * joined back into it (event waits queued on the streams), so that their
 * launches overlap the large orders' small levels; the sums are the same
 * either way (bitwise).  No host
 * synchronisation, no allocation: capturable in a graph (the fork and join
 * are event waits).
 * d_Goff may be NULL when the configurations are stored back to back.
 * d_stub is required iff the batch was planned with COS_F_STUBS.
 * Writes d_out[c] = S_c. */
cos_status cos_connected_sum_batched(cos_batch_t b, const double *d_G, const int64_t *d_Goff,
                                     const double *d_stub, double cycle_weight, double *d_out,
                                     void *stream);

/* Reverse mode: given d_out_bar[c] = dL/dS_c, writes d_G_bar (layout of d_G)
 * = dL/dG and, with COS_F_STUBS, d_stub_bar (layout of d_stub) = dL/dsigma.
 * The forward pass is recomputed inside; d_out (optional, may be NULL)
 * receives S_c.  Asynchronous on `stream`.  The first reverse call on b (or
 * cos_batch_autotune with d_out_bar) allocates the reverse-sweep workspace
 * (every forward level of a chunk of groups); later calls allocate nothing,
 * so make one call before capturing the adjoint in a graph. */
cos_status cos_connected_sum_adjoint(cos_batch_t b, const double *d_G, const int64_t *d_Goff,
                                     const double *d_stub, double cycle_weight,
                                     const double *d_out_bar, double *d_out, double *d_G_bar,
                                     double *d_stub_bar, void *stream);

/* For callers that cannot allocate device memory -- code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc: the forward
 * sums of cos_connected_sum_batched for nconf configurations of one order n
 * (1 <= n <= COS_STATIC_NMAX) stored back to back (d_G holds nconf blocks of
 * nmat*n*n doubles, nmat = 1 for COS_UNIFORM and nflav otherwise; d_stub
 * nconf blocks of nstub weights, required iff flags = COS_F_STUBS, the only
 * flag taken), with no batch handle.  Writes d_out[c] = S_c, the same values
 * as the batched call (same kernels).  Every workspace lives in one static
 * device array of COS_STATIC_SCRATCH_BYTES per device, which each device the
 * library runs on holds until the process ends: its state tables for orders
 * 1..COS_STATIC_NMAX, then the call's schedule, packed inputs and two level
 * windows (a call processes its groups of 64 configurations in chunks of as
 * many as fit).  A call that needs more than the array holds (too many
 * configurations or flavour slots for the packed inputs plus one group's
 * windows) returns COS_ERANGE with the sizes in cos_last_error.  The first
 * call on a device takes the array's address and uploads the tables
 * (synchronous, not capturable); later calls only queue kernels on `stream`
 * and can be captured in a graph.  No call allocates device memory.  All
 * calls on one device share the array, so calls that overlap on one device
 * (another stream, another thread) race: serialise them. */
#define COS_STATIC_NMAX 8
#define COS_STATIC_SCRATCH_BYTES (64 << 20)
cos_status cos_connected_sum_static(int32_t nconf, int32_t n, int32_t nflav, int32_t variant, int32_t flags,
                                    const double *d_G, const double *d_stub, double cycle_weight,
                                    double *d_out, void *stream);

/* One configuration from HOST buffers (G: nmat*n*n, or nmat*(2n)*(2n) with
 * COS_F_SUBLATTICE; stub: nstub or NULL when flags lacks COS_F_STUBS);
 * copies to the device, runs the GPU kernel, synchronises and writes *out.
 * Convenience for small callers and tests. */
cos_status cos_connected_sum(int32_t n, int32_t nflav, int32_t variant, int32_t flags,
                             const double *G, const double *stub, double cycle_weight,
                             double *out);

/* Free propagator matrices on the device (Methods, square-lattice model):
 * xi_g(k) = -2 t (cos kx + cos ky) - mu[g] + alpha[g] on k = 2 pi (mx, my)/L,
 * G(k, tau) = -exp(-xi tau)(1 - nF) for tau > 0 and exp(-xi tau) nF for
 * tau <= 0 (an equal-time pair is 0^-), G_g[k][j] = L^-2 sum_k
 * cos(k.(r_k - r_j)) G(k, tau_k - tau_j).  d_dG (may be NULL) receives
 * dG_g/dxi for a uniform move of xi_g (so d/dmu_g = -d/dxi).
 * d_sites: int32 [sum n][2] lattice coordinates in [0, L), 1 <= L <= 32; d_tau [sum n];
 * d_voff[c]: first vertex of config c; mu, alpha: HOST arrays [nmat].
 * Output layout as d_G above with nmat matrices per configuration. */
cos_status cos_build_g0(int32_t nconf, const int32_t *d_n, const int64_t *d_voff,
                        const int32_t *d_sites, const double *d_tau, int32_t L, double t,
                        double beta, int32_t nmat, const double *mu, const double *alpha,
                        const int64_t *d_Goff, double *d_G, double *d_dG, void *stream);

/* Free propagator matrices of the honeycomb lattice for COS_F_SUBLATTICE
 * batches (Methods, honeycomb model): per matrix g the Bloch Hamiltonian
 * H_g(k) = [[delta[g] - (mu[g] - alpha[g]), eps(k)], [conj(eps(k)),
 * -delta[g] - (mu[g] - alpha[g])]] with eps(k) = -t (1 + e^{i k.b1} +
 * e^{i k.b2}) on the L x L grid k.b_i = 2 pi m_i / L (sublattice A of cell R
 * hops to B of R, R + b1, R + b2); G(k, tau) = -exp(-H tau)(1 - nF(H)) for
 * tau > 0 and exp(-H tau) nF(H) for tau <= 0 (an equal-time pair is 0^-);
 * entry [2a+p][2b+q] = L^-2 sum_k e^{i k.(R_a - R_b)} G_pq(k, tau_a - tau_b).
 * d_cells: int32 [sum n][2] unit-cell coordinates in [0, L), 1 <= L <= 32;
 * d_tau [sum n]; d_voff[c]: first vertex of config c; mu, alpha, delta: HOST
 * arrays [nmat].  Output: nmat matrices of side 2 n_c per configuration at
 * d_G[d_Goff[c] + (g*2n_c + i)*2n_c + j].  d_dG (may be NULL) receives, in
 * the same layout, dG_g/dxi for a uniform move H_g -> H_g + xi (xi = -(mu[g]
 * - alpha[g]); so d/dmu_g = -d/dxi), for cos_chain_mu_shift.  The equal-time
 * shift the CoS formulation puts on the diagonal is left to the caller. */
cos_status cos_build_g0_honeycomb(int32_t nconf, const int32_t *d_n, const int64_t *d_voff,
                                  const int32_t *d_cells, const double *d_tau, int32_t L, double t,
                                  double beta, int32_t nmat, const double *mu, const double *alpha,
                                  const double *delta, const int64_t *d_Goff, double *d_G, double *d_dG,
                                  void *stream);

/* Chain rule to the chemical potential and the shift (Methods: xi = eps -
 * mu + alpha, shift weight sigma = alpha / U).  Per configuration c and
 * matrix g: xb = sum_kj G_bar[g][k][j] * dG[g][k][j] over the d_n[c] x d_n[c]
 * entries of matrix g (d_n[c] is the matrix side: n_c, or 2 n_c for
 * sublattice matrices);
 *   d_mu_bar[c*nmat + g]    = -xb
 *   d_alpha_bar[c*nmat + g] = +xb + stub_bar[c*nstub + g] / U   (stub_bar may be NULL)
 * For COS_UNIFORM (nmat = 1) the per-flavour shift derivative at equal shifts
 * is d_alpha_bar / nflav by flavour symmetry. */
cos_status cos_chain_mu_shift(int32_t nconf, const int32_t *d_n, int32_t nmat,
                              const int64_t *d_Goff, const double *d_G_bar, const double *d_dG,
                              const double *d_stub_bar, int32_t nstub, double U,
                              double *d_mu_bar, double *d_alpha_bar, void *stream);

/* Plan counts for order n, per flavour (exact integers, host only): the
 * size of the dynamic programme's state space with visited sets merged for
 * contact interactions (Results: the O(n^3 3^n) form with per-vertex counts
 * 0, 1, 2): states, extension transitions, closes, shift transitions (the
 * SB-CoS shift heads of Alg. 3), masks, rows (a row = one (mask, head) pair).
 * COS_ERANGE for n outside [1, COS_NMAX]. */
cos_status cos_plan_counts(int32_t n, int64_t *states, int64_t *extensions, int64_t *closes,
                           int64_t *shift_edges, int64_t *masks, int64_t *rows);

/* Memory of the reverse sweep.  The reverse levels need the forward states of
 * every level; segments = 1 stores them all (about 7 times the largest
 * level per group at n = 12), segments = 2 stores only levels h+1..2n during
 * the forward, reverses them, then computes levels 1..h again into the same
 * store and reverses those (h chosen so that both halves hold about the same
 * number of rows: about 40% less memory per group, the lower levels'
 * forward run twice).  0 (the default) takes 2 when storing every level would
 * split the batch's groups into several chunks (cos_set_workspace_limit),
 * else 1.  Results are the same either way (S bitwise; gradients up to the
 * summation order of their accumulation).  If the reverse workspace already
 * exists it is freed (after waiting for the device) and planned again at the
 * next reverse call.  COS_EINVAL for other values. */
cos_status cos_batch_set_adjoint_segments(cos_batch_t b, int32_t segments);
/* The reverse-sweep plan of order n, after a reverse call: the split level
 * (0: every level stored), groups of 64 configurations per chunk, and bytes
 * of workspace per group (stored forward states and the two adjoint
 * windows).  Any output may be NULL.  COS_EINVAL before the first reverse
 * call or for an order the batch does not have. */
cos_status cos_batch_adjoint_plan(cos_batch_t b, int32_t n, int32_t *split_level, int32_t *groups_per_chunk,
                                  int64_t *bytes_per_group);

/* Autotuner (Results, GPU parallelization: launch shape per problem size).
 * For every order in the batch, times the level kernels over the caller's
 * inputs for each candidate launch shape -- wavefronts per workgroup of the
 * forward kernel (4, 8, 16; 8, 16 with COS_F_SUBLATTICE) and the most masks
 * (state-table tiles) per wavefront of the forward (1, 2, 4, 8, 16) and, when
 * d_out_bar is not NULL, of the reverse kernel (2, 4, 6, 8, 12, 16, 24, 32, 48, 64;
 * a reverse level is cut into as few rounds of one workgroup per CU as that
 * cap allows, its masks spread evenly) -- keeps the fastest per order and
 * uses it for every later call on b.  Arguments as cos_connected_sum_batched
 * / _adjoint; the output
 * buffers are overwritten and on return hold what a call with the chosen
 * shapes writes.  Synchronous (waits for the stream).  S does not depend on
 * the launch shape (bitwise); the gradients do only through the summation
 * order of their accumulation. */
cos_status cos_batch_autotune(cos_batch_t b, const double *d_G, const int64_t *d_Goff,
                              const double *d_stub, double cycle_weight, const double *d_out_bar,
                              double *d_out, double *d_G_bar, double *d_stub_bar, void *stream);
/* The launch shape in use for order n (COS_EINVAL if the batch has none). */
cos_status cos_batch_launch_shape(cos_batch_t b, int32_t n, int32_t *fwd_waves,
                                  int32_t *fwd_masks, int32_t *adj_masks);
/* Set the launch shape of order n instead of tuning it (for instance one that
 * cos_batch_autotune found before): fwd_waves in [1, 16], fwd_masks in
 * [1, 16], adj_masks in [1, 64] (the forward clamps
 * its masks per wavefront to 4 with several flavour slots).  COS_EINVAL for
 * values outside these ranges or an order the batch does not have. */
cos_status cos_batch_set_launch_shape(cos_batch_t b, int32_t n, int32_t fwd_waves, int32_t fwd_masks,
                                      int32_t adj_masks);

/* Phase timing, a measurement aid.  After cos_batch_timing_enable(b, 1),
 * every forward or adjoint call on b records HIP events on its own stream at
 * the boundaries of its phases (COS_PHASE_*).  cos_batch_timing_read waits
 * for the last recorded event, writes into ms[COS_NPHASES] the device time of
 * each phase summed over every call since the previous read (milliseconds)
 * and into *ncalls (may be NULL) the number of those calls, and starts a new
 * accumulation.  Phases: packing of the inputs and zeroing of the gradient
 * accumulators; the forward levels (recomputed inside the adjoint); the
 * reverse levels; unpacking of the gradients.  Not for use under stream
 * capture. */
enum { COS_PHASE_PACK = 0, COS_PHASE_FORWARD = 1, COS_PHASE_REVERSE = 2, COS_PHASE_UNPACK = 3,
       COS_NPHASES = 4 };
cos_status cos_batch_timing_enable(cos_batch_t b, int32_t enable);
cos_status cos_batch_timing_read(cos_batch_t b, double *ms, int32_t *ncalls);

/* Plan counts of the sublattice-labelled state space for order n (1..8),
 * per flavour: states, extension transitions, closes, masks, rows. */
cos_status cos_plan_counts_sublattice(int32_t n, int64_t *states, int64_t *extensions, int64_t *closes,
                                      int64_t *masks, int64_t *rows);

/* State counts of the mask-only variant (COS_F_MASK_ONLY; Alg. 1), for
 * order n (1..COS_NMAX, or 1..COS_NMAX_SUBLATTICE with flags =
 * COS_F_SUBLATTICE; flags may hold nothing else): the slots the level kernels
 * visit, i.e. the states (head point, current point, mask) reachable from the
 * start, the extension transitions out of them, and the states that close a
 * cycle (a once-visited interaction exists, or the mask is full).  Host-only;
 * any output pointer may be NULL. */
cos_status cos_plan_counts_mask_only(int32_t n, int32_t flags, int64_t *states, int64_t *extensions,
                                     int64_t *closes);

/* Monte Carlo support (the series coefficients are integrals of the
 * connected sum over vertex sites and times; Methods, diagrammatic
 * expansion).  cos_mc_sample writes nconf configurations of order n for the
 * G0 builders: vertex 0 at site (0, 0) and time 0 (translation invariance),
 * vertices 1..n-1 uniform over the L x L sites and [0, beta), drawn from a
 * counter-based generator: the splitmix64 output function (Steele, Lea,
 * Flood 2014) of seed + 0x9E3779B97F4A7C15 * (ctr + 1), with ctr =
 * ((first + c) * n + k) * 2 + q for component q (0 site, 1 time) of vertex k
 * of configuration c; site = ((z >> 32) * L^2) >> 32 as x + L y, time =
 * beta * (z >> 11) * 2^-53.  d_sites int32 [nconf*n][2], d_tau [nconf*n]
 * (configurations back to back).  Asynchronous on `stream`. */
cos_status cos_mc_sample(int32_t nconf, int32_t n, int32_t L, double beta, uint64_t seed, int64_t first,
                         int32_t *d_sites, double *d_tau, void *stream);
/* d_acc[0] += sum_i d_x[i], d_acc[1] += sum_i d_x[i]^2 over count values
 * (device buffers, fixed summation order).  Asynchronous on `stream`. */
cos_status cos_accumulate_moments(int32_t count, const double *d_x, double *d_acc, void *stream);
/* [m/k] Pade approximant of sum_{i=0}^{m+k} a_i x^i evaluated at x (HOST
 * arrays; Results, Pade re-summation): *value, and when grad is not NULL
 * grad[i] = d value / d a_i for i = 0..m+k (for the linear error propagation
 * delta^2 = sum_i grad_i^2 delta_a_i^2).  COS_ERANGE when the approximant
 * does not exist (singular denominator system). */
cos_status cos_pade(int32_t m, int32_t k, const double *a, double x, double *value, double *grad);

/* CDet comparison path (Methods: the 3^n labelled principal minors by
 * Schur complements with pseudo-pivots, then the connected part by the
 * subset recursion; the paper's instability study) for the SU(2) bipartite
 * model.  Per configuration d_A holds two 2n x 2n matrices, spin up then
 * spin down, index 2k + s as for COS_F_SUBLATTICE ([nconf][2][2n][2n]).
 * d_out[c] = sum over the 2^n full labellings of the connected part of
 * det A_up[T] det A_dn[T] (the quantity of Alg. 1, which equals the
 * two-flavour COS_F_SUBLATTICE sum divided by 2^n).  precision 0: FP64;
 * 1: double-double (software, about 32 significant digits).  A pivot of
 * magnitude below eps is replaced by C = sum |A| / (2n)^2 and the affected
 * minors are corrected afterwards by multilinearity (deepest first).
 * 1 <= n <= COS_NMAX_SUBLATTICE.  The caller provides d_work of at least
 * the size cos_cdet_workspace returns.  Asynchronous on `stream`. */
cos_status cos_cdet_workspace(int32_t n, int32_t nconf, int32_t precision, uint64_t *bytes);
cos_status cos_cdet_su2(int32_t nconf, int32_t n, const double *d_A, int32_t precision, double eps,
                        void *d_work, uint64_t work_bytes, double *d_out, void *stream);

/* Integer counting mode: the number of connected diagrams of order n when
 * every propagator is 1 and every closed cycle carries the integer weight
 * cycle_weight (x = w * N for the uniform SU(N) variant; x = +1 counts the
 * diagrams, x = -N gives the sum with unit propagators and fermion loops),
 * computed by the same dynamic programme in unsigned 64-bit integers on the
 * device: *count is the exact count modulo 2^64, read as a signed number (so
 * exact while |count| < 2^63: for x = +1 up to n = 10).  Synchronous, default
 * stream.  The full sum over all diagrams is x (x + 1) ... (x + 2n - 1), and
 * the connected counts follow from it by the exponential formula (Methods,
 * connected-part recursion). */
cos_status cos_connected_count(int32_t n, int64_t cycle_weight, int64_t *count);

/* Testing aid for the error paths (no effect unless called): of the device
 * allocations (kind 0) or kernel launches (kind 1) that the batch calls
 * (cos_batch_create, the batched forward, reverse and autotuning calls,
 * cos_connected_sum, cos_connected_sum_static) and the propagator, chain-rule,
 * sampling and CDet calls make from now on, the next `skip` proceed and the
 * `count` after them fail -- an
 * allocation as if the device were out of memory (the calls then return
 * COS_ENOMEM, or retry the level workspaces with smaller chunks, see
 * cos_set_workspace_limit), a launch is skipped and its call returns
 * COS_EDEVICE (launches queued before it stay queued).  count = 0 clears.
 * Process-wide; COS_EINVAL for another kind or negative numbers. */
cos_status cos_inject_failures(int32_t kind, int32_t skip, int32_t count);

/* Diagnostics. */
const char *cos_status_string(cos_status s);
const char *cos_last_error(void);
/* Frees the cached state tables of every device.  Batch handles point into
 * these tables, so while any handle is alive nothing is freed and COS_EINVAL
 * is returned; destroy every handle (after its work has completed) first. */
cos_status cos_release(void);

#ifdef __cplusplus
}
#endif
#endif /* LIBCOS_H */
