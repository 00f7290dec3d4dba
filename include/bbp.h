/*
 * bbp.h - C ABI of libbbp: block belief propagation (block BP) for 2D PEPS
 * on an MI355X (gfx950) GPU.
 *
 * Method: Guo, Poletti and Arad, "Block belief propagation algorithm for
 * two-dimensional tensor networks".  The double-layer network <psi|psi>
 * (Sec. II, Fig. 1(a,b)) is cut into blocks (Fig. 1(c)); every directed
 * message between neighbouring blocks is an MPS along their shared edge,
 * updated by Eq. (1) from the other three incoming messages of the sending
 * block, with the block contracted column by column as MPO x MPS variational
 * fits truncated to bond chi (App. A).  Observables use the converged
 * messages as the block environment (Sec. II; App. A; App. B).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All arithmetic is FP64 unless the "precision" option says otherwise.
 *  - Site tensor layout: A[site][s][u][l][d][r], C order, doubles.  s is the
 *    physical index (dimension d, default 2, s=0 <-> sigma_z=+1); u,l,d,r
 *    the up/left/down/right virtual legs, each stored with dimension D.
 *    Sites are row-major (y outer, x inner).
 *  - Finite lattices have open boundaries: a leg pointing off the lattice
 *    has true dimension 1 and must be zero for indices > 0 (zero padding);
 *    otherwise BBP_EINVAL.  Infinite lattices take the ucx*ucy tensors of
 *    the unit cell, every leg of true dimension D.
 *  - Operators: one-site op[s'][s] (d x d, row-major); two-site
 *    op[(s0',s1')][(s0,s1)] (d^2 x d^2) with the first site as major index.
 *    Expectation values are <psi|O|psi>/<psi|psi> for real tensors.
 *  - Ownership: the caller owns every host buffer; the library copies on
 *    entry and never keeps a caller pointer.  The context owns the device
 *    memory it allocates (hipMalloc) and frees it in bbp_destroy.
 *  - Errors: every call returns a bbp_status; bbp_last_error() gives a
 *    context-local message.  Arguments are validated before any state
 *    changes.  A failed sweep leaves the previous messages in place.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef BBP_H
#define BBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bbp_ctx bbp_ctx;

typedef enum {
  BBP_OK = 0,
  BBP_EINVAL = 1,   /* invalid argument or tensor content              */
  BBP_ENOMEM = 2,   /* device or host allocation failed                */
  BBP_EDEVICE = 3,  /* HIP runtime error or no usable gfx950 device    */
  BBP_ESTATE = 4,   /* call not valid in the current state             */
  BBP_ENUMERIC = 5  /* zero-norm or non-finite message or boundary     */
} bbp_status;

/*
 * Create a context.  Finite open lattice: infinite = 0, Lx x Ly sites,
 * ucx = ucy = 0 (the unit cell is the lattice).  Infinite lattice (Sec. II,
 * iPEPS paragraph: one block exchanging messages with its own copies):
 * infinite = 1, Lx = Ly = 0, unit cell ucx x ucy, and the block must be a
 * multiple of the cell.  Blocks are bx x by sites (Fig. 1(c)); a finite
 * lattice that is not a multiple of the block is padded with trivial sites,
 * which leaves <psi|psi> unchanged.  D is the PEPS bond dimension, chi the
 * message bond cap (chi_m of Sec. II, App. A).
 * Errors: BBP_EINVAL for non-positive sizes or an incommensurate block,
 * BBP_EDEVICE if no GPU is usable, BBP_ENOMEM.
 */
bbp_status bbp_create(bbp_ctx **out, int32_t infinite, int32_t Lx, int32_t Ly,
                      int32_t ucx, int32_t ucy, int32_t bx, int32_t by,
                      int32_t D, int32_t chi);

/*
 * Set an option before bbp_set_tensors (later changes return BBP_ESTATE,
 * except "n_fit" and "chi_env", which may change at any time):
 *   "d"        physical dimension (default 2)
 *   "chi_env"  boundary bond for observables (default 2*D^2+10, Sec. II)
 *   "n_fit"    full fit sweeps per column absorption (default 2, App. A)
 *   "seed"     seed of the counter-based fit initial states (default 0)
 *   "init"     initial messages (before bbp_set_tensors, which applies
 *              them): 0 (default) the identity product MPDO; 1 a random
 *              product MPDO (App. A), per site m[(k,k')] = sum_a R[k][a]
 *              R[k'][a] with R the D x D counter-based uniform values of
 *              (seed, 2^41 + message index, site), scaled to unit 2-norm
 *   "hbm_budget" device bytes the context may hold (any time; default 0: no
 *              limit): an allocation that would pass it fails like an
 *              out-of-memory one (the kept buffers are freed and it is tried
 *              once more, then BBP_ENOMEM; the context stays usable)
 *   "timing"   1: record per-kernel-class launch times (any time; resets)
 *   "precision" 64 (default), 32 or 16 (any time): with 32 the fit's
 *              visit and environment contractions run on FP32 MFMA with
 *              FP32 accumulation in every fused visit (any D, bond cap
 *              <= 64); with 16 they run on BF16 MFMA (operands rounded to
 *              BF16, FP32 accumulation) in the generic fused visit (any D,
 *              bond cap <= 64; at D=4 that visit is slower than the
 *              specialised FP32 one); fits whose visits run as separate
 *              kernels (bond caps above 64, e.g. the observables at a
 *              chi_env above 64) stay FP64; QR, normalisation, overlaps and
 *              every stored message stay FP64.  Sweeps in 16, then 32, then
 *              64 reach the FP64 fixed point from the lower-precision ones.
 *   "graphs"   1 (default) or 0 (any time): once a message batch's column
 *              absorptions all start warm (from the second sweep on), their
 *              launches are captured as a HIP graph and replayed in later
 *              sweeps; 0 launches them one by one.  Results do not depend
 *              on it.  Not used while "timing" is 1.
 *   "skip_padding" 1 (default) or 0 (any time): the column absorptions'
 *              visit and environment kernels stop at every item's true bond
 *              dimensions instead of the padded cap (the skipped terms are
 *              zeros, so results are bitwise the same); 0 runs the padding.
 *   "single_layer" 0 (default) or 1 (before bbp_set_tensors): the network
 *              is the single layer sum_s A[s] (Sec. V classical Ising: a
 *              tensor network of bond dimension D, messages MPSs over its
 *              bonds, App. A) instead of the double layer <psi|psi>: the
 *              bra layer of every site is fixed to index 0 on every leg, so
 *              the fused leg (k, k') carries the network's bond k at k' = 0.
 *              A one-site operator O then inserts sum_s (sum_s' O[s',s]) A[s]
 *              (for a diagonal O the impurity sum_s O[s,s] A[s]), and
 *              bbp_log_norm gives log|Z| of the network.
 *   "shift_x", "shift_y" 0..bx-1, 0..by-1 (default 0; finite lattices,
 *              before bbp_set_tensors): a partition of the lattice into blocks
 *              shifted by (shift_x, shift_y) sites (Sec. II: several
 *              partitions that differ by a shift cover every bond at the
 *              centre of some block).  The lattice is padded with shift_x
 *              trivial columns on the left and shift_y trivial rows on top,
 *              the same as shifting an open lattice embedded in a periodic
 *              one with dimension-1 bonds at its edges; sites keep their
 *              lattice coordinates in every call.
 *   "message_split" 0..4 (default 2; before bbp_set_tensors): the messages
 *              of one shape are updated as this many batches (of at least 8
 *              messages each), one per lane, so that one batch's QRs overlap
 *              another's visits; 0 updates every message as a batch of its
 *              own (the plain per-message form, for comparison).  Results
 *              do not depend on it.
 *   "lanes"    1..4 (default 3; before bbp_set_tensors): independent batches
 *              run on this many streams (the context stream and lanes-1
 *              streams the context creates) and overlap on the GPU: the
 *              message batches one per shape, the observables' boundary
 *              stacks with every shape split over the lanes.  Results do not
 *              depend on it; the context stream waits for every lane before
 *              a call returns.
 * Unknown keys or out-of-range values: BBP_EINVAL.
 */
bbp_status bbp_set_option(bbp_ctx *c, const char *key, double value);

/* Launch all work of this context on the given hipStream_t (default: the
 * null stream).  The pointer is a HIP stream handle; NULL selects the null
 * stream.  Every transfer the context makes is ordered on this stream, so a
 * non-blocking stream is fine; it must stay valid until bbp_destroy, which
 * synchronises it.  With "lanes" > 1 the context also launches on streams of
 * its own, forked from and joined back into this one inside each call. */
bbp_status bbp_set_stream(bbp_ctx *c, void *hip_stream);

/* Device memory through the caller's allocator instead of hipMalloc/hipFree
 * (for example PyTorch's caching allocator, which then accounts for it).
 * alloc(bytes, user) returns a device pointer, or NULL on failure;
 * free_(ptr, user) takes back a pointer alloc returned.  The library
 * synchronises its stream before it hands memory back, so a stream-ordered
 * allocator may reuse it at once.
 * Both functions or neither (NULL, NULL: hipMalloc/hipFree); user is passed
 * through.  Must be called before bbp_set_tensors (BBP_ESTATE afterwards);
 * both functions must stay callable until bbp_destroy returns.
 * Out of memory (either allocator): the context frees the device buffers it
 * only keeps for reuse by later observable calls and tries the allocation
 * once more; if that fails too, the call returns BBP_ENOMEM and the context
 * stays usable. */
typedef void *(*bbp_alloc_fn)(size_t bytes, void *user);
typedef void (*bbp_free_fn)(void *ptr, void *user);
bbp_status bbp_set_allocator(bbp_ctx *c, bbp_alloc_fn alloc, bbp_free_fn free_, void *user);

/*
 * Upload the site tensors (host FP64, layout above; n = number of doubles =
 * nsites*d*D^4 with nsites = Lx*Ly or ucx*ucy), form the per-message rotated
 * copies, and reset the messages to the identity product state (one site
 * m[(k,k')] = delta_kk'/sqrt(D)) and the fit warm starts.
 * Errors: BBP_EINVAL for a wrong n, NaN/Inf entries, or nonzero padding on
 * an open edge.
 */
bbp_status bbp_set_tensors(bbp_ctx *c, const double *A, size_t n);

/*
 * Copy the context's site tensors (as last set, or as bbp_ite_step left
 * them) to host memory A, the layout of bbp_set_tensors; n must be that
 * count.  Errors: BBP_ESTATE before bbp_set_tensors, BBP_EINVAL for a wrong
 * n or a null pointer.
 */
bbp_status bbp_get_tensors(bbp_ctx *c, double *A, size_t n);

/*
 * Exactly n synchronous sweeps of Eq. (1): every directed message between
 * neighbouring blocks is recomputed from the previous sweep's messages
 * (Sec. II: all messages of one iteration are independent).  No early exit.
 * *residual (may be NULL) receives the last sweep's residual: the mean over
 * directed messages of max(0, 2 - 2|<m_new, m_old>|) for unit-norm messages
 * (the squared sign-aligned distance; App. A's mean-square error).
 * With the environment variable BBP_SWEEP_LOG naming a file, every sweep
 * appends one JSON line to it: {"ctx", "sweep" (counted from the last
 * bbp_set_tensors), "residual", "ms" (host wall time of the sweep),
 * "fit_flops" (counted on the split-layer schedule), "messages"}.
 * Errors: BBP_ESTATE before bbp_set_tensors, BBP_ENUMERIC for a zero-norm
 * or non-finite message (messages then stay at their previous values).
 */
bbp_status bbp_sweep(bbp_ctx *c, int32_t n, double *residual);

/*
 * <O> at site (x, y) from the current messages (Sec. II, App. A, App. B):
 * the site's block with its four incoming messages; boundary MPSs absorbed
 * from top and bottom at bond chi_env; the site's row contracted exactly.
 * Infinite lattices: (x, y) in unit-cell coordinates, evaluated at the copy
 * nearest the centre of the block.  op: d*d doubles.
 */
bbp_status bbp_expect_site(bbp_ctx *c, int32_t x, int32_t y,
                           const double *op, double *out);

/*
 * <O> on the nearest-neighbour bond (x0,y0)-(x1,y1) with (x1,y1) =
 * (x0+1,y0) or (x0,y0+1).  A bond inside a block uses that block; a bond
 * crossing two blocks uses the union of the two blocks with its six
 * incoming messages.  Vertical bonds are contracted along their column.
 * op: d^2*d^2 doubles.  Errors: BBP_EINVAL for other site pairs.
 */
bbp_status bbp_expect_bond(bbp_ctx *c, int32_t x0, int32_t y0, int32_t x1,
                           int32_t y1, const double *op, double *out);

/*
 * Batched forms of the two calls above: n sites (xs[i], ys[i]) with one
 * shared operator, or n bonds.  out has n entries.
 */
bbp_status bbp_expect_sites(bbp_ctx *c, int32_t n, const int32_t *xs,
                            const int32_t *ys, const double *op, double *out);
bbp_status bbp_expect_bonds(bbp_ctx *c, int32_t n, const int32_t *x0,
                            const int32_t *y0, const int32_t *x1,
                            const int32_t *y1, const double *op, double *out);

/*
 * Site and bond expectation values from one call (Sec. II; App. B): the
 * results of bbp_expect_sites(ns, xs, ys, op_site, out_sites) and
 * bbp_expect_bonds(nb, x0, y0, x1, y1, op_bond, out_bonds), bit for bit,
 * with the regions of both (blocks, and the unions of two blocks that
 * bonds crossing blocks need) contracted together, so that their boundary
 * stacks run side by side on the context's lanes.  ns or nb may be 0 (the
 * matching arrays may then be null).  Errors as the two calls.
 */
bbp_status bbp_expect_terms(bbp_ctx *c, int32_t ns, const int32_t *xs, const int32_t *ys,
                            const double *op_site, int32_t nb, const int32_t *x0,
                            const int32_t *y0, const int32_t *x1, const int32_t *y1,
                            const double *op_bond, double *out_sites, double *out_bonds);

/*
 * Reduced density matrices from the same region contractions as the
 * expectation values (App. C): rho[a][b] with <O> = Tr(rho O), unit trace.
 * Sites: n matrices of d x d (a = s, b = s').  Bonds (the pairs of
 * bbp_expect_bonds): n matrices of d^2 x d^2 with a = (s0, s1), b =
 * (s0', s1'), the first site the major index.  rho receives n*d^2 or n*d^4
 * doubles.  Errors as bbp_expect_sites / bbp_expect_bonds.
 */
bbp_status bbp_rdm_sites(bbp_ctx *c, int32_t n, const int32_t *xs,
                         const int32_t *ys, double *rho);
bbp_status bbp_rdm_bonds(bbp_ctx *c, int32_t n, const int32_t *x0,
                         const int32_t *y0, const int32_t *x1,
                         const int32_t *y1, double *rho);

/*
 * Trace distance D(rho, sigma) = Tr|rho - sigma| / 2 with |Z| = sqrt(Z^T Z)
 * (App. C) of two m x m real matrices (row-major, host): half the sum of the
 * singular values of the difference (one-sided Jacobi on the host).  No
 * context.  Errors: BBP_EINVAL for m outside [1, 64], null or non-finite
 * input.
 */
bbp_status bbp_trace_distance(int32_t m, const double *rho, const double *sigma,
                              double *out);

/*
 * Truncated SVD of a batch of real m x n matrices (m >= n) on the GPU, FP64:
 * A_b = U_b diag(S_b) V_b^T by one-sided (Hestenes) Jacobi rotations, of
 * which the k largest singular triplets are kept -- the compression step of
 * the standard alternative to the zip-up fit (App. A: multiply the MPO into
 * the MPS, then compress it bond by bond).  No context.
 *  - A: device, batch x m x n doubles, row-major, item b at A + b m n; read
 *    only.  U: device, batch x m x k row-major; S: device, batch x k, in
 *    descending order; V: device, batch x n x k row-major.  err2 (or null):
 *    device, batch doubles, the discarded weight sum_{i >= k} S_i^2.
 *    sweeps (or null): device, batch int32, the Jacobi sweeps taken,
 *    negative if max_sweeps ended the iteration before a sweep rotated
 *    nothing.  The caller owns every buffer; nothing is allocated.
 *  - Each U column and its V column are signed so that the largest-magnitude
 *    entry of the U column (the first of equal ones) is positive; the U
 *    column of a zero singular value is zero.  Equal singular values keep
 *    the order of the columns they came from.
 *  - A pair of columns is rotated while |a_p . a_q| > tol |a_p| |a_q|; tol 0
 *    takes sqrt(m) times the FP64 epsilon.  At most max_sweeps sweeps.
 *  - The work is enqueued on hip_stream (null: the null stream) and the
 *    call returns without waiting.  Each item's result is the same, bit for
 *    bit, whatever else the batch holds.  Non-finite input gives non-finite
 *    output, not an error.
 *  - Errors: BBP_EINVAL for batch < 0, n outside [1, 64], m < n, k outside
 *    [1, n], m n + n n > BBP_SVD_MAX_WORDS, max_sweeps outside [1, 100],
 *    tol outside [0, 1), or a null A, U, S or V with batch > 0;
 *    BBP_EDEVICE if the launch fails.
 */
#define BBP_SVD_MAX_WORDS 19968
bbp_status bbp_svd_jacobi(int32_t batch, int32_t m, int32_t n, int32_t k,
                          const double *A, double *U, double *S, double *V,
                          double *err2, int32_t *sweeps, int32_t max_sweeps,
                          double tol, void *hip_stream);

/*
 * log|<psi|psi>| estimated by the block Bethe formula
 * sum_blocks log|Z_A| - sum_edges log|Z_AB| (Z_A: block A with its four
 * incoming unit-norm messages; Z_AB = <m_{A->B}, m_{B->A}>).  Exact when
 * the block graph is a tree.  Infinite lattices: per block.
 */
bbp_status bbp_log_norm(bbp_ctx *c, double *log_abs, int32_t *sign);

/*
 * Messages as flat FP64: for each directed message in enumeration order
 * (blocks row-major, directions L,R,U,D, only existing neighbours), an
 * int-valued header [nsites, b_0..b_nsites] (bond dims as doubles) followed
 * by each site [b_i][D*D][b_{i+1}] in C order.  bbp_get_messages writes at
 * most n doubles and reports the size needed in *needed; bbp_set_messages
 * replaces every message (and clears the fit warm starts).
 */
bbp_status bbp_get_messages(bbp_ctx *c, double *buf, size_t n, size_t *needed);
bbp_status bbp_set_messages(bbp_ctx *c, const double *buf, size_t n);

/* Number of directed messages and the floating-point operations of the
 * last sweep counted on the split-layer schedule (fit contractions only). */
bbp_status bbp_stats(bbp_ctx *c, int32_t *n_messages, double *sweep_flops);

/*
 * Launch statistics of kernel class cls (0 .. 8) collected while the
 * "timing" option is 1, summed over the process since the last reset: the
 * class name (static string), number of launches, total duration in ms
 * measured with HIP events on the stream the kernels were launched on, and
 * the algorithmic floating-point operations and HBM bytes of those launches:
 * the split-layer contractions of App. A Eq. (update) and its environment
 * recursion counted on every item's true bond dimensions, and the bytes of
 * their operands read plus results written, once each (for a fit visit and
 * its environment update together: Lenv, X, Renv, the site tensor, Yt, Y and
 * the new environment).  The observables' final line contractions count at
 * the bond cap chi_env.  Synchronises the recorded events.  Classes:
 * fit_visit (the fused contractions of one fit visit on MFMA), fit_T1,
 * fit_ket, fit_bra, fit_local (the same contractions as separate kernels,
 * used when the fused tiles do not fit in LDS), fit_env (environment
 * recursion of App. A), fit_end (end-site contractions), qr (Householder
 * QR/LQ of the true panels), other.  Errors: BBP_EINVAL for cls out of
 * range.
 */
bbp_status bbp_kernel_stats(bbp_ctx *c, int32_t cls, const char **name,
                            int64_t *launches, double *ms, double *flops,
                            double *bytes);

/* The same launches counted the way the kernels are shaped: every
 * contraction at the padded bond cap K, and the bytes of the kernels' own
 * data flow (padded operands and the intermediate T3 a fused visit hands to
 * the environment update through HBM).  Errors as bbp_kernel_stats. */
bbp_status bbp_kernel_stats_padded(bbp_ctx *c, int32_t cls, double *flops,
                                   double *bytes);
bbp_status bbp_kernel_stats_reset(bbp_ctx *c);

/* Device bytes the context holds now and the most it has held (every
 * buffer it allocated for messages, fits, environments and observables). */
bbp_status bbp_memory(const bbp_ctx *c, size_t *now, size_t *peak);

const char *bbp_last_error(const bbp_ctx *c);
void bbp_destroy(bbp_ctx *c);

/* ------------------------------------------------------------------------
 * The blockBP update (App. B, Eq. (Ut)): one first-order Trotter step of
 * imaginary time evolution of a finite open double-layer PEPS, the
 * environment of every gate taken from the context's block-BP messages.
 *
 * gate (host, d^2 x d^2, row-major [(s0',s1')][(s0,s1)], the first site of
 * a bond the major index) is applied to every nearest-neighbour bond,
 * horizontal bonds row by row (y, then x ascending), then vertical bonds
 * column by column (x, then y ascending); the first site is the left or
 * upper one.  For each bond the two tensors are split into isometries on
 * their outer legs and reduced tensors R_a [k][s][shared], L_b
 * [shared][s][k] (k = min(D^3, d D), QR and LQ); the environment N of the
 * reduced tensors is the normalised two-site reduced density matrix of the
 * network whose two sites carry their isometries (the isometry bond as
 * their physical index, the shared leg at index 0), contracted on the GPU
 * by the same region contraction as bbp_rdm_bonds with the messages the
 * step started from; R_a L_b is then refitted at bond D to the gate applied
 * to it, minimising the distance in the metric of N (bbp_ite_fit), and the
 * two new tensors are scaled to a largest entry of 1 and replace the old
 * ones at once, so that later gates of the step see them.  The messages
 * stay fixed through the step (the caller sweeps between steps); on
 * return the context holds the new tensors with the messages it had
 * (their fit warm starts cleared).  A gate's result depends only on the
 * tensors of its region (its block, or the two blocks its bond joins), so
 * gates whose regions share no block run together: their environments in
 * one batched contraction, their fits on host threads; the result is that
 * of the sequential order.
 *
 * The environment contractions run on a second context that the call
 * creates and destroys, on the context's stream, with the context's
 * allocator and a device budget equal to its "hbm_budget" (if set).
 * n_als: alternating least-squares passes per gate (1..64).  info (host,
 * optional, 5 doubles): the number of gates applied, the sum over the
 * gates of the relative fit error in the metric of N, the seconds spent in
 * the environment contractions (GPU, with their setup), the seconds in the
 * host splits and fits, and the number of levels of gates run together.
 * Errors: BBP_ESTATE (no tensors), BBP_EINVAL (infinite or single-layer
 * context, min(D^3, d D) > 8, n_als out of range, null or non-finite gate),
 * BBP_ENUMERIC (singular fit or a vanishing region contraction); the
 * context then keeps the tensors and messages it had before the step.
 * ------------------------------------------------------------------------ */
bbp_status bbp_ite_step(bbp_ctx *c, const double *gate, int32_t n_als, double *info);

/*
 * The reduced-tensor fit of one gate (App. B), host only: R[k][d][D] and
 * L[D][d][kb] minimising || R L - G Theta || in the metric
 * N[(a,b)][(a',b')] (k kb x k kb), where Theta[k][d][d][kb] is the pair's
 * product and G = gate as in bbp_ite_step.  Starts from the rank-D
 * truncated SVD of G Theta (singular values split evenly, each singular
 * pair signed so that the largest-magnitude entry of its left vector is
 * positive, which fixes the gauge of the bond R L) and makes n_als
 * passes, each solving the normal equations for R, then for L, with N
 * symmetrised and 1e-12 trace(M)/n added to each system's diagonal.
 * *loss (optional): the relative error of the fit in the metric of N.
 * All pointers are host memory owned by the caller.
 * Errors: BBP_EINVAL (d, D outside [1, 8], k, kb outside [1, 64], n_als
 * outside [1, 64], null or non-finite input), BBP_ENUMERIC (singular
 * system or non-finite result).
 */
bbp_status bbp_ite_fit(int32_t d, int32_t D, int32_t k, int32_t kb, const double *N,
                       const double *theta, const double *gate, int32_t n_als,
                       double *R, double *L, double *loss);

/* ------------------------------------------------------------------------
 * One directed message update outside a context: Eq. (1) for a single
 * message, the block contracted with its three other incoming messages
 * column by column, each column an MPO x MPS variational fit truncated to
 * bond chi (App. A), as one step of bbp_sweep computes it.
 *
 * Canonical frame: the receiving block lies to the left of this block.  A
 * holds the block's H x W site tensors in that frame, row-major (y outer, x
 * inner), each [s][u][l][d][r] with every leg stored with dimension D (a
 * sweep rotates the lattice's tensors into this frame for each direction).
 * Messages are open MPSs whose site i is a chi x D^2 x chi slot of doubles,
 * [b_i][(k,k')][b_{i+1}] zero-padded to chi, with true bonds b (n+1 ints, 1
 * at both ends): mt the top message (W sites, left to right), mr the right
 * message (H sites, top to bottom), mb the bottom message (W sites, left to
 * right).  A null message (and its null bond list) is the trivial message of
 * a lattice edge.  The columns are absorbed from W-1 down to 0; each fit
 * starts from the counter-based random state of (seed, slot + column)
 * (a sweep uses slot = 2^40 + 256 e for message e) and makes n_fit full
 * sweeps.
 *
 * Outputs: out (device, H slots) the message m_{A->B}, top to bottom, scaled
 * to unit 2-norm; out_bonds (host, H+1 ints) its bond dimensions;
 * *log_scale (host) the logarithm of the scale removed.  All tensor and
 * message pointers are device pointers (HIP), read and written on
 * hip_stream (NULL: the null stream); the call returns once the update is
 * done.  The caller owns every buffer.
 * Errors: BBP_EINVAL (malformed spec, bonds, null pointers), BBP_ENOMEM,
 * BBP_EDEVICE, BBP_ENUMERIC (a column's fit has zero or non-finite norm;
 * out is then unspecified).  The message is in bbp_update_last_error().
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t H, W;   /* block rows (sites of the message) and columns       */
  int32_t D, d;   /* PEPS bond dimension (<= 8), physical dimension      */
  int32_t chi;    /* message bond cap (<= 128): slots are chi x D^2 x chi */
  int32_t n_fit;  /* full fit sweeps per column (>= 1, App. A)           */
  uint64_t seed;  /* seed of the counter-based fit starts                */
  uint64_t slot;  /* slot base: column c uses slot + c                   */
} bbp_update_spec;

/* Device bytes of the workspace one update of this shape uses. */
bbp_status bbp_update_workspace(const bbp_update_spec *spec, size_t *bytes);

/* The update, with a workspace allocated (hipMalloc) and freed by the call. */
bbp_status bbp_update_message(const bbp_update_spec *spec, const double *A,
                              const double *mt, const int32_t *mt_bonds,
                              const double *mr, const int32_t *mr_bonds,
                              const double *mb, const int32_t *mb_bonds,
                              double *out, int32_t *out_bonds, double *log_scale,
                              void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * update (bitwise the same results) with its workspace in a static device
 * array of BBP_UPDATE_NOALLOC_BYTES that each GPU holds until the process
 * ends; no hipMalloc, hipFree or allocating library routine is called.  The
 * caller still passes the inputs and outputs.  Every call on a GPU shares
 * that GPU's array (the workspace is cleared at the start of each call), so
 * calls that overlap on one GPU race.  A shape whose workspace
 * (bbp_update_workspace) exceeds the array returns BBP_EINVAL. */
#define BBP_UPDATE_NOALLOC_BYTES (64ull << 20)
bbp_status bbp_update_message_noalloc(const bbp_update_spec *spec, const double *A,
                                      const double *mt, const int32_t *mt_bonds,
                                      const double *mr, const int32_t *mr_bonds,
                                      const double *mb, const int32_t *mb_bonds,
                                      double *out, int32_t *out_bonds,
                                      double *log_scale, void *hip_stream);

/* Error message of the calling thread's last failed update call. */
const char *bbp_update_last_error(void);

/* ------------------------------------------------------------------------
 * Request server: independent block-BP solves of finite open lattices
 * (Sec. II; each one the problem bbp_create states) on one GPU with
 * continuous batching.  Infinite lattices are not served: their solve is
 * one block's four self-messages with outputs over the unit cell, a problem
 * of another shape than the request below describes; run it on a context of
 * its own.  Requests are admitted
 * first-in first-out between sweeps while fewer than max_slots are resident
 * and their device-memory estimate (bbp_server_estimate) fits in what
 * budget_bytes leaves free.  Every resident request then sweeps together:
 * one synchronous sweep of all of them is one set of shared batches, every
 * message of every request in the batch of its shape (block size, bond cap,
 * D, d), so one launch of each fit kernel covers every resident solve; the
 * messages stay resident on the device and the fit warm starts are kept
 * when requests join or leave.  A request whose residual drops below tol (or
 * that reaches max_sweeps) has its outputs evaluated on a stream of its own
 * while the others keep sweeping, then frees its memory.  Each result is the
 * same, bitwise, whether its request ran alone or in a mix.
 * ------------------------------------------------------------------------ */
typedef struct bbp_server bbp_server;

typedef struct {
  int32_t Lx, Ly;     /* open lattice, tensors as for bbp_set_tensors      */
  int32_t bx, by;     /* block size (lattice padded with trivial sites)    */
  int32_t D, chi;     /* bond dimension and message bond cap (<= 128)      */
  int32_t max_sweeps; /* sweep cap (>= 1)                                  */
  int32_t outputs;    /* BBP_OUT_* bits                                    */
  int32_t n_site_ops; /* operators of the ops array of bbp_server_submit:  */
  int32_t n_bond_ops; /*   0..16 one-site (2x2), 0..16 two-site (4x4)      */
  double tol;         /* residual target (>= 0)                            */
} bbp_request;

enum { BBP_OUT_SZ = 1, BBP_OUT_SS = 2, BBP_OUT_LOGNORM = 4 };
enum {
  BBP_REQ_QUEUED = 0,
  BBP_REQ_RUNNING = 1,
  BBP_REQ_DONE = 2,
  BBP_REQ_FAILED = 3,
  BBP_REQ_CANCELLED = 4
};

/* Upper bound of the device bytes one request's context allocates.
 * BBP_EINVAL for a malformed request. */
bbp_status bbp_server_estimate(const bbp_request *r, size_t *bytes);

/* budget_bytes > 0; 1 <= max_slots <= 64 concurrent requests. */
bbp_status bbp_server_create(bbp_server **out, size_t budget_bytes, int32_t max_slots);

/* Queues a request; the host tensors A (n doubles, layout of
 * bbp_set_tensors, d = 2) and the operators ops (n_site_ops one-site op[s'][s]
 * of 4 doubles, then n_bond_ops two-site op[(s0',s1')][(s0,s1)] of 16
 * doubles; may be NULL when there are none) are copied.  The observables use
 * chi_env = max(chi, 2 D^2 + 10).  *ticket identifies the request in later
 * calls.  Errors: BBP_EINVAL (malformed request, n, or non-finite
 * operators), BBP_ENOMEM (estimate above the whole budget: it could never be
 * admitted), BBP_ESTATE (server stopping). */
bbp_status bbp_server_submit(bbp_server *s, const bbp_request *r, const double *A, size_t n,
                             const double *ops, int64_t *ticket);

/* State of a request (BBP_REQ_*); times (3 doubles, may be NULL) receive
 * the submit, admit and finish times in seconds since the server was
 * created (0 until reached).  Once BBP_REQ_DONE, out (n >= *needed doubles)
 * receives [converged (1/0), sweeps, last residual, log|Z|, sign of Z,
 * device bytes peak of the request's context, then <sigma_z> of every site
 * (row-major, y outer) if BBP_OUT_SZ, then <S.S> of every horizontal bond
 * (x,y)-(x+1,y) row-major and then of every vertical bond (x,y)-(x,y+1) if
 * BBP_OUT_SS, then for each one-site operator of ops <O> of every site, then
 * for each two-site operator <O> of every bond in the same order]; log|Z|
 * and the sign are 0 unless BBP_OUT_LOGNORM.  Errors: BBP_EINVAL (unknown
 * ticket, or out too short). */
bbp_status bbp_server_poll(bbp_server *s, int64_t ticket, int32_t *state, double *out, size_t n,
                           size_t *needed, double *times);

/* Cancels a queued request at once, a running one before its next sweep. */
bbp_status bbp_server_cancel(bbp_server *s, int64_t ticket);

/* Requests admitted and not finished (sweeping or evaluating outputs) and
 * queued now, the estimated bytes admitted now, and the most requests that
 * have been admitted at the same time. */
bbp_status bbp_server_stats(bbp_server *s, int32_t *running, int32_t *queued,
                            size_t *bytes_in_use, int32_t *max_running);

/* Shared sweeps run so far, the request sweeps they covered (summed over
 * the requests of each), the most requests one shared sweep covered, and
 * (busy, 3 doubles, may be NULL) the seconds spent in shared sweeps, in
 * admitting requests (contexts, tensor uploads), and in evaluating outputs
 * (summed over the finisher threads). */
bbp_status bbp_server_sweeps(bbp_server *s, int64_t *sweeps, int64_t *request_sweeps,
                             int32_t *max_together, double *busy);

/* Why a request failed (empty string otherwise); valid until destroy. */
const char *bbp_server_error(bbp_server *s, int64_t ticket);

/* Cancels what is queued or running, joins the workers, frees everything. */
void bbp_server_destroy(bbp_server *s);

#ifdef __cplusplus
}
#endif
#endif /* BBP_H */
