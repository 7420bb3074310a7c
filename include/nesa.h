/*
 * nesa.h -- C ABI of the MI355X NESA EFIE library.
 *
 * The library builds, once, the nested equivalent source approximation (NESA)
 * of the Galerkin EFIE matrix of a closed PEC surface meshed with triangles,
 * and applies it on one GPU (gfx950) at every iteration of a GMRES solve.
 * Operation names follow the paper (Zafari et al., "Task parallel
 * implementation of a solver for electromagnetic scattering problems"):
 *
 *   Sec. 2, Eq. (1)-(3)   EFIE, Galerkin testing, dense system Z j = b
 *   Sec. 2, Eq. (4)-(7)   Z_far ~ U B..B D C..C V over an oct-tree
 *   Sec. 3, Eq. (9)       near-field product
 *   Sec. 3, Eq. (10)-(14) radiation, source transfer, translation,
 *                         potential transfer, reception
 *   Sec. 2 / Sec. 5       the product is applied many times inside an
 *                         iterative solver while the structure is built once
 *
 * Conventions
 *   - Lengths are in wavelengths; k = 2 pi; eta = 376.730313668 ohm.
 *   - Unknowns are RWG functions on the interior edges of the mesh, numbered in
 *     increasing (min vertex, max vertex) order ("canonical order"); the plus
 *     triangle of an edge is the lower-index one.
 *   - Complex vectors are interleaved (re, im) pairs: complex128 (double2) in
 *     NESA_C128 mode, complex64 (float2) otherwise.  Vectors of several
 *     right-hand sides are stored RHS-major: x[r * n + i].
 *   - Pointers named *_dev are device pointers on the current HIP device;
 *     the caller owns them.  Handles are owned by the library and released
 *     with the matching *_free call.  `stream` is a hipStream_t (NULL = the
 *     default stream); calls enqueue work on it and return without waiting,
 *     except where stated.
 *   - Every call returns a nesa_status; on failure nesa_last_error() gives a
 *     message (thread-local).  No exception crosses the ABI.
 */
#ifndef NESA_H
#define NESA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NESA_OK = 0,
  NESA_EINVAL = -1,      /* bad argument (null pointer, size, parameter) */
  NESA_ENOMEM = -2,      /* host or device allocation failed */
  NESA_EHIP = -3,        /* a HIP runtime call failed */
  NESA_EMESH = -4,       /* mesh is not a closed 2-manifold, or too coarse */
  NESA_ENOCONV = -5,     /* GMRES stopped at max_iters above tolerance */
  NESA_EBREAKDOWN = -6,  /* non-finite value in the solver */
  NESA_ENOTIMPL = -7
} nesa_status;

typedef enum {
  NESA_C128 = 0,         /* complex FP64 storage and arithmetic */
  NESA_C64 = 1,          /* complex FP32 storage and arithmetic */
  NESA_C64_SPLIT = 2,    /* complex FP32 vectors; translation and aggregation
                            contractions as split-bf16 (hi*hi + hi*lo + lo*hi)
                            matrix-core products with FP32 accumulation */
  NESA_C64_SPLIT_FP16 = 3 /* as NESA_C64_SPLIT with fp16 parts (11-bit
                            mantissas, about 22 bits per operand): each
                            matrix family and each level's sources or
                            potentials carry one power-of-two scale that puts
                            their largest part below 2^14 (the sources' scale
                            is found on the device in every product) */
} nesa_precision;

typedef struct nesa_tree nesa_tree;
typedef struct nesa_near nesa_near;
typedef struct nesa_far nesa_far;
typedef struct nesa_op nesa_op;

/* Oct-tree parameters (Sec. 2 partition, Sec. 3 level rules).
 *   leaf_size: leaf box side in wavelengths (> 0); L = ceil(log2(longest
 *     bounding-box side / leaf_size)), root cube anchored 1e-9 below the
 *     vertex bounding-box minimum.
 *   l0_max: coarsest far level is min(l0_max, L) (2 = four boxes along the
 *     root side, the rule of Sec. 3; larger values start the far field at
 *     finer boxes, which bounds the equivalent sources per box on bodies many
 *     wavelengths long; at most 6).
 *   buffer: near boxes are those at Chebyshev index distance <= buffer
 *     (1 = adjacent boxes including diagonal ones and the box itself). */
typedef struct {
  double leaf_size;
  int l0_max;
  int buffer;
} nesa_tree_params;

/* Medium: wavenumber k and impedance eta (Sec. 2, Eq. 1). */
typedef struct {
  double k;
  double eta;
} nesa_em_params;

/* Far-field operator construction (Sec. 2, Eq. 4-7: equivalence on
 * fictitious spheres around the boxes).
 *   d0: accuracy digits of the per-level equivalent-source count
 *     Q_l = (ceil(kr + 1.8 d0^(2/3) (kr)^(1/3)) + 1)^2, r = (sqrt3/2) a_l.
 *   q_min: lower bound on Q_l (0 = none).
 *   tau: Tikhonov parameter of the fitting operator, relative to the largest
 *     singular value of G(check points, equivalent points).
 *   eps: the equivalent points of a box sit on the complex radius
 *     r_e (1 + i eps) (complex source points, distance = principal square root
 *     of the summed squared coordinate differences); 0 gives real points,
 *     which lose accuracy on every box whose k r_e is near a zero of a
 *     spherical Bessel function j_n.  Range [0, 1); 0.1 is the usual value. */
typedef struct {
  int d0;
  int q_min;
  double tau;
  double eps;
} nesa_far_params;

typedef struct {
  int64_t n_rwg;
  int64_t n_tri;
  int L;                 /* leaf level */
  int l0;                /* coarsest far level */
  int64_t n_box[32];     /* boxes at level l0 + i, i = 0 .. L - l0 */
  int64_t near_entries;  /* stored near-field matrix entries */
  int64_t n_pairs[32];   /* translation pairs at level l0 + i */
  int Q[32];             /* equivalent sources per box at level l0 + i
                            (0 until nesa_assemble_translations) */
  int64_t max_leaf;      /* RWGs of the largest leaf */
  int64_t near_entries_half;  /* entries of the blocks Z_ab with b >= a (leaf order):
                                 what the single-RHS product stores and reads,
                                 Z_ba = Z_ab^T being the Galerkin EFIE's reciprocity */
  int64_t near_transposed;    /* outputs Z_ab^T x_a (b > a) that the single-RHS
                                 product writes and reads back per product */
} nesa_tree_info;

/* Build the RWG basis and the oct-tree of a closed triangle mesh.
 *   verts: host [nv][3] doubles (wavelengths); tris: host [nt][3] int32,
 *   vertex ids; orientation is irrelevant.  Returns NESA_EMESH if an edge is
 *   not shared by exactly two triangles.  Host-only; copies its inputs. */
int nesa_build_tree(const double* verts, int64_t nv, const int32_t* tris, int64_t nt,
                    const nesa_tree_params* params, nesa_tree** out);
/* Several closed meshes in one tree structure (batching of bodies; not in
 * the paper, whose setting is one scatterer).  Body i keeps the partition
 * rules of nesa_build_tree on its own grid; the levels of all bodies are
 * aligned at the leaf level (same box side at every level), so one launch
 * per stage serves every body, and the equivalent-source spheres of a level
 * are shared (radius = the largest any body needs).  RWGs are numbered body
 * by body (canonical order of body 0, then body 1, ...), leaves likewise;
 * bodies do not interact (the operator is block-diagonal over bodies).
 * verts[i], tris[i]: host arrays of body i as in nesa_build_tree. */
int nesa_build_forest(int nbodies, const double* const* verts, const int64_t* nv, const int32_t* const* tris,
                      const int64_t* nt, const nesa_tree_params* params, nesa_tree** out);
/* Number of bodies and the canonical RWG range of each:
 * rwg_ptr[i] .. rwg_ptr[i + 1] (host [nbodies + 1], nullable; at most nmax
 * values written).  A tree from nesa_build_tree has one body. */
int nesa_tree_bodies(const nesa_tree* tree, int64_t* rwg_ptr, int nmax, int* nbodies);
int nesa_tree_get_info(const nesa_tree* tree, nesa_tree_info* info);
/* perm[i] = canonical RWG index of leaf-order position i (host [n_rwg]). */
int nesa_tree_perm(const nesa_tree* tree, int64_t* perm);
/* Per leaf a (leaf order, host [n_box[L - l0]] each, either nullable): S[a] =
 * RWGs of leaf a, W[a] = RWGs of its near leaves (Sec. 3, the near field of
 * Eq. 9: leaf a's near block is S[a] x W[a], sum S W = near_entries). */
int nesa_tree_leaf_sizes(const nesa_tree* tree, int64_t* S, int64_t* W);
void nesa_tree_free(nesa_tree* tree);

/* Near-field Galerkin blocks Z_ab, b in the near list of leaf a (Sec. 2;
 * Sec. 3, Eq. 9), computed on the host with the 3-point triangle rule and
 * closed-form static singular integrals for triangle pairs that share a
 * vertex (mean of both integration orders, so Z = Z^T).  Host-only. */
int nesa_assemble_near(const nesa_tree* tree, const nesa_em_params* em, nesa_near** out);
/* The same blocks computed on the current device: one thread per entry, FP64,
 * the same integration rules and summation order (entries agree with
 * nesa_assemble_near up to the rounding of the device's math functions), copied
 * back into a host handle that every consumer of nesa_assemble_near's accepts.
 * Device memory: 16 bytes per entry plus the mesh, freed before returning.
 * Errors: NESA_EINVAL (null pointer, k or eta not positive, a near list longer
 * than 128), NESA_EHIP. */
int nesa_assemble_near_device(const nesa_tree* tree, const nesa_em_params* em, nesa_near** out);
/* Copy the entries Z[rows[i]][cols[j]] (canonical indices, both RWGs in near
 * leaves) into host out[i * ncols + j] (complex128); missing entries -> 0. */
int nesa_near_entries(const nesa_tree* tree, const nesa_near* near, const int64_t* rows,
                      int64_t nrows, const int64_t* cols, int64_t ncols, double* out);
void nesa_near_free(nesa_near* near);

/* Far-field operators (Sec. 2, Eq. 4-7): per level the equivalent and check
 * points and the Tikhonov fitting operator, and the transfer matrices C (and
 * B = C^T); the fits and C are computed in FP64 on the current device when
 * there is one (environment NESA_FIT_HOST=1, NESA_C_HOST=1: on the host; the
 * results agree to rounding), on the host otherwise, and copied into the host
 * handle.  The radiation matrices V (U = V^T) and the translation matrices D
 * are assembled on the device by nesa_op_create from what this call records
 * (the finest level's fitting operator, the points, the offsets that occur).
 * Errors: NESA_EINVAL for bad parameters, NESA_EMESH for a mesh too coarse for
 * the leaf size, NESA_EHIP when a device call fails, NESA_ENOMEM. */
int nesa_assemble_translations(const nesa_tree* tree, const nesa_em_params* em,
                               const nesa_far_params* params, nesa_far** out);
/* Q of every level l0..L into Q[0 .. nmax-1]. */
int nesa_far_get_q(const nesa_far* far, int* Q, int nmax);
void nesa_far_free(nesa_far* far);

/* Upload near and far operators to the current device in the given precision
 * (nesa_precision; EINVAL for any other value), assemble V and D there, and
 * allocate work buffers for up to max_nrhs right-hand sides.  Products of one
 * right-hand side read the near field in reciprocity half storage (the blocks
 * Z_ab of near leaves b >= a, Z_ba = Z_ab^T); the full blocks are uploaded as
 * well when max_nrhs > 1.  Split precisions also keep the 16-bit planes of the
 * translation and transfer matrices, and per level a buffer for the sources
 * split once per product (4 max_nrhs x Q rounded up to 32 values per box). */
int nesa_op_create(const nesa_tree* tree, const nesa_near* near, const nesa_far* far,
                   int precision, int max_nrhs, nesa_op** out);
void nesa_op_free(nesa_op* op);

/* y = Z_NESA x for nrhs right-hand sides (1 <= nrhs <= max_nrhs), x and y in
 * canonical order, RHS-major.  Applies the near-field product (Eq. 9) and the
 * five far-field stages (Eq. 10-14) with GPU kernels on `stream`; the near field
 * and the finest level's translations run on two streams of the operator forked
 * from `stream` and joined back into it, so the call is ordered on `stream` as
 * a whole (also under HIP graph capture).  Products on one operator share its
 * work buffers: calls that overlap in time race. */
int nesa_matvec(nesa_op* op, const void* x_dev, void* y_dev, int64_t nrhs, void* stream);

/* Products of several operators in one call (batching, not in the paper: its
 * Sec. 5.1 suggests letting one task handle several groups): y_i = Z_i x_i for
 * operator ops[i] with nrhs[i] right-hand sides (canonical order, RHS-major),
 * i < n_ops.  The products of different operators are independent and run side
 * by side on the library's worker streams (four per device, forked from and
 * joined back into `stream`, so the call is ordered on `stream` as a whole).
 * An operator may appear once (NESA_EINVAL otherwise: its buffers would race);
 * arguments are checked before any work is queued.  (Bodies that share one tree
 * are better batched as a forest, nesa_build_forest: one launch per stage for
 * all of them.) */
int nesa_matvec_batched(nesa_op* const* ops, int n_ops, const void* const* x_dev, void* const* y_dev,
                        const int64_t* nrhs, void* stream);

/* Same product in leaf order (no permutation), for callers that keep their
 * vectors in the order of nesa_tree_perm. */
int nesa_matvec_leaf(nesa_op* op, const void* x_dev, void* y_dev, int64_t nrhs, void* stream);

/* One product (nrhs = 1, leaf order) with hipEvents recorded between the
 * stages on `stream`; blocks, then writes the elapsed milliseconds of
 * ms[0] radiation (Eq. 10), ms[1] source transfer (Eq. 11), ms[2] translation
 * (Eq. 12), ms[3] potential transfer (Eq. 13), ms[4] near field + reception
 * (Eq. 9, 14). */
int nesa_matvec_phase_times(nesa_op* op, const void* x_dev, void* y_dev, void* stream, float* ms);

/* One product (nrhs = 1, leaf order) with a hipEvent after every kernel
 * launch; blocks, then writes for each launch i < *count (at most
 * max_launches): its duration ms[i], its kind[i] (1 radiation, 2 upward GEMM,
 * 3 upward sum, 4 upward (FP64), 5 translation GEMM, 6 translation sum,
 * 7 translation (FP64), 8 downward GEMM, 9 downward (FP64), 10 near field +
 * reception) and the tree level[i] it works on. */
int nesa_matvec_launch_times(nesa_op* op, const void* x_dev, void* y_dev, void* stream, float* ms,
                             int32_t* kind, int32_t* level, int32_t max_launches, int32_t* count);
/* The same for nrhs right-hand sides in leaf order (RHS-major; complex64 and
 * split operators; nrhs = 1 is nesa_matvec_launch_times). */
int nesa_matvec_launch_times_nrhs(nesa_op* op, const void* x_dev, void* y_dev, int64_t nrhs, void* stream,
                                  float* ms, int32_t* kind, int32_t* level, int32_t max_launches,
                                  int32_t* count);

/* Plane-wave right-hand sides b_m = -<e_inc, phi_m> (Sec. 2, Eq. 2),
 * e_inc = pol exp(-i k khat.r); khat, pol: host [nrhs][3].  Writes device b
 * in canonical order, RHS-major, in the op's vector precision. */
int nesa_rhs_plane_wave(nesa_op* op, const double* khat, const double* pol, int64_t nrhs,
                        void* b_dev, void* stream);

/* Host version of the right-hand side: b (host, complex128 interleaved,
 * [nrhs][n_rwg], canonical order). */
int nesa_rhs_plane_wave_host(const nesa_tree* tree, double k, const double* khat, const double* pol,
                             int64_t nrhs, double* b);

/* Preconditioners (right, inside flexible GMRES):
 *   BLOCKDIAG  z_a = Z_aa^-1 r_a with Z_aa the near-field self block of leaf a;
 *   SCHWARZ    restricted additive Schwarz over the near lists: z_a = rows of
 *              leaf a of Z_N^-1 r_N, Z_N the near-field matrix restricted to
 *              the RWGs of the near list of a (setup on the host at first use);
 *   LEARNED    a base preconditioner (BLOCKDIAG or SCHWARZ) plus the
 *              correction of the per-leaf network attached with
 *              nesa_op_set_mlp; falls back to the base when a restart cycle
 *              does not reduce the true residual or yields a non-finite value
 *              (that cycle is then discarded). */
typedef enum { NESA_PRECOND_NONE = 0, NESA_PRECOND_BLOCKDIAG = 1, NESA_PRECOND_LEARNED = 2,
               NESA_PRECOND_SCHWARZ = 3 } nesa_precond;

/* Build the data of a preconditioner now instead of at its first use. */
int nesa_precond_setup(nesa_op* op, int precond);
/* z = M r for one vector in leaf order (BLOCKDIAG or SCHWARZ), on `stream`. */
int nesa_precond_apply(nesa_op* op, int precond, const void* r_dev, void* z_dev, void* stream);

/* Restarted GMRES(m) (flexible when a preconditioner is used) around the
 * NESA product: Arnoldi with two passes of classical Gram-Schmidt, FP64 dot
 * products, norms, Hessenberg matrix and Givens rotations; stop when the
 * estimated relative residual <= tol, confirmed by the true residual
 * ||b - Z_NESA x|| / ||b|| recomputed at every restart and at exit. */
typedef struct {
  int restart;           /* m */
  int max_iters;
  double tol;
  int precond;           /* nesa_precond */
  double fallback_ratio; /* LEARNED: a restart cycle whose true residual is
                            above fallback_ratio x the previous one hands over
                            to the base preconditioner (0 means 1: only a cycle
                            that does not reduce it) */
} nesa_gmres_params;

typedef struct {
  int iters;
  int restarts;
  double true_rel_residual;
  double seconds;
  int fell_back;         /* learned preconditioner replaced by its base */
} nesa_gmres_report;

/* Solve Z_NESA x = b for nrhs right-hand sides (each its own Krylov space).
 * b_dev, x_dev: canonical order, RHS-major; x_dev holds x0 on entry.
 * Complex64 operators with nrhs > 1 run the right-hand sides in lock step: each
 * iteration every unconverged one takes one Arnoldi step of its own restart
 * cycle and their vectors go through one multi-RHS product (report.seconds is
 * then the wall time of the whole batch); complex128 solves them one by one.
 * history (host, nullable): estimated relative residual after each iteration
 * of RHS 0, up to history_len values.  Blocks until the solve ends. */
int nesa_gmres_solve(nesa_op* op, const void* b_dev, void* x_dev, int64_t nrhs,
                     const nesa_gmres_params* params, nesa_gmres_report* report,
                     double* history, int64_t history_len, void* stream);

/* For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid hipMalloc): the same solve as nesa_gmres_solve, right-hand sides
 * one at a time (same arithmetic as its nrhs = 1 form, so the same iterates),
 * with every work buffer taken from one fixed device array of
 * NESA_NOALLOC_SCRATCH_BYTES per device, held from library load to process end,
 * and the per-iteration host scalars from thread-local storage.  The call
 * makes no hipMalloc, hipFree, hipHostMalloc or other allocating call.
 * Workspace: 8 (complex64) or 16 (complex128) bytes x n x (m + 5, plus m when
 * a preconditioner is used), plus under 1 MiB; a larger request returns
 * NESA_EINVAL without touching the device.  A Schwarz preconditioner must have
 * been built by nesa_precond_setup and a learned one attached beforehand
 * (NESA_EINVAL otherwise).  Every call on a device shares that device's array
 * and leaves its contents behind: calls that overlap in time on one device
 * (any thread, any stream, any operator) race and are not allowed.  The solve
 * synchronises `stream` once per iteration, so it cannot be captured in a HIP
 * graph as a whole. */
#define NESA_NOALLOC_SCRATCH_BYTES (256u << 20)
int nesa_gmres_solve_noalloc(nesa_op* op, const void* b_dev, void* x_dev, int64_t nrhs,
                             const nesa_gmres_params* params, nesa_gmres_report* report,
                             double* history, int64_t history_len, void* stream);

/* Learned per-leaf preconditioner network (no counterpart in the paper,
 * which does not precondition; flexible GMRES after Saad 1993).
 *   features of leaf a for a vector r and the base output b = M_base r
 *   (leaf order, S_a RWGs of the leaf, zero padded to s_max):
 *     u = [Re r_a, Im r_a] / ||r_a||, [Re b_a, Im b_a] / ||b_a||   (4 s_max;
 *     a block whose norm is zero is zero);
 *   network, weights shared by all leaves, FP16 weights and activations with
 *   FP32 accumulation on the matrix cores, FP32 biases:
 *     y = W3 relu(W2 relu(W1 u + c1) + c2) + c3,
 *     W1 [hidden][4 s_max], W2 [hidden][hidden], W3 [2 s_max][hidden];
 *   z_a = b_a + ||b_a|| (y[0:S_a] + i y[s_max:s_max+S_a]).
 * Parameters: FP32 host vector W1, c1, W2, c2, W3, c3 (row-major, in this
 * order; nesa_mlp_num_params gives the length).  With W3 = 0 and c3 = 0 the
 * network is its base preconditioner.
 * Training pairs (r, e) satisfy Z_NESA e = r (residuals and errors of the
 * method's own solves); target of leaf a: (e_a - b_a) / ||b_a||; loss = mean
 * over leaves with ||b_a|| > 0 of the squared error on the S_a valid entries;
 * the optimiser is Adam with bias correction (FP32 master weights). */
typedef struct nesa_mlp nesa_mlp;
typedef struct {
  int s_max;             /* multiple of 32 in [32, 512], >= the largest leaf */
  int hidden;            /* multiple of 64 in [64, 512] */
  int base;              /* NESA_PRECOND_BLOCKDIAG or NESA_PRECOND_SCHWARZ */
} nesa_mlp_params;
typedef struct {
  double lr, beta1, beta2, eps;
} nesa_adam_params;

int nesa_mlp_num_params(const nesa_mlp_params* params, int64_t* count);
/* Network for the leaves of `op` with initial parameters theta0 (host).
 * Freeing op first leaves the network usable only for nesa_mlp_free and the
 * parameter calls. */
int nesa_mlp_create(nesa_op* op, const nesa_mlp_params* params, const float* theta0, nesa_mlp** out);
void nesa_mlp_free(nesa_mlp* net);
/* Training pair of an iterate x of a solve with converged solution xs:
 * r = b - Z_NESA x and e = xs - x (so Z_NESA e = r up to the solve
 * tolerance).  One vector each, device, canonical order; r and e must not
 * alias the inputs. */
int nesa_residual_error(nesa_op* op, const void* b_dev, const void* xs_dev, const void* x_dev, void* r_dev,
                        void* e_dev, void* stream);
/* Replace the parameters (host FP32) and reset the optimiser state. */
int nesa_mlp_set_params(nesa_mlp* net, const float* theta);
int nesa_mlp_get_params(const nesa_mlp* net, float* theta);
/* Save the network's parameters (FP32), s_max, hidden and base to a file;
 * nesa_mlp_load creates a network for `op` from such a file (as
 * nesa_mlp_create with those values).  Layout: the 8 bytes "NESAMLP1", int32
 * s_max, hidden, base, int64 parameter count, the FP32 parameters (host byte
 * order).  Errors: NESA_EINVAL (null argument, file not writable / readable,
 * not such a file, sizes that nesa_mlp_create rejects). */
int nesa_mlp_save(const nesa_mlp* net, const char* path);
int nesa_mlp_load(nesa_op* op, const char* path, nesa_mlp** out);
/* Training set: nsamples pairs (r, e), device, canonical order, sample-major
 * [nsamples][n_rwg], in the op's vector precision.  The base preconditioner is
 * applied to every r here; features and targets stay on the device. */
int nesa_mlp_set_data(nesa_mlp* net, const void* r_dev, const void* e_dev, int64_t nsamples, void* stream);
/* `steps` full-batch Adam steps; loss_history (host, nullable) gets the loss
 * before each step. */
int nesa_mlp_train(nesa_mlp* net, const nesa_adam_params* adam, int steps, double* loss_history, void* stream);
/* Loss and gradient (host FP32, parameter order) at the current parameters. */
int nesa_mlp_gradient(nesa_mlp* net, float* grad, double* loss);
/* Network outputs y of the training rows (host [nsamples * n_leaf][2 s_max],
 * row = sample * n_leaf + leaf). */
int nesa_mlp_outputs(nesa_mlp* net, float* y);
/* z = M_base r + correction for one vector in leaf order, on `stream`. */
int nesa_mlp_apply(nesa_mlp* net, const void* r_dev, void* z_dev, void* stream);
/* Network used by NESA_PRECOND_LEARNED (NULL detaches; not owned by op). */
int nesa_op_set_mlp(nesa_op* op, nesa_mlp* net);

const char* nesa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NESA_H */
