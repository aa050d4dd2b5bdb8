/*
 * lsp.h -- C ABI of the lattice-spline evaluation library (gfx950).
 *
 * The library evaluates the lattice convolution sum
 *
 *     f(x) = sum over lattice sites n in L Z^s of  c_n * phi(x - n)
 *
 * (Sec. 1, Eq. 1) at many query points, in the unrolled sub-region form of
 * Sec. 4 (Algorithm 1): locate the region of evaluation and the sub-region,
 * apply the symmetry transform to the reference sub-region, fetch the stencil
 * coefficients and evaluate the reference polynomial in Horner form.
 *
 * Conventions shared by every entry point:
 *   * Everything is extern "C"; no C++ exception crosses the boundary.
 *   * Argument errors are detected on the host, synchronously, before any
 *     work is queued; the call then returns a status other than LSP_OK and
 *     `lsp_last_error()` (thread-local) holds a human-readable detail.
 *   * Device work is queued asynchronously on the caller's `stream` (0 means
 *     the null stream); a launch failure returns LSP_E_HIP.
 *   * Pointers documented as "device" must be device-accessible memory of the
 *     current HIP device; "host" pointers are read before the call returns.
 *   * The caller owns every buffer it passes in; the library never frees
 *     them.  The library owns its handles and the internal coefficient
 *     buffer of a volume; each is released by the matching *_destroy call.
 *   * lsp_eval, lsp_eval_grad, lsp_eval_hessian and lsp_backward allocate nothing: scratch
 *     space of the backward pass is a caller-provided workspace.
 *   * Handles are immutable between lsp_volume_set_coeffs calls, so several
 *     threads or streams may evaluate one volume concurrently.
 *
 * Coefficient layout (the memory lookup of Sec. 4.1: one array per Cartesian
 * coset of the lattice).  A lattice L Z^3 is stored as n_cosets Cartesian
 * cosets; coset m holds the sites n = D * (i, j, k) + shift_m with
 * 0 <= i < dims[0], 0 <= j < dims[1], 0 <= k < dims[2], in C order [k][j][i]
 * (i fastest).  Sites outside this range are taken as zero (zero padding).
 *   Z^3  (L = I):                        1 coset,  D = 1
 *   BCC  (L Z^3 = 2Z^3 u 2Z^3+(1,1,1)):  2 cosets, D = 2, shifts (0,0,0),(1,1,1)
 *   FCC  (L Z^3 = {n : n_x+n_y+n_z even}): 4 cosets, D = 2,
 *        shifts (0,0,0),(1,1,0),(1,0,1),(0,1,1)
 *
 * The basis function is phi(y) = |det L| * M_Xi(y + Xi*1/2): the box spline
 * of the direction matrix Xi, centred, and scaled so that its lattice
 * translates sum to one.
 */
#ifndef LSP_H
#define LSP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lsp_status {
    LSP_OK = 0,
    LSP_E_INVALID_ARG = 1,  /* null pointer, negative size, bad enum value */
    LSP_E_UNSUPPORTED = 2,  /* (L, Xi) pair for which no code was generated */
    LSP_E_DTYPE = 3,        /* dtype not accepted for this argument */
    LSP_E_SHAPE = 4,        /* sizes out of the supported range */
    LSP_E_WORKSPACE = 5,    /* workspace missing or smaller than required */
    LSP_E_HIP = 6,          /* a HIP runtime call or kernel launch failed */
    LSP_E_OOM = 7           /* device allocation failed */
} lsp_status;

typedef enum lsp_dtype {
    LSP_F32 = 0,
    LSP_F64 = 1,
    LSP_BF16 = 2,
    LSP_F16 = 3
} lsp_dtype;

typedef struct lsp_spline lsp_spline;  /* opaque: (L, Xi) and its generated code */
typedef struct lsp_volume lsp_volume;  /* opaque: a spline plus bound coefficients */

typedef struct lsp_spline_info {
    int s;                 /* dimension (3) */
    int kind;              /* 0 tricubic on Z^3, 1 BCC 8-direction, 2 FCC 6-direction,
                              3 trilinear, 4 BCC linear (4-direction), 5 triquadratic,
                              6 Z^3 7-direction, 7 BCC quartic (7-direction),
                              8 Z^3 face diagonals (6-direction) */
    int n_cosets;          /* Cartesian cosets of the lattice */
    int D[3];              /* coset scale */
    int shift[4][3];       /* coset shifts (first n_cosets rows used) */
    int taps;              /* stencil size of one reference sub-region */
    int union_taps;        /* union of the reference sub-regions' stencils */
    int n_reference;       /* reference sub-regions (polynomials) */
    int degree;            /* total degree of the reference polynomials */
    int radius;            /* max |component| of a stencil offset, lattice units */
    int fma_eval;          /* FMAs of the generated value code, per point */
    int pad;               /* zero halo of the internal layout, coset units */
    int continuity;        /* phi is C^continuity: the fewest directions whose
                              removal leaves Xi not spanning, minus 2 (Sec. 2) */
} lsp_spline_info;

/* Human-readable name of a status; never NULL. */
const char* lsp_status_string(lsp_status st);

/* Detail of the last error raised on the calling thread ("" if none). */
const char* lsp_last_error(void);

/* Library version string. */
const char* lsp_version(void);

/*
 * Process-wide evaluation options (take effect for launches issued after the
 * call; not synchronised with launches in flight on other threads).
 *   LSP_OPT_MFMA: how the monomial coefficients A = W c of one-sub-region
 *     splines with more than 16 taps (the BCC 8-direction and quartic
 *     splines) are formed: 0 (default, or the value of LSP_MFMA in the
 *     environment) per-lane FMAs over the generated shared-term form of W,
 *     1 matrix cores (MFMA) for every coefficient storage, 2 matrix cores for
 *     BF16/FP16 storage and FMAs for FP32.  Every setting gives results
 *     within the FP32 tolerance of the convolution sum; other splines, the
 *     dL/dx pass and batch plans always use per-lane FMAs.
 *   LSP_OPT_PREDICATED: how a spline with two reference sub-region
 *     polynomials (the FCC 6-direction spline) picks its polynomial in
 *     lsp_eval, lsp_eval_grad and lsp_eval_hessian: 0 (default, or
 *     LSP_FCC_PREDICATED=1 in the environment for 1) a branch per point, 1
 *     evaluate both and select (the branch-free form of Sec. 5.1).  Both give
 *     the same values up to rounding; the binned, backward and batch paths
 *     always branch.
 *   LSP_OPT_SPLIT_MAXN: lsp_eval, lsp_eval_grad and the dL/dx of
 *     lsp_backward for the separable
 *     splines (trilinear, triquadratic, tricubic) use four lanes per point,
 *     one per z-slab of the stencil, when N is at most this count (0 never;
 *     -1, the default unless LSP_SPLIT_MAXN is set in the environment,
 *     restores each spline's own measured limit: always for tricubic, 2^18
 *     points for triquadratic, 2^17 for trilinear).  Four times the
 *     wavefronts hide the gather latency.  Results agree with the one-lane
 *     kernel up to the order of the last additions.
 * Returns LSP_E_INVALID_ARG for an unknown option or value.
 */
#define LSP_OPT_MFMA 1
#define LSP_OPT_PREDICATED 2
#define LSP_OPT_SPLIT_MAXN 3
lsp_status lsp_set_option(int option, int value);

/* --------------------------------------------------------------- splines */

/*
 * Create the spline of a lattice and a box-spline direction matrix
 * (the pair (L, Xi) that Sec. 3 takes as the description of a shift-invariant
 * space).
 *   s       dimension; only 3 is supported.
 *   L       host, s*s int32, row-major; the COLUMNS are the lattice
 *           generators.  Any basis of the same lattice is accepted.
 *   Xi      host, s*n_dirs int32, row-major; the COLUMNS are the directions.
 *           Direction order and signs do not matter (phi is centred).
 *   out     receives a handle owned by the caller (lsp_spline_destroy).
 * Supported pairs (the box splines of Sec. 5.1's comparisons): Z^3 with
 * Xi = [I I] (trilinear), [I I I] (triquadratic), [I I I I] (tricubic) and
 * [I, the four diagonals (+-1,+-1,+-1)] (7-direction, fourth order); the BCC
 * lattice with its four diagonals once (linear), twice (8-direction) or with
 * 2I (quartic, 7-direction); the FCC lattice with the six directions
 * (1,+-1,0), (1,0,+-1), (0,1,+-1); Z^3 with the same six face diagonals.
 * Anything else returns LSP_E_UNSUPPORTED.  Host only; touches no device.
 */
lsp_status lsp_spline_create(int s, const int32_t* L, const int32_t* Xi, int n_dirs,
                             lsp_spline** out);

/*
 * A spline compiled at run time (the analogue of the paper's just-in-time
 * code generation, Sec. 3.3): `path` names a shared library built from the
 * generated code of one (L, Xi) pair together with this library's kernel
 * headers (paper_2102_08518_amd.jit builds them).  It must export
 * lsp_plugin_describe and lsp_plugin_eval of the same library version.  The
 * plugin stays loaded until the process ends.  Volumes of such a spline
 * support lsp_volume_*, lsp_eval, lsp_eval_grad, lsp_eval_hessian and the
 * dL/dx of lsp_backward; the binned order, dL/dc and batch plans return
 * LSP_E_UNSUPPORTED.  Host only.
 *   path    host, NUL-terminated file name.
 *   out     receives a handle owned by the caller (lsp_spline_destroy).
 * Returns LSP_E_UNSUPPORTED if the file cannot be loaded, lacks the entry
 * points or was built for another version.
 */
lsp_status lsp_spline_load_plugin(const char* path, lsp_spline** out);
void lsp_spline_destroy(lsp_spline* sp);
/* Fill `out` (host) with the spline's description.  Host only. */
lsp_status lsp_spline_get_info(const lsp_spline* sp, lsp_spline_info* out);

/* --------------------------------------------------------------- volumes */

/*
 * Create a volume: the spline plus an internal, zero-padded device buffer of
 * n_cosets * dims[0]*dims[1]*dims[2] coefficients stored as `storage`
 * (LSP_F32, LSP_BF16 or LSP_F16; FP32 evaluation in every case).  The buffer
 * is allocated on the current device and zero-filled before return.
 *   dims    host, 3 int64, per-coset extent (X, Y, Z), each in [1, 2^20], with
 *           the padded internal buffer below 2^31 bytes (the halo is a few
 *           sites per side; see lsp_spline_info.pad).
 * The volume keeps a reference to nothing the caller owns; the spline handle
 * may be destroyed afterwards.
 */
lsp_status lsp_volume_create(const lsp_spline* sp, const int64_t dims[3], lsp_dtype storage,
                             lsp_volume** out);
void lsp_volume_destroy(lsp_volume* vol);
lsp_status lsp_volume_info(const lsp_volume* vol, lsp_spline_info* spline, int64_t dims[3],
                           lsp_dtype* storage);

/*
 * Load coefficients.  coset_ptrs: host array of n_cosets DEVICE pointers, each
 * to dims[2]*dims[1]*dims[0] values of dtype `src` (F32, F64, BF16 or F16) in
 * C order [k][j][i].  They are converted (round to nearest even) to the
 * storage dtype and packed into the volume's internal layout on `stream`.
 * The source buffers must stay valid until that work has run.
 */
lsp_status lsp_volume_set_coeffs(lsp_volume* vol, const void* const* coset_ptrs, lsp_dtype src,
                                 hipStream_t stream);

/* ------------------------------------------------------------ evaluation */

/*
 * Forward pass: out[i] = f(x_i) (Eq. 1, evaluated as in Algorithm 1).
 *   pts        device, N*3 values of pts_dtype (F32 or F64), xyz interleaved.
 *              With F64 points the lattice-relative offset x - k is formed in
 *              FP64 and then rounded to FP32.
 *   N          number of points, 0 <= N < 2^31 (N == 0 queues nothing).
 *   out        device, N floats.
 * A point with a NaN coordinate gives NaN; points outside the stored lattice
 * see zero coefficients (infinite coordinates give 0).  Never faults on any
 * coordinate value.
 */
lsp_status lsp_eval(const lsp_volume* vol, const void* pts, lsp_dtype pts_dtype, int64_t N,
                    float* out, hipStream_t stream);

/*
 * Value and gradient: val[i] = f(x_i) (val may be NULL), grad[3i+a] = df/dx_a
 * (x_i).  The gradient is the derivative of the sub-region polynomial carried
 * back through the symmetry transform (Sec. 3: the symmetry analysis applies
 * to the derivative polynomials as well).
 */
lsp_status lsp_eval_grad(const lsp_volume* vol, const void* pts, lsp_dtype pts_dtype, int64_t N,
                         float* val, float* grad, hipStream_t stream);

/*
 * Value, gradient and Hessian: hess[6i..6i+5] = the second partials
 * (xx, xy, xz, yy, yz, zz) of f at x_i; val[i] = f(x_i) and grad[3i+a] =
 * df/dx_a (x_i) as for lsp_eval_grad, each skipped when NULL.  The Hessian is
 * that of the sub-region polynomial carried back through the symmetry
 * transform: for y = G (x - k) with G a signed permutation it is G^T H_y G
 * (Sec. 3 applies to every derivative of the reference polynomial).  Where
 * phi is only C^1 (triquadratic) the second partials jump across sub-region
 * boundaries and the value of the sub-region the point is assigned to is
 * returned.  Requires continuity >= 1 (lsp_spline_info): for the C^0 splines
 * (trilinear, BCC linear) it returns LSP_E_UNSUPPORTED before queueing work.
 * A NaN point gives NaN in every output, a point outside the stored lattice
 * zeros.  Allocates nothing.
 *   hess       device, N*6 floats (required when N > 0).
 */
lsp_status lsp_eval_hessian(const lsp_volume* vol, const void* pts, lsp_dtype pts_dtype,
                            int64_t N, float* val, float* grad, float* hess, hipStream_t stream);

/*
 * The same results as lsp_eval (val) and lsp_eval_grad (grad, nullable), bit
 * for bit, computed in spatially binned order: the points are first grouped
 * by coarse blocks of the lattice (counted, scanned and scattered into the
 * workspace), then evaluated block by block so that the stencils of
 * neighbouring work-items share cache lines; results are written back to the
 * callers' indices.  Pays off for large N in random order.  Workspace:
 * device, at least lsp_eval_binned_workspace_size bytes, 256-byte aligned.
 * Allocates nothing.
 */
lsp_status lsp_eval_binned_workspace_size(const lsp_volume* vol, lsp_dtype pts_dtype, int64_t N,
                                          size_t* bytes);
lsp_status lsp_eval_binned(const lsp_volume* vol, const void* pts, lsp_dtype pts_dtype, int64_t N,
                           float* val, float* grad, void* workspace, size_t ws_bytes,
                           hipStream_t stream);

/*
 * Bytes of device workspace lsp_backward needs for N points.
 */
lsp_status lsp_backward_workspace_size(const lsp_volume* vol, int64_t N, size_t* bytes);

/*
 * Backward pass of out = f(pts) for a loss with dL/df = dL_df (device, N floats):
 *   dL_dc  (nullable) device, n_cosets * dims product floats in the same
 *          coset-major C-order layout as lsp_volume_set_coeffs' sources:
 *          dL/dc_n = sum_i dL_df[i] * phi(x_i - n).  Overwritten.
 *          Computed without floating-point atomics; bit-reproducible.
 *   dL_dx  (nullable) device, N*3 floats: dL/dx_i = dL_df[i] * grad f(x_i),
 *          evaluated in the points' order (lsp_backward_dx_from_grad forms
 *          the same values from a gradient saved by the forward pass).
 *   workspace, ws_bytes: device scratch of at least
 *          lsp_backward_workspace_size(vol, N) bytes (needed when dL_dc is
 *          requested), aligned to 256 bytes.
 * Points with a NaN coordinate and points whose stencil misses the stored
 * lattice (infinite and far coordinates included) add nothing to dL_dc;
 * their dL_dx is NaN and 0 respectively.  N == 0 gives dL_dc = 0.
 */
lsp_status lsp_backward(const lsp_volume* vol, const void* pts, lsp_dtype pts_dtype, int64_t N,
                        const float* dL_df, float* dL_dc, float* dL_dx, void* workspace,
                        size_t ws_bytes, hipStream_t stream);

/*
 * dL/dx_i = dL_df[i] * grad_f[i] from gradients saved by lsp_eval_grad or
 * lsp_eval_binned (the chain rule through the query point; the gradient of
 * f is the derivative of the reference sub-region polynomial mapped back by
 * the symmetry transform, Sec. 3 and 4.2).  Gives exactly what lsp_backward
 * writes to dL_dx for the same points, without evaluating the spline again:
 * a training step that needs dL/dx computes value and gradient in its
 * forward pass and calls this, and lsp_backward only for dL/dc.
 *   dL_df   device, N floats;  grad_f  device, N*3 floats (f's gradient);
 *   dL_dx   device, N*3 floats, overwritten (may be the same array as grad_f).
 * NaN gradients (NaN points) stay NaN.  Allocates nothing.
 */
lsp_status lsp_backward_dx_from_grad(int64_t N, const float* dL_df, const float* grad_f,
                                     float* dL_dx, hipStream_t stream);

/* --------------------------------------------------------------- batches */

typedef struct lsp_batch_plan lsp_batch_plan;  /* opaque: bound work list + captured graph */

#define LSP_BATCH_AUTOTUNE 1  /* time candidate launch shapes at creation */

/*
 * Plan the evaluation of n_vol volumes of uneven size in one persistent
 * launch (the per-point work of lsp_eval / lsp_eval_grad, Algorithm 1, for
 * every volume, with the per-point body those entry points use for the
 * volume's point count under the LSP_OPT_SPLIT_MAXN setting in force when
 * the plan is created, so the results are the same).  Per volume v (host
 * arrays of n_vol entries):
 *   vols[v]  volume handle (any spline and storage type; must outlive the plan
 *            and keep its coefficients bound)
 *   pts[v]   device, N[v]*3 FP32 points
 *   val[v]   device, N[v] floats, or NULL if grad[v] is given
 *   grad[v]  (grad itself may be NULL) device N[v]*3 floats for value+gradient,
 *            or NULL for value only
 * Pointers and sizes are bound into the plan: lsp_batch_run evaluates
 * whatever the bound buffers hold at that time.  The work is a list of
 * (volume, tile) items consumed by a persistent grid through an atomic work
 * counter; with LSP_BATCH_AUTOTUNE the tile size and grid size are chosen by
 * timing candidates on `stream` (the outputs are written while doing so).
 * The persistent kernels are captured in a HIP graph; each launch leaves its
 * work counter at zero for the next.  Allocates the plan's device tables;
 * synchronizes `stream` before returning.
 */
lsp_status lsp_batch_plan_create(int n_vol, const lsp_volume* const* vols, const float* const* pts,
                                 const int64_t* N, float* const* val, float* const* grad, int flags,
                                 hipStream_t stream, lsp_batch_plan** out);
/* Chosen tile (points per work item), grid size and number of work items. */
lsp_status lsp_batch_plan_info(const lsp_batch_plan* plan, int* tile, int* blocks, int* n_items);
/* Replay the captured graph on `stream`.  Plans must not run concurrently
 * with themselves (they share one work counter). */
lsp_status lsp_batch_run(lsp_batch_plan* plan, hipStream_t stream);
void lsp_batch_plan_destroy(lsp_batch_plan* plan);

/* ----------------------------------------------------------- diagnostics */

/*
 * Host-only diagnostics of the location step (no device work, no allocation)
 * for a volume of this spline, dims and storage dtype.  For each of N points
 * (host, N*3 doubles, rounded to FP32 as lsp_eval does with F32 points) it
 * writes the byte offset of every union-stencil tap into the internal buffer
 * (offs, host, N*union_taps int32) and a flag word (flags, host, N int32:
 * bit0 active, bit1 NaN, bits 2.. reference sub-region).  Used to check on
 * the CPU that every fetch of an active point stays inside the buffer.
 */
lsp_status lsp_debug_tap_offsets(const lsp_spline* sp, const int64_t dims[3], lsp_dtype storage,
                                 const double* pts, int64_t N, int32_t* offs, int32_t* flags);
/* Internal layout: out (host, 20 int32) = bytes per coefficient, halo,
 * kmin[3], kmax[3] (range of ROE lattice points whose stencil reaches a
 * stored site), log2 brick extent[3], brick stride[3] and in-brick site
 * stride[3] in bytes, storage code, n_cosets, 0; *nbytes = buffer size in
 * bytes.  The byte offset of coset m's site with index idx is
 * m * es + sum_a ((i_a >> lb_a) * bs_a + (i_a & (2^lb_a - 1)) * is_a) with
 * i = idx + halo. */
lsp_status lsp_debug_geometry(const lsp_spline* sp, const int64_t dims[3], lsp_dtype storage,
                              int32_t* out, size_t* nbytes);

#ifdef __cplusplus
}
#endif

#endif /* LSP_H */
