/*
 * mpts -- multiple-precision Taylor series integrator for the Lorenz system
 * on AMD Instinct MI355X (gfx950).
 *
 * The method is the N-th order Taylor series method of Dimova et al.,
 * "OpenMP parallelization of multiple precision Taylor series method":
 *   - the Lorenz system, equation (1) (Section 2), parameters sigma, R, b;
 *   - the Taylor step x_{n+1} = x_n + sum_{i=1}^N alpha_i tau^i, equation (2),
 *     evaluated by Horner's rule (Section 2);
 *   - the Taylor coefficients from the Leibniz recursion, equation (3), whose
 *     two Cauchy-product sums are the reduction the paper parallelises
 *     (Section 2, last paragraph; Section 4).
 *
 * Numbers: binary floating point with p = 32*L bits of mantissa, L 32-bit
 * limbs.  Precision from decimal digits K: L = 2*ceil(ceil(K*log2(10))/64).
 * Rounding is round-to-nearest, ties-to-even, at these points only: each
 * Cauchy sum (exact sum of exact products, rounded once), each new
 * coefficient (exact numerator divided by i+1, rounded once), each Horner
 * step h <- h*tau + c_i (rounded once).  Results therefore do not depend on
 * how the GPU orders or splits the reductions.
 *
 * Conventions for every call:
 *   - returns MPTS_OK (0) or a negative MPTS_E* code; no exception or abort
 *     crosses this interface;
 *   - host buffers are owned by the caller; the library owns only the
 *     context; all device memory is a caller-provided workspace
 *     (mpts_workspace_bytes) and device state buffers (mpts_state_bytes);
 *   - `stream` is a hipStream_t (NULL = default stream); calls are
 *     stream-ordered; the host-buffer variants synchronise before returning;
 *   - a context is not thread-safe: use one context per host thread/stream.
 */
#ifndef MPTS_H
#define MPTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPTS_OK 0
#define MPTS_EINVAL (-1)       /* null pointer, bad string, K<1, N<1, nsteps<0, ... */
#define MPTS_ENOSPC (-2)       /* workspace smaller than mpts_workspace_bytes */
#define MPTS_EHIP (-3)         /* HIP runtime error (see mpts_last_error) */
#define MPTS_ERANGE (-4)       /* an exact sum spread over more than the device
                                  window (see MPTS_MAX_SPREAD_BITS) or an
                                  exponent left the int32 range */
#define MPTS_EARCH (-5)        /* the current device is not gfx950 */
#define MPTS_EUNSUPPORTED (-6) /* size beyond the compiled limits */

/* Exponent difference (in bits) between the terms of one exact sum that
 * the device accumulators always hold: every sum whose terms lie within
 * this many bits of each other is exact on every schedule.  A term further
 * than this from the first term of its sum makes the call fail with
 * MPTS_ERANGE (some schedules still hold a somewhat wider spread exactly);
 * a result is never inexact. */
#define MPTS_MAX_SPREAD_BITS 672

/* flags for mpts_integrate / mpts_integrate_batch */
#define MPTS_CHECKPOINTS 1u    /* keep every per-step state (see checkpoints) */
#define MPTS_GRAPH 2u          /* batch: capture the launch in a hipGraph and replay it */
#define MPTS_AUTOTUNE 4u       /* batch: measure schedules before the run */

typedef struct mpts_ctx mpts_ctx;

/* A big-float: value = sign * M * 2^exp with M = sum_j limbs[j] * 2^(32 j),
 * j = 0..L-1, and the top bit of limbs[L-1] set; sign is -1, 0 or +1 and a
 * zero has sign 0 (limbs all 0, exp 0).  `limbs` points to L caller-owned
 * uint32_t. */
typedef struct {
  int32_t sign;
  int32_t exp;
  uint32_t *limbs;
} mpts_bf;

/* Problem definition (equation (1) parameters, Taylor order N of equation
 * (2), step tau).  sigma, R, b, tau are exact decimal ("-15.8", "1e-2") or
 * rational ("8/3") strings, each rounded once to p bits.  K_digits >= 1 sets
 * the precision (L from the rule above); 1 <= N <= 8192.
 * Errors: MPTS_EINVAL (bad argument), MPTS_EARCH, MPTS_EHIP. */
int mpts_create(const char *sigma, const char *R, const char *b,
                int32_t K_digits, int32_t N, const char *tau, mpts_ctx **out);

/* As mpts_create with the limb count L (1 <= L <= 1024) given directly. */
int mpts_create_limbs(const char *sigma, const char *R, const char *b,
                      int32_t L, int32_t N, const char *tau, mpts_ctx **out);

void mpts_destroy(mpts_ctx *ctx);

/* L, p = 32 L and N of a context (any pointer may be NULL). */
int mpts_limbs(const mpts_ctx *ctx, int32_t *L, int32_t *p_bits, int32_t *N);

/* The rounded parameters: which = 0 sigma, 1 R, 2 b, 3 tau. */
int mpts_param(const mpts_ctx *ctx, int32_t which, mpts_bf *out);

/* Exact parse of a decimal or rational string, one rounding to p bits. */
int mpts_bf_from_str(const mpts_ctx *ctx, const char *s, mpts_bf *out);
/* A double, rounded to p bits (exact when p >= 53). */
int mpts_bf_from_double(const mpts_ctx *ctx, double v, mpts_bf *out);
/* Nearest double (RNE); |v| beyond the double range gives +-inf. */
int mpts_bf_to_double(const mpts_ctx *ctx, const mpts_bf *v, double *out);

/* Workgroups per trajectory for single-trajectory calls (0 = automatic,
 * the number of compute units).  Results do not depend on it. */
int mpts_set_schedule(mpts_ctx *ctx, int32_t workgroups);

/* Device workspace needed by mpts_integrate*, mpts_coefficients and
 * mpts_grad for `nsteps` steps. */
int mpts_workspace_bytes(const mpts_ctx *ctx, int64_t nsteps, uint32_t flags,
                         size_t *bytes);

/* Bytes of one device state (3 components) in the packed device format
 * [sign, exp, limbs[L]] x 3, int32 words. */
int mpts_state_bytes(const mpts_ctx *ctx, size_t *bytes);
/* Host-side packing of x[3] into / out of that format. */
int mpts_pack_state(const mpts_ctx *ctx, const mpts_bf x[3], void *packed);
int mpts_unpack_state(const mpts_ctx *ctx, const void *packed, mpts_bf x[3]);

/* `nsteps` Taylor steps (equation (2)) from x0 (host); the final state is
 * written to x_out (host).  With checkpoints != NULL it receives the
 * 3*(nsteps+1) states s_0..s_nsteps (each with L limbs of storage).
 * Synchronises `stream`.  MPTS_ERANGE is returned if any exact sum did not
 * fit the device window (the outputs are then undefined). */
int mpts_integrate(mpts_ctx *ctx, const mpts_bf x0[3], int64_t nsteps,
                   mpts_bf x_out[3], mpts_bf *checkpoints, void *workspace,
                   size_t ws_bytes, void *stream, uint32_t flags);

/* Device-resident variant, asynchronous on `stream`: x0_dev and xout_dev are
 * packed device states, ckpt_dev (may be NULL) receives nsteps+1 packed
 * states.  Errors found on the device are reported by mpts_check. */
int mpts_integrate_dev(mpts_ctx *ctx, const void *x0_dev, int64_t nsteps,
                       void *xout_dev, void *ckpt_dev, void *workspace,
                       size_t ws_bytes, void *stream);

/* Synchronises `stream` and returns the device error status recorded in
 * the workspace by the last call (MPTS_OK or MPTS_ERANGE).  workspace NULL:
 * the status of the last mpts_integrate_dev_noalloc call on the current
 * device. */
int mpts_check(mpts_ctx *ctx, void *workspace, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * integration as mpts_integrate_dev, with the workspace taken from a device
 * array inside the library (MPTS_NOALLOC_SCRATCH_BYTES bytes, one copy per
 * GPU, held until the process ends) instead of caller memory.  The call
 * allocates nothing: it launches the same kernels and copies its small
 * descriptors into that array on `stream`.  x0_dev, xout_dev and ckpt_dev
 * (may be NULL) are caller-owned packed device states as for
 * mpts_integrate_dev.  Sizes whose workspace exceeds the array (the rows of
 * 3 (N+1) coefficients, about 3 (N+1) (4L + 200) bytes, plus about 0.3 MB)
 * return MPTS_ENOSPC with the need in mpts_last_error.  Every call on one
 * GPU shares that GPU's array, which keeps the last call's contents; calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  Device errors: mpts_check(ctx, NULL, stream). */
#define MPTS_NOALLOC_SCRATCH_BYTES (32u << 20)
int mpts_integrate_dev_noalloc(mpts_ctx *ctx, const void *x0_dev, int64_t nsteps,
                               void *xout_dev, void *ckpt_dev, void *stream);

/* The Taylor coefficients alpha_i, beta_i, gamma_i, i = 0..N (equation (3))
 * of one step from x0, each N+1 arrays of caller-owned mpts_bf (L limbs). */
int mpts_coefficients(mpts_ctx *ctx, const mpts_bf x0[3], mpts_bf *alpha,
                      mpts_bf *beta, mpts_bf *gamma, void *workspace,
                      size_t ws_bytes, void *stream);

/* Batched ensemble: `count` trajectories, trajectory t with its own context
 * ctxs[t] (its own K, N), initial state x0[3t..3t+2], nsteps[t] steps, final
 * state into x_out[3t..3t+2].  All run in one persistent launch; with
 * MPTS_GRAPH the launch is captured in a hipGraph and replayed.  The device
 * workspace size comes from mpts_batch_workspace_bytes. */
int mpts_batch_workspace_bytes(mpts_ctx *const *ctxs, int32_t count,
                               const int64_t *nsteps, uint32_t flags,
                               size_t *bytes);
int mpts_integrate_batch(mpts_ctx *const *ctxs, int32_t count,
                         const mpts_bf *x0, const int64_t *nsteps,
                         mpts_bf *x_out, void *workspace, size_t ws_bytes,
                         void *stream, uint32_t flags);

/* Losses of the final state x(T) = (x, y, z), T = nsteps*tau, for the
 * gradient calls.  Each seeds the reverse sweep with its exact adjoint of
 * x(T): MPTS_LOSS_SQNORM is x^2 + y^2 + z^2 (seed 2 x(T)); MPTS_LOSS_X,
 * _Y, _Z are one component of x(T) (seed the unit vector), so the three
 * give the rows of the Jacobian of x(T) with respect to the inputs. */
#define MPTS_LOSS_SQNORM 0
#define MPTS_LOSS_X 1
#define MPTS_LOSS_Y 2
#define MPTS_LOSS_Z 3

/* Gradient of a loss of x(T) (MPTS_LOSS_*) with respect to (x0, y0, z0,
 * sigma, R, b) by a hand-written reverse sweep of equations (2)-(3) in the
 * same p-bit arithmetic: per-step states are checkpointed by a forward run
 * and the coefficients are recomputed per step; the derivative with respect
 * to b is taken at the p-bit b.  grad_out receives 6 doubles (each the RNE of
 * the p-bit result); loss_out (may be NULL) the loss of the p-bit final state,
 * computed exactly and rounded once to double; grad_bf (may be NULL) the 6
 * p-bit values; x_out (may be NULL) the final state.  The workspace size is
 * mpts_workspace_bytes(ctx, nsteps, MPTS_CHECKPOINTS).  Synchronises
 * `stream`.  Errors: MPTS_EINVAL (unknown loss, null pointer), MPTS_ENOSPC,
 * MPTS_ERANGE, MPTS_EUNSUPPORTED (the reverse kernel does not fit one
 * compute unit at this L, N), MPTS_EHIP. */
int mpts_grad(mpts_ctx *ctx, const mpts_bf x0[3], int64_t nsteps, int32_t loss,
              double grad_out[6], double *loss_out, mpts_bf *grad_bf, mpts_bf x_out[3],
              void *workspace, size_t ws_bytes, void *stream);

/* Gradients of `count` trajectories in one forward launch and one reverse
 * launch: trajectory t has context ctxs[t] (its own K, N), initial state
 * x0[3t..3t+2] and nsteps[t] steps; grad_out receives 6 doubles per
 * trajectory (grad_out[6t..6t+5], ordered as in mpts_grad), loss_out (may
 * be NULL) `count` losses, x_out (may be NULL) 3*count final states.  All
 * trajectories use the same loss.  Each result equals what mpts_grad
 * returns for that trajectory alone (bit for bit).  The device workspace
 * size comes from mpts_grad_batch_workspace_bytes.  Synchronises `stream`.
 * Errors as mpts_grad; MPTS_EUNSUPPORTED also when count exceeds the
 * workgroups resident at once. */
int mpts_grad_batch_workspace_bytes(mpts_ctx *const *ctxs, int32_t count,
                                    const int64_t *nsteps, size_t *bytes);
int mpts_grad_batch(mpts_ctx *const *ctxs, int32_t count, const mpts_bf *x0,
                    const int64_t *nsteps, int32_t loss, double *grad_out,
                    double *loss_out, mpts_bf *x_out, void *workspace,
                    size_t ws_bytes, void *stream);

/* Destroys every cached instantiated batch graph (mpts_destroy already
 * evicts the graphs of the context it frees).  For an orderly shutdown
 * before the HIP runtime is torn down; later batch calls re-capture. */
int mpts_release_caches(void);

/* Measured issue rate of one arithmetic unit on the current device, for the
 * roofline of the measurement (not part of the method): unit
 * MPTS_PROBE_VALU_MAD gives 32x32 -> 64-bit signed multiply-adds per
 * second (v_mad_i64_i32, formed as the 8x8 digit tiles of the product
 * loop), MPTS_PROBE_MFMA_I8 int8 multiply-adds per second of
 * v_mfma_i32_32x32x32_i8 (the piece products of the matrix-core path).
 * out_dev: caller's device scratch of at least 8 * 1024 * (compute units)
 * bytes (the probe kernels' results, written so they are not optimised
 * away).  Synchronises `stream`.  Errors: MPTS_EINVAL, MPTS_ENOSPC,
 * MPTS_EHIP. */
#define MPTS_PROBE_VALU_MAD 0
#define MPTS_PROBE_MFMA_I8 1
int mpts_probe_rate(int32_t unit, double *per_second, void *out_dev, size_t out_bytes,
                    void *stream);

const char *mpts_strerror(int status);
/* Text of the last error recorded on this context ("" if none). */
const char *mpts_last_error(const mpts_ctx *ctx);

/* ---- Polynomial vector fields of degree at most two ----
 *
 * The paper notes (Section 2, the paragraph on automatic differentiation,
 * and Section 6) that the recursion of equation (3) extends to any
 * right-hand side built from sums and products: each product term gives a
 * Cauchy-product sum.  A system here is
 *   dx_v/dt = c_v + sum_u A_vu x_u + sum_{u<=w} B_vuw x_u x_w,  v < nvar <= 4,
 * given as terms coef * x_u * x_w of equation eq (u = w = -1: the constant
 * c_eq; w = -1: a linear term).  Per index i: S_uw = sum_k x_{u,i-k} x_{w,k}
 * rounded once for each distinct pair; x_{v,i+1} = ([i=0] c_v + sum A x_{u,i}
 * + sum B S_uw) / (i+1) rounded once (exact numerator); the step is
 * equation (2) by Horner's rule, one rounding per step; every coefficient
 * and tau rounded once to p bits.  With the Lorenz terms this is exactly the
 * Lorenz recursion above.
 *
 * Limits (MPTS_EUNSUPPORTED beyond them): at most 5 distinct product pairs,
 * at most one constant term per equation, per equation at most 4 terms
 * whose coefficient is not +-1 plus 2 whose coefficient is +-1 (further
 * +-1 terms count as the former), rows of at most 1024 words (L up to about
 * 800 limbs), and the LDS of one compute unit (160 KB; about L = 300 at
 * N = 600).  One workgroup integrates one trajectory. */
typedef struct mpts_poly mpts_poly;

typedef struct {
  int32_t eq, u, w;   /* equation; variables (-1: absent) */
  const char *coef;   /* exact decimal or rational string */
} mpts_poly_term;

/* nvar variables, nterms terms (caller-owned, read during the call), L
 * limbs (p = 32 L), order N, step tau (string).  Errors: MPTS_EINVAL (bad
 * term, index or string), MPTS_EUNSUPPORTED (limits above). */
int mpts_poly_create(int32_t nvar, const mpts_poly_term *terms, int32_t nterms, int32_t L,
                     int32_t N, const char *tau, mpts_poly **out);
void mpts_poly_destroy(mpts_poly *ctx);

/* Exact parse of a decimal or rational string, one rounding to p bits. */
int mpts_poly_bf_from_str(const mpts_poly *ctx, const char *s, mpts_bf *out);

/* `nsteps` steps of `count` trajectories in one launch: x0 and x_out hold
 * count * nvar big-floats (trajectory-major, host, L limbs each).
 * Synchronises `stream`; allocates and frees its device memory.
 * MPTS_ERANGE: an exact sum did not fit the device window (outputs then
 * undefined); MPTS_EHIP: a HIP error. */
int mpts_poly_integrate(mpts_poly *ctx, int32_t count, const mpts_bf *x0, int64_t nsteps,
                        mpts_bf *x_out, void *stream);

/* The Taylor coefficients x_{v,i}, i = 0..N, of one step from x0 (nvar
 * values): coefs holds nvar * (N + 1) big-floats, variable-major. */
int mpts_poly_coefficients(mpts_poly *ctx, const mpts_bf *x0, mpts_bf *coefs, void *stream);

/* Text of the last error of a polynomial context ("" if none). */
const char *mpts_poly_last_error(const mpts_poly *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MPTS_H */
