/*
 * bg.h -- C ABI of the MI355X (gfx950) Berends-Giele library libbg_mi355x.so.
 *
 * The library evaluates colour-ordered n-gluon tree amplitudes with the
 * Berends-Giele recursion of arXiv:2502.07060 (Sec. 2.2: the current
 * recursion, the three- and four-gluon vertices V3 and V4, the sub-range
 * momenta P_{i,j}), for many phase-space points at once, over two fields:
 *
 *   bg_amplitudes_c128  complex numbers in IEEE binary64 (the paper's
 *                       double-precision complex path, Sec. 3);
 *   bg_amplitudes_fp    the prime field Z_p, p an odd prime below 2^31 (the
 *                       paper's finite-field path, Sec. 3, default
 *                       p = 2^31 - 19), results exact.
 *
 * What is returned.  Legs 1..n carry momenta k_l and polarisation vectors
 * eps_l, each with d components, metric diag(+1,-1,...,-1) (Sec. 2.3),
 * products bilinear (no complex conjugation).  With N = n - 1 and currents
 * J(S) over the contiguous sub-ranges S of legs 1..N, J([l]) = eps_l and
 *     J(S) = K(S) / P_S^2,
 *     K(S) = sum over splits S = A|B of
 *              (J_A.J_B)(P_A - P_B) + 2 (P_B.J_A) J_B - 2 (P_A.J_B) J_A
 *          + sum over splits S = A|B|C of
 *              2 (J_A.J_C) J_B - (J_A.J_B) J_C - (J_B.J_C) J_A,
 * which is the paper's recursion with the factor i of each vertex cancelled
 * against the -i of each propagator.  The value returned per point is
 *     M = eps_n . K([1..N]),
 * the amplitude built from the (n-1)-point current with the off-shell
 * propagator removed (Sec. 2.2); the amplitude with all phases is A = i M.
 * k_n is never read (it enters only through momentum conservation, which the
 * caller's momenta are expected to satisfy; nothing is checked).
 *
 * Data layout (all compute entry points).  Arrays are device pointers owned
 * by the caller (for example torch tensors); nothing is retained after the
 * call returns:
 *     momenta[l][mu][q], pols[l][mu][q]   l < n, mu < d, q < ld, q fastest;
 *     element (l, mu, q) at offset (l * d + mu) * ld + q elements.
 * For complex128 an element is two doubles (real, imaginary).  out[q] and
 * status[q] for q < npts.  ld >= npts.
 *
 * Per-point status byte (status may be NULL):
 *     BG_PT_OK         0  result valid
 *     BG_PT_SINGULAR   1  some propagator denominator P_S^2 is exactly zero
 *                         (2 <= |S| <= n-2); out[q] is the sentinel
 *     BG_PT_BADRESIDUE 2  (F_p) a component of k_1..k_{n-1} or eps_1..eps_n
 *                         is >= p; out[q] is the sentinel (takes precedence)
 * Sentinels: NaN + i NaN (complex128), 0xFFFFFFFF (F_p).
 *
 * Errors.  Argument errors are reported by a negative return value before
 * anything is enqueued.  A failed kernel launch returns BG_EHIP.  Calls are
 * asynchronous on the given HIP stream (NULL = the default stream): results
 * are valid once the stream has been synchronised.  npts == 0 is a no-op.
 * The compute entry points allocate no device memory and are thread safe.
 */
#ifndef BG_MI355X_H
#define BG_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BG_OK = 0,
  BG_EINVAL = -1,      /* NULL pointer, ld < npts, npts < 0, bad field tag  */
  BG_EDOMAIN = -2,     /* n outside [3, BG_MAX_N] or d outside [1, BG_MAX_D] */
  BG_ENOTPRIME = -3,   /* p not an odd prime below 2^31                      */
  BG_EHIP = -4,        /* a HIP runtime call or kernel launch failed         */
  BG_ENOTIMPL = -5,    /* no kernel for this (field, n, d)                   */
  BG_ENOMEM = -6,      /* a request does not fit the serving budget          */
  BG_EBUSY = -7        /* serving queue full; retry later                    */
};

enum { BG_PT_OK = 0, BG_PT_SINGULAR = 1, BG_PT_BADRESIDUE = 2 };

#define BG_MAX_N 14
#define BG_MAX_D 10

/* Field tags for the batched and serving entry points. */
enum { BG_FIELD_C128 = 0, BG_FIELD_FP = 1 };

/*
 * bg_amplitudes_c128 -- amplitudes over complex binary64 (paper Sec. 2.2,
 * Sec. 3 double-precision complex path).
 *   n        number of gluons, 3 <= n <= BG_MAX_N
 *   d        number of momentum components, 1 <= d <= BG_MAX_D (d = 4 is
 *            four-dimensional; d > 4 states padded with zeros give the
 *            four-dimensional result, Sec. 2.3)
 *   npts     number of phase-space points (>= 0)
 *   ld       leading dimension of momenta and pols (>= npts)
 *   momenta  device, complex128 [n][d][ld] (re, im interleaved)
 *   pols     device, complex128 [n][d][ld]
 *   out      device, complex128 [npts]: M per point
 *   status   device, uint8 [npts] or NULL
 *   hip_stream  hipStream_t or NULL
 * Returns BG_OK or a negative error code.
 */
int bg_amplitudes_c128(int n, int d, int64_t npts, int64_t ld,
                       const double* momenta, const double* pols,
                       double* out, uint8_t* status, void* hip_stream);

/*
 * bg_amplitudes_fp -- amplitudes over Z_p (paper Sec. 2.2; Sec. 3 finite
 * fields: p < 2^31, exact arithmetic, division by the modular inverse).
 *   p        odd prime, 3 <= p < 2^31 (checked with a deterministic
 *            Miller-Rabin test; BG_ENOTPRIME otherwise)
 *   momenta, pols  device, uint32 [n][d][ld], canonical residues in [0, p)
 *   out      device, uint32 [npts]: M mod p in [0, p), or 0xFFFFFFFF
 *   other arguments as for bg_amplitudes_c128.
 */
int bg_amplitudes_fp(int n, int d, int64_t npts, int64_t ld, uint32_t p,
                     const uint32_t* momenta, const uint32_t* pols,
                     uint32_t* out, uint8_t* status, void* hip_stream);

/*
 * bg_currents_c128, bg_currents_fp -- the root current K([1..n-1]) instead
 * of M (paper Sec. 2.2: the amplitude is the contraction of the current of
 * legs 1..n-1, its propagator removed, with eps_n): M = eps_n . K, so one
 * call gives M for every polarisation of leg n.  Same arguments, layouts,
 * statuses and errors as bg_amplitudes_*, except
 *   cur      device [d][ld] (complex128, or uint32 residues in [0, p)):
 *            component mu of point q at mu * ld + q; every component of a
 *            point with a non-zero status holds the sentinel.
 * pols row n-1 (eps_n) does not enter K but is read and must hold
 * canonical residues over Z_p.  Mostly-minus metric.
 */
int bg_currents_c128(int n, int d, int64_t npts, int64_t ld, const double* momenta,
                     const double* pols, double* cur, uint8_t* status, void* hip_stream);
int bg_currents_fp(int n, int d, int64_t npts, int64_t ld, uint32_t p, const uint32_t* momenta,
                   const uint32_t* pols, uint32_t* cur, uint8_t* status, void* hip_stream);

/*
 * Metric of every Minkowski product (propagators P^2 and all contractions).
 *   BG_METRIC_MOSTLY_MINUS  diag(1, -1, ..., -1)           (paper Sec. 2.2; the
 *                           metric of bg_amplitudes_c128 / _fp and of every
 *                           batched and served call)
 *   BG_METRIC_ALTERNATING   diag(1, -1, 1, -1, 1, ...)     (paper Sec. 3.1, the
 *                           convention of Caravel)
 */
enum { BG_METRIC_MOSTLY_MINUS = 0, BG_METRIC_ALTERNATING = 1 };

/*
 * bg_amplitudes_c128_metric, bg_amplitudes_fp_metric -- bg_amplitudes_c128
 * and bg_amplitudes_fp with the metric chosen by `metric` (one of
 * BG_METRIC_*; BG_EINVAL otherwise); the inputs are vectors in that metric
 * (e.g. massless means k.k = 0 there).  Same layouts, outputs, statuses and
 * errors.  The alternating metric is reached exactly by multiplying the
 * components 2, 4, 6, ... of every input vector by a square root of -1 as it
 * is loaded, which turns every product into the mostly-minus one; over Z_p
 * this needs p = 1 (mod 4) (BG_EDOMAIN otherwise), with i = g^((p-1)/4) for
 * the smallest quadratic non-residue g (M does not depend on the choice).
 * Over Z_p, alternating-metric calls whose selected kernel is a one-lane
 * register kernel run the two-lane one of the same (n, d): its alternating
 * form is the faster of the two.
 */
int bg_amplitudes_c128_metric(int metric, int n, int d, int64_t npts, int64_t ld,
                              const double* momenta, const double* pols,
                              double* out, uint8_t* status, void* hip_stream);
int bg_amplitudes_fp_metric(int metric, int n, int d, int64_t npts, int64_t ld, uint32_t p,
                            const uint32_t* momenta, const uint32_t* pols,
                            uint32_t* out, uint8_t* status, void* hip_stream);

/*
 * Polarisation states of massless d-dimensional gluons (paper Sec. 2.3, in
 * its square-root-free normalisation): for each point q, a massless d-vector
 * k and a massless four-dimensional reference chi give the d - 2 states
 * e_1..e_{d-2} and their duals e~_1..e~_{d-2} with k.e_i = 0,
 * e_i.e~_j = -delta_ij and sum_i e_i^mu e~_i^nu = -g^{mu nu} + (k^mu eta^nu +
 * eta^mu k^nu)/(k.eta), eta = (k^0..k^3, -k^4, ..., -k^{d-1}) (d >= 5):
 *   k4 = (k^0..k^3, 0, ...), mu^2 = k4.k4, kb = k4 - mu^2/(2 chi.k4) chi,
 *   e_1 = <kb|gamma|chi]/(2 [kb chi]),  e_2 = [kb|gamma|chi>/<kb chi>,
 *   e~_1 = e_2, e~_2 = e_1,
 *   e_3 = kb - mu^2/(2 chi.k4) chi, e~_3 = e_3/mu^2               (d >= 5),
 *   e_4 = (0,0,0,0, k^5, -k^4, 0, ...), e~_4 = e_4/(k^4 k^4 + k^5 k^5) (d >= 6),
 *   e_x^i = k^i k^{x+1} (4 <= i <= x), e_x^{x+1} = -mu_{x+1}^2,
 *   e~_x = e_x/(mu_{x+1}^2 mu_{x+2}^2)  (5 <= x <= d-2), mu_y^2 = sum_{4<=i<y} (k^i)^2.
 * Spinors of a massless four-vector v: lam = (1, (v^1 + i v^2)/v+),
 * lamt = (v+, v^1 - i v^2) when v+ = v^0 + v^3 is non-zero (F_p) or
 * |v+|^2 >= |v-|^2 (complex), else lam = ((v^1 - i v^2)/v-, 1),
 * lamt = (v^1 + i v^2, v-), v- = v^0 - v^3.
 *   d        4 <= d <= BG_MAX_D
 *   momenta  device [d][ld] (k), chi device [4][ld]
 *   eps, epst  device [d-2][d][ld]: state s, component mu at (s d + mu) ld + q
 *   status   device uint8 [npts] or NULL: BG_PT_OK; BG_PT_SINGULAR when a
 *            required denominator vanishes (chi.k4, a bracket, a spinor chart,
 *            mu^2 products); BG_PT_BADRESIDUE (F_p) for an input >= p.  Both
 *            outputs then hold the sentinel in every slot of the point.
 * bg_states_fp needs p = 1 (mod 4) (BG_EDOMAIN otherwise): i is
 * g^((p-1)/4) mod p for the smallest quadratic non-residue g.  Residues in
 * and out are canonical.  Other arguments and errors as for bg_amplitudes_*.
 */
int bg_states_c128(int d, int64_t npts, int64_t ld, const double* momenta, const double* chi,
                   double* eps, double* epst, uint8_t* status, void* hip_stream);
int bg_states_fp(int d, int64_t npts, int64_t ld, uint32_t p, const uint32_t* momenta,
                 const uint32_t* chi, uint32_t* eps, uint32_t* epst, uint8_t* status,
                 void* hip_stream);

/*
 * bg_state_sum_c128, bg_state_sum_fp -- sum over the states of one cut leg
 * of a product of two trees (paper Sec. 2.1, the leading pole of the cut
 * equation, with the states of Sec. 2.3):
 *   S[q] = sum_{s < d-2} (e_s . K_L)(e~_s . K_R)     (mostly-minus products)
 * where K_L, K_R are root currents (bg_currents_*) of two trees whose last
 * leg is the cut leg (momentum l in one, -l in the other) and e_s, e~_s the
 * states and duals of l (bg_states_*), so that M_L(e_s) = e_s . K_L and
 * M_R(e~_s) = e~_s . K_R.
 *   d        4 <= d <= BG_MAX_D (BG_EDOMAIN otherwise)
 *   kl, kr   device [d][ld]; eps, epst device [d-2][d][ld] (as bg_states_*)
 *   out      device [npts] (complex128, or uint32 in [0, p))
 *   status   device uint8 [npts] or NULL: BG_PT_OK; over Z_p BG_PT_BADRESIDUE
 *            when an input is >= p (e.g. a sentinel; out is 0xFFFFFFFF);
 *            over C BG_PT_SINGULAR when the result is not a number.
 */
int bg_state_sum_c128(int d, int64_t npts, int64_t ld, const double* kl, const double* kr,
                      const double* eps, const double* epst, double* out, uint8_t* status,
                      void* hip_stream);
int bg_state_sum_fp(int d, int64_t npts, int64_t ld, uint32_t p, const uint32_t* kl,
                    const uint32_t* kr, const uint32_t* eps, const uint32_t* epst, uint32_t* out,
                    uint8_t* status, void* hip_stream);

/*
 * From Z_p samples back to rational numbers (paper Sec. 1 and Sec. 3: values
 * computed over F_p at rational kinematic points are reconstructed as
 * rationals, e.g. to compare with another program's result).
 *
 * bg_fp_from_rational -- residues of fractions, elementwise:
 *   out[i] = num[i] / den[i] mod p, canonical in [0, p)
 *   p        odd prime below 2^31 (BG_ENOTPRIME otherwise)
 *   count    number of values (>= 0)
 *   num, den device int64 [count]; out device uint32 [count]
 *   status   device uint8 [count] or NULL: 0, or 1 when p divides den[i]
 *            (out[i] = 0xFFFFFFFF)
 * Use it to map rational momenta and polarisations onto each prime before
 * bg_amplitudes_fp.
 *
 * bg_rational_reconstruct -- Chinese remaindering and rational
 * reconstruction, one point per lane.  With M = p_1 ... p_k and
 * B = floor(sqrt((M - 1) / 2)), the residues r_i give the unique
 * 0 <= x < M with x = r_i (mod p_i); the extended Euclidean algorithm on
 * (M, x) is run to the first remainder r <= B, with cofactor t; the result is
 * a / b = sign(t) r / |t| when 0 < |t| <= B and gcd(t, M) = 1 (Wang's
 * rational reconstruction, as in von zur Gathen and Gerhard, Modern Computer
 * Algebra, Sec. 5.10).  Any fraction with |a| <= B, 0 < b <= B,
 * gcd(a, b) = 1 and a = b x (mod M) is unique, and is the one returned.
 *   nprimes  1 <= nprimes <= BG_RR_MAX_PRIMES (BG_EINVAL otherwise)
 *   primes   host uint32 [nprimes]: distinct odd primes below 2^31
 *            (BG_ENOTPRIME / BG_EINVAL)
 *   residues device uint32 [nprimes][ld]: the value modulo primes[i] of
 *            point q at i * ld + q (e.g. the out arrays of bg_amplitudes_fp)
 *   num      device int32 [L][ld], L = BG_RR_LIMBS(nprimes): a in two's
 *            complement, 32-bit limbs least significant first
 *   den      device uint32 [L][ld]: b, same limb order
 *   status   device uint8 [npts] or NULL: 0 reconstructed; 1 no fraction
 *            within the bound (more primes are needed); 2 a residue is not
 *            in [0, p_i) (e.g. the sentinel of a singular point).  num and
 *            den are zero unless the status is 0.
 * Both calls are asynchronous on hip_stream and allocate nothing.
 */
#define BG_RR_MAX_PRIMES 32
#define BG_RR_LIMBS(nprimes) (((nprimes) + 2) / 2)
int bg_fp_from_rational(uint32_t p, int64_t count, const int64_t* num, const int64_t* den,
                        uint32_t* out, uint8_t* status, void* hip_stream);
int bg_rational_reconstruct(int nprimes, const uint32_t* primes, int64_t npts, int64_t ld,
                            const uint32_t* residues, int32_t* num, uint32_t* den,
                            uint8_t* status, void* hip_stream);

/*
 * Standalone batched Z_p operations (paper Sec. 3: the finite-field library
 * under the recursion, usable on its own).  Residues are canonical uint32 in
 * [0, p), p an odd prime below 2^31 (BG_ENOTPRIME otherwise); element e of
 * event q is at e * ld + q (the event index fastest).
 *
 * bg_fp_contract -- z[i][k] = sum_j x[i][j] y[j][k] mod p for every event:
 *   I, J, K  1 .. BG_FP_MAX_DIM (BG_EDOMAIN otherwise); each of i, j, k
 *            stands for any group of tensor indices, flattened by the caller
 *            (e.g. z_{n i}^{k} = x_{n i j l} y_n^{j l k} has J = dim(j) dim(l))
 *   x        device uint32 [I][J][ld]
 *   y        device uint32 [J][K][ld] when y_batched != 0 (one y per event),
 *            else [J][K] (one y shared by every event)
 *   z        device uint32 [I][K][ld]
 *   status   device uint8 [npts] or NULL: BG_PT_OK, or BG_PT_BADRESIDUE when
 *            an input of the event is >= p (then every z of the event is
 *            0xFFFFFFFF)
 *
 * bg_fp_divide -- z[q] = x[q] / y[q] mod p elementwise (count values):
 *   x, y, z  device uint32 [count]
 *   status   device uint8 [count] or NULL: BG_PT_OK; BG_PT_SINGULAR when
 *            y[q] = 0; BG_PT_BADRESIDUE when x[q] or y[q] >= p; z[q] is
 *            0xFFFFFFFF unless the status is BG_PT_OK
 * bg_fp_divide_scalar -- the same with one y for every value (host
 *            argument; BG_EDOMAIN when y = 0, BG_EINVAL when y >= p).
 * All three are asynchronous on hip_stream and allocate nothing.
 */
#define BG_FP_MAX_DIM 4096
int bg_fp_contract(uint32_t p, int I, int J, int K, int64_t npts, int64_t ld,
                   const uint32_t* x, const uint32_t* y, int y_batched, uint32_t* z,
                   uint8_t* status, void* hip_stream);
int bg_fp_divide(uint32_t p, int64_t count, const uint32_t* x, const uint32_t* y,
                 uint32_t* z, uint8_t* status, void* hip_stream);
int bg_fp_divide_scalar(uint32_t p, int64_t count, const uint32_t* x, uint32_t y,
                        uint32_t* z, uint8_t* status, void* hip_stream);

/*
 * Batched form: many (field, n, d) groups in one call.  The paper traces the
 * fixed offset it sees at small event counts to run-time flexibility and
 * proposes compiling ahead of time for a set number of legs and dimension
 * (Sec. 3.2, discussion of Fig. 1b and Fig. 4); this call runs such
 * precompiled kernels for many (n, d) at once.  Each group has the
 * layout and meaning of one bg_amplitudes_* call; every group is validated
 * before anything is enqueued (the first invalid group's error is returned).
 * Groups run the kernel variant selected for their (field, n, d), longest
 * first, spread over internal streams that fork from and join back to
 * hip_stream: results are valid once hip_stream has been synchronised.
 * Groups must not overlap in their outputs.
 */
typedef struct {
  int field;            /* BG_FIELD_C128 or BG_FIELD_FP                         */
  int n, d;
  uint32_t p;           /* prime, F_p groups only                               */
  int64_t npts, ld;
  const void* momenta;  /* complex128 or uint32 [n][d][ld], device            */
  const void* pols;     /* same layout                                          */
  void* out;            /* complex128 or uint32 [npts], device                  */
  uint8_t* status;      /* uint8 [npts] or NULL                                 */
} bg_group;

int bg_batch_run(const bg_group* groups, int ngroups, void* hip_stream);

/*
 * The same call with options.  BG_BATCH_QUEUE: every group whose selected
 * kernel is a lane-group (runtime-n) kernel is served by one persistent launch
 * per such kernel variant instead of one launch per group.  Its blocks stay
 * resident and take (group, point range) tiles from a device work queue, the
 * groups ordered by work per point, longest first; register-kernel groups run
 * as in bg_batch_run.  The queue's counters and group table (about 160 bytes
 * a group) are device memory this call allocates stream-ordered on
 * hip_stream and frees after its launches.  Results equal bg_batch_run's bit
 * for bit (same kernels, same arithmetic per point).  flags = 0 is
 * bg_batch_run.  Errors: as bg_batch_run, BG_EINVAL for unknown flags,
 * BG_ENOMEM if the queue memory cannot be allocated.
 */
#define BG_BATCH_QUEUE 1
int bg_batch_run_ex(const bg_group* groups, int ngroups, int flags, void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): bg_batch_run_ex with
 * BG_BATCH_QUEUE, but the queue lives in a fixed device array of the library
 * (256 KiB per GPU, held until the process ends; enough for about 1500
 * lane-group groups per call) and every launch goes to hip_stream in turn,
 * so the call allocates nothing, creates no streams and calls no allocating
 * routine.  The array keeps the previous call's contents; each call rewrites
 * the tables and zeroes the counters before its launches.  Calls that overlap
 * on one GPU (concurrent streams or host threads) race on the array and must
 * be serialised by the caller.  BG_ENOMEM if the call's queue does not fit the
 * array; otherwise as bg_batch_run_ex.
 */
int bg_batch_run_noalloc(const bg_group* groups, int ngroups, void* hip_stream);

/*
 * A batch plan records the launches of a fixed set of groups (pointers and
 * sizes fixed, kernel variants as selected at creation) as one hipGraph of
 * independent kernel nodes; bg_batch_plan_launch replays it on hip_stream with
 * a single graph launch.  Plans own no device memory (but see
 * bg_batch_plan_create_ex).
 */
typedef struct bg_batch_plan bg_batch_plan;
int bg_batch_plan_create(const bg_group* groups, int ngroups, bg_batch_plan** plan);
/* flags as bg_batch_run_ex: with BG_BATCH_QUEUE the plan owns the queue's
 * device memory (allocated and written at creation, freed by destroy) and
 * each replay zeroes the counters with a kernel node before the persistent
 * launches. */
int bg_batch_plan_create_ex(const bg_group* groups, int ngroups, int flags, bg_batch_plan** plan);
int bg_batch_plan_launch(bg_batch_plan* plan, void* hip_stream);
int bg_batch_plan_destroy(bg_batch_plan* plan);

/*
 * Serving loop.  The paper leaves memory management for a continuous stream
 * of evaluations to future work (Sec. 3, the closing remarks on the
 * implementation); this is one design for it.  A server owns one device
 * arena of hbm_budget_bytes (one allocation at creation, on the current device), a few streams and one
 * scheduler thread.  Requests are bg_group records whose four pointers are
 * HOST memory (pinned memory lets copies overlap kernels): momenta and pols
 * [n][d][ld] with ld the host leading dimension, out [npts] and status
 * [npts] (status may be NULL).  The host buffers must stay valid until the
 * request completes.
 *
 * Each request occupies npts (2 n d s + s + 1) bytes of the arena while it
 * runs (s = 16 complex, 4 F_p; columns padded to 64 points, parts to 256
 * bytes).  Requests are admitted first come, first served as arena space
 * and launch slots free up; requests waiting for the same (field, n, d, p)
 * are merged into one kernel launch over adjacent columns; several launches
 * are in flight at once on separate streams, their copies overlapping other
 * launches' kernels.  Every point is computed exactly as by
 * bg_amplitudes_c128 / bg_amplitudes_fp with the kernel variant selected
 * for its (field, n, d), so a request's results do not depend on what it
 * was batched with.
 *
 * With flags = BG_SERVER_PLAIN the server runs one request per launch, one at
 * a time, in arrival order, on one stream (the plain baseline).
 */
#define BG_SERVER_PLAIN 1
typedef struct bg_server bg_server;

typedef struct {
  int64_t submit_ns;    /* steady-clock times (bg_server_now_ns): submitted,  */
  int64_t launch_ns;    /* its copies and kernel enqueued,                     */
  int64_t done_ns;      /* completion seen by the scheduler (results on host)  */
  int32_t batch_requests;  /* requests that shared its kernel launch          */
} bg_request_times;

typedef struct {
  int64_t submitted, completed, rejected;
  int64_t batches;           /* kernel launches made                          */
  int64_t points;            /* points of completed requests                  */
  int64_t queued;            /* requests waiting for admission                */
  int64_t inflight_batches;
  int64_t arena_bytes, arena_in_use, arena_peak;
} bg_server_stats;

/* BG_EINVAL (bad flags, budget < 256 B), BG_ENOMEM (arena allocation
 * failed), BG_EHIP. */
int bg_server_create(size_t hbm_budget_bytes, int flags, bg_server** srv);

/* Validates like bg_batch_run (same codes); BG_ENOMEM if the request alone
 * exceeds the arena, BG_EBUSY if 2^20 requests are already queued.  On
 * BG_OK *id names the request; npts == 0 completes at once. */
int bg_server_submit(bg_server* srv, const bg_group* request, uint64_t* id);

/* 1 if done, 0 if not yet, BG_EINVAL for an unknown id. */
int bg_server_poll(bg_server* srv, uint64_t id);

/* Blocks until the request is done (timeout_s < 0: no limit), fills times
 * (may be NULL) and forgets the id.  Returns the request's result code
 * (BG_OK, or BG_EHIP if a copy or launch failed), BG_EBUSY on timeout (the id
 * stays valid), BG_EINVAL for an unknown id. */
int bg_server_wait(bg_server* srv, uint64_t id, double timeout_s, bg_request_times* times);

int bg_server_get_stats(bg_server* srv, bg_server_stats* out);

/* The clock of bg_request_times, in nanoseconds. */
int64_t bg_server_now_ns(void);

/* Finishes every submitted request, then frees the arena and the streams. */
int bg_server_destroy(bg_server* srv);

/*
 * Kernel variants (tuning interface).  Several kernels may be compiled for one
 * (field, n, d): lanes per point, components per lane, per-point tables in
 * registers or LDS, or the runtime-n kernel.  The library picks one by
 * default; a tuner may measure them and pin one.  Selections are process-wide
 * and thread safe.
 */
typedef struct {
  int index;            /* pass to bg_select_variant                           */
  int lanes;            /* lanes cooperating on one point                      */
  int comps_per_lane;   /* Lorentz components held by each lane (>= d / lanes) */
  int lds_tables;       /* per-point scalar and momentum tables in LDS          */
  int generic;          /* runtime-n kernel (tables in LDS; lanes > 1: that many
                           lanes share one point's tables)                       */
  int padded;           /* lanes > 1 runtime-n kernel whose LDS table rows are
                           padded to an odd number of 16-byte units            */
  int max_d;            /* largest d the kernel handles                        */
  int selected;         /* 1 if this variant is the one currently in use        */
} bg_variant_info;

/* Fills up to cap entries for (field, n, d); returns the number available
 * (possibly > cap) or a negative error code. */
int bg_variants(int field, int n, int d, bg_variant_info* out, int cap);

/* Pins variant `index` (from bg_variants) for (field, n, d); index -1 restores
 * the default choice.  BG_EINVAL if the index does not fit (field, n, d).
 * This is the selection of the mostly-minus metric, the one bg_variants
 * reports as `selected`. */
int bg_select_variant(int field, int n, int d, int index);

/* The same for launches in metric BG_METRIC_* (paper Sec. 3.1): the two
 * metric forms of one kernel can run at different speeds, so alternating-
 * metric launches have pins of their own.  Without one they take the
 * mostly-minus selection (over Z_p with a one-lane register kernel replaced
 * by the two-lane one).  BG_EINVAL for an unknown metric. */
int bg_select_variant_metric(int metric, int field, int n, int d, int index);

/*
 * bg_autotune -- times every variant compiled for (field, n, d) on npts
 * synthetic points (uniform residues mod p, or complex values with parts in
 * [-1, 1)), reps launches each after one warm-up, on hip_stream; the variants
 * within 5 % of the fastest are timed three more times, in turns, each keeping
 * its best time.  Pins the fastest and returns its index (>= 0) or a negative
 * error code.  ms_out (may be NULL) receives the time per launch of each
 * variant in bg_variants order, up to cap entries.  Allocates and frees its
 * own device buffers; it synchronises the stream.  p is ignored for the
 * complex field.
 */
int bg_autotune(int field, int n, int d, uint32_t p, int64_t npts, int reps,
                double* ms_out, int cap, void* hip_stream);

/* bg_autotune in metric BG_METRIC_* (BG_EINVAL otherwise): times the launches
 * in that metric and pins the fastest for it (bg_select_variant_metric).
 * Over Z_p the alternating metric needs p = 1 (mod 4) (BG_EDOMAIN). */
int bg_autotune_metric(int metric, int field, int n, int d, uint32_t p, int64_t npts, int reps,
                       double* ms_out, int cap, void* hip_stream);

/* Writes the pinned selections of both metrics to a text file (one line per
 * pinned (field, n, d, metric), naming the kernel by lanes, components per
 * lane, LDS tables, generic, padded, max_d; the metric is the last column). */
int bg_tune_save(const char* path);

/* Applies selections written by bg_tune_save (a line without the metric
 * column pins the mostly-minus metric); returns how many matched a compiled
 * kernel, or a negative error code. */
int bg_tune_load(const char* path);

/*
 * bg_issue_rate -- measures the issue rate of one VALU instruction class on
 * the current device: blocks x 256 lanes each run 8 independent dependency
 * chains of `iters` rounds of that instruction, reps timed launches after
 * one warm-up on hip_stream.  *lane_ops_per_s receives lane-operations per
 * second (every lane of a wave counts), *ms_per_launch (may be NULL) the
 * time per launch.  This is the roofline denominator of the Z_p path, whose
 * arithmetic is 64-bit integer multiply-add modulo p (Sec. 3) and has no
 * published peak; BG_PROBE_FMA_F64 checks the method against the published
 * FP64 rate.  Allocates and frees an 8-byte-per-lane sink buffer and
 * synchronises the stream (a measurement call, not for hot paths).
 * BG_EINVAL for an unknown kind or non-positive sizes.
 */
enum {
  BG_PROBE_MAD_I64_I32 = 0,   /* v_mad_i64_i32: (int64) a * b + c, a, b int32 */
  BG_PROBE_MAD_U64_U32 = 1,   /* v_mad_u64_u32                                */
  BG_PROBE_FMA_F64 = 2,       /* v_fma_f64                                    */
  BG_PROBE_MUL_LO_U32 = 3,    /* v_mul_lo_u32                                 */
  BG_PROBE_DPP_MOV_B32 = 4    /* v_mov_b32 with a DPP lane permutation        */
};
int bg_issue_rate(int kind, int blocks, int iters, int reps, double* lane_ops_per_s,
                  double* ms_per_launch, void* hip_stream);

/* Human-readable text for a return code (static storage). */
const char* bg_strerror(int code);

/* Library version as major * 10000 + minor * 100 + patch. */
int bg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BG_MI355X_H */
