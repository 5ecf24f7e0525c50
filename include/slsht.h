/*
 * slsht.h -- C ABI of the MI355X (gfx950) directional SLSHT library.
 *
 * The directional spatially localized spherical harmonic transform of
 * Khalid, Kennedy, Durrani, Sadeghi, Wiaux and McEwen (IEEE Trans. Signal
 * Processing, 2013) maps a band-limited signal f on the sphere and an
 * asymmetric band-limited window h to the distribution
 *
 *     g(rho; l, m) = int_{S^2} f(x) (D_rho h)(x) conj(Y_l^m(x)) ds(x)
 *
 * (Definition 1, eq. Eq:stft_spatial) for rotations rho = (phi, theta, omega)
 * = (alpha, beta, gamma) on an SO(3) grid and spectral indices (l, m).
 *
 * The library evaluates it in separated form: Wigner-3j coupling of f into
 * A^p_q(l, m) = conj((conj(f) Y_l^m)_p^q)  (eqs. Eq:harmonic_formulation and
 * Eq:alternative_harmonic_formulation), then, per (l, m), the contraction with
 * h and Wigner-d(theta) over p, and pruned Fourier synthesis over omega and phi
 * (eq. Eq:alternative_harmonic_formulation_wigner with the separation-of-
 * variables remark of Section IV-B).
 *
 * Conventions used by every entry point:
 *  - Band-limits are exclusive: f_l^m = 0 for l >= L_f, h_s^r = 0 for s >= L_h.
 *    g(.; l, m) vanishes for l >= L_f + L_h - 1 (remark after
 *    Eq:harmonic_formulation).
 *  - Coefficient arrays (f, h, f_out) are complex double, interleaved
 *    (re, im), at flat index l*l + l + m.
 *  - Spherical harmonics carry the Condon-Shortley phase; Wigner-D is
 *    D^l_{m,m'}(alpha,beta,gamma) = e^{-i m alpha} d^l_{m,m'}(beta) e^{-i m' gamma}
 *    (eq. Eq:Dlm); rotations are zyz (Section II-B).
 *  - SO(3) grid (Section II-D, definition of E_L, with per-axis sizes):
 *    phi_a = 2 pi a / n_phi, theta_b = 2 pi b / n_phi (b < n_theta =
 *    (n_phi + 1) / 2, n_phi odd), omega_c = 2 pi c / n_omega.
 *  - Output index of (l, m): lm = l*l + l + m - l_lo*l_lo.
 *    FULL output:   g[lm][c][b - theta_lo][a]  (phi contiguous), complex128
 *                   (SLSHT_FP64) or complex64 (SLSHT_FP32_MIXED).
 *    ENERGY output: E[l - l_lo][c][b - theta_lo][a] = sum_{|m|<=l} |g|^2, float;
 *                   needs SLSHT_FP32_MIXED, n_omega <= 64 and
 *                   ceil(((n_phi+1)/2)/16) * T <= 136, T = ceil(n_omega/16)
 *                   rounded up to 1, 2 or 4 (n_phi <= 1087 for n_omega > 32).
 *  - Device pointers are HIP device memory owned by the caller; the library
 *    never frees them and keeps no reference after a call returns.  A
 *    `stream` argument is a hipStream_t (NULL = the default stream); work is
 *    enqueued asynchronously on it.  slsht_forward, slsht_forward_batch,
 *    slsht_forward_windows, slsht_coupling, slsht_synthesize and slsht_inverse
 *    enqueue kernels only (no allocation, memset or host synchronisation), so
 *    they may be captured in a HIP graph.
 *  - Every function returns an slsht_status; nothing throws across the ABI.
 *    Argument checks run on the host before any launch.  The message of the
 *    last failure on the calling thread is available from slsht_last_error().
 */
#ifndef SLSHT_H
#define SLSHT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SLSHT_OK = 0,
    SLSHT_EINVAL = -1,     /* bad argument or descriptor                        */
    SLSHT_ENOMEM = -2,     /* device or host allocation failed                  */
    SLSHT_EDEVICE = -3,    /* HIP runtime / kernel launch error                 */
    SLSHT_EBUSY = -4,      /* serving: no capacity right now, retry later       */
    SLSHT_ENOTFOUND = -5,  /* serving: unknown ticket                           */
    SLSHT_ETOOBIG = -6     /* serving: request can never fit the HBM budget     */
} slsht_status;

enum { SLSHT_FP64 = 0, SLSHT_FP32_MIXED = 1 };      /* slsht_desc.precision   */
enum { SLSHT_OUT_FULL = 0, SLSHT_OUT_ENERGY = 1 };  /* slsht_desc.output_mode */
/* slsht_desc.flags: f and h are real-signal consistent (c_l^{-m} =
 * (-1)^m conj(c_l^m)), so g(rho; l, -m) = (-1)^m conj(g(rho; l, m))
 * (last remark of Section IV-B); the library then synthesises m >= 0 only.   */
enum { SLSHT_REAL_PAIR = 1u };

#define SLSHT_MAX_LH 32        /* largest supported window band-limit L_h     */
#define SLSHT_MAX_LF 2048      /* largest supported signal band-limit L_f     */
#define SLSHT_MAX_NPHI 2047    /* largest supported n_phi                     */

/* Problem statement (Definition 1; Section IV-A for the grid). */
typedef struct {
    int32_t L_f;          /* signal band-limit, 1 <= L_f <= SLSHT_MAX_LF            */
    int32_t L_h;          /* window band-limit, 1 <= L_h <= SLSHT_MAX_LH            */
    int32_t l_lo, l_hi;   /* output degrees l_lo <= l < l_hi <= L_f + L_h - 1       */
    int32_t n_phi;        /* odd, 1 <= n_phi <= SLSHT_MAX_NPHI                      */
    int32_t n_theta;      /* must equal (n_phi + 1) / 2                             */
    int32_t n_omega;      /* >= 1                                                   */
    int32_t precision;    /* SLSHT_FP64 or SLSHT_FP32_MIXED                         */
    int32_t output_mode;  /* SLSHT_OUT_FULL or SLSHT_OUT_ENERGY                     */
    uint32_t flags;       /* 0 or SLSHT_REAL_PAIR                                   */
    int32_t theta_lo;     /* first theta row computed, 0 <= theta_lo < theta_hi     */
    int32_t theta_hi;     /* one past the last row; 0 means n_theta                 */
    int32_t n_az;         /* azimuthal band-limit of a steerable window: h_s^r = 0  */
                          /* for |r| >= n_az (such coefficients are not read);      */
                          /* 0 <= n_az <= L_h, 0 means L_h (Section IV-B, remark on */
                          /* steerable windows).  The theta and omega contractions  */
                          /* then run over |q'| < n_az only, and n_omega = 2 n_az-1 */
                          /* samples of omega determine g for every omega.          */
} slsht_desc;

typedef struct slsht_plan_s* slsht_plan_t;
typedef struct slsht_server_s* slsht_server_t;

/* Message of the last failure on the calling thread ("" if none). The pointer
 * stays valid until the next library call on this thread. */
const char* slsht_last_error(void);

/* Host-only check of a descriptor against the rules above.  Needs no GPU. */
int slsht_validate(const slsht_desc* desc);

/* Host-only byte counts for a descriptor: device memory a plan holds
 * (Wigner-d table, twiddles, beta weights, coupling scratch, synthesis workspace), the output
 * buffer slsht_forward writes, and per-call scratch.  Any pointer may be NULL.
 * Needs no GPU. */
int slsht_footprint(const slsht_desc* desc, size_t* plan_bytes, size_t* out_bytes,
                    size_t* scratch_bytes);

/* Number of complex coefficients of the coupling output for a descriptor:
 * (l_hi^2 - l_lo^2) * L_h^2.  Needs no GPU. */
int64_t slsht_coupling_size(const slsht_desc* desc);

/* Build a plan on `device`: validates desc, computes the Wigner-d(theta_b)
 * table d^p_{q,q'}(theta_b) for p < L_h, |q|,|q'| <= p (Section II-B,
 * eq. Eq:Dlm) on the GPU in FP64 by the three-term recursion in p (stored in
 * FP32 for SLSHT_FP32_MIXED), the phi and omega twiddles, and the beta weights
 * q(theta_b) of the discrete inverse (Section IV-A).  The plan owns that memory,
 * a coupling scratch of slsht_coupling_size() complex doubles and a synthesis
 * workspace: for ENERGY plans that of the energy kernels (W table, P/M fragments of
 * one chunk of orders, partial energies; up to about 19 GiB), for FULL plans with
 * L_h > 16 the W table and the coupling in MFMA fragment order; included in
 * plan_bytes of slsht_footprint.  Forward,
 * coupling and inverse calls on one plan share that scratch: issue them on one
 * stream, or use one plan per stream.  The tables are built on a private stream
 * that is synchronised before return. */
int slsht_plan(const slsht_desc* desc, int device, slsht_plan_t* out);
int slsht_plan_destroy(slsht_plan_t plan);
/* Copy of the descriptor a plan was built from. */
int slsht_plan_desc(slsht_plan_t plan, slsht_desc* out);

/* Forward transform (Definition 1, evaluated as described at the top):
 *   f: device, complex128[L_f * L_f]      signal coefficients f_l^m
 *   h: device, complex128[L_h * L_h]      window coefficients h_s^r
 *   g: device, FULL or ENERGY layout above, caller-allocated, at least
 *      out_bytes of slsht_footprint()
 * With SLSHT_REAL_PAIR set, f and h must be real-signal consistent (not
 * checked); m < 0 outputs are then written from m > 0 by the conjugate
 * symmetry.  Asynchronous on `stream`. */
int slsht_forward(slsht_plan_t plan, const void* f, const void* h, void* g, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the transform of
 * slsht_forward on the same plan, f, h and g, with the coupling scratch taken
 * from a static device array of SLSHT_NOALLOC_SCRATCH_BYTES per GPU instead of
 * the plan's own buffer.  The call allocates and frees nothing.  Results equal
 * slsht_forward's.  The array's device address is resolved once per device, at
 * the first slsht_plan (or first call) on it.
 * SLSHT_ETOOBIG if the coupling scratch, (l_hi^2 - l_lo^2) * L_h^2 * 16 bytes,
 * exceeds SLSHT_NOALLOC_SCRATCH_BYTES.  Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents: calls that overlap on one GPU
 * (on several streams, or from several threads) race; issue them on one
 * stream.  Asynchronous on `stream`. */
#define SLSHT_NOALLOC_SCRATCH_BYTES (64u << 20)
int slsht_forward_noalloc(slsht_plan_t plan, const void* f, const void* h, void* g, void* stream);

/* Coupling stage alone: A[lm][p*p + p + q] = sum_{l'} f_{l'}^{m-q} T(l', m-q; p, q; l, m)
 * = int f Y_p^q conj(Y_l^m) ds, the coefficient that multiplies
 * h_p^{q'} D^p_{q,q'}(rho) in Eq:harmonic_formulation (it equals
 * conj((conj(f) Y_l^m)_p^q) of Eq:alternative_harmonic_formulation).
 *   f: device complex128[L_f * L_f];  A: device complex128[slsht_coupling_size()].
 * Useful to analyse several windows against one signal (remark on multiple
 * windows, Section IV-B).  Asynchronous on `stream`. */
int slsht_coupling(slsht_plan_t plan, const void* f, void* A, void* stream);

/* Synthesis stage alone, from a given coupling (the rest of slsht_forward after
 * slsht_coupling; separation of variables of Section IV-B):
 *   A: device complex128[slsht_coupling_size()], layout of slsht_coupling;
 *   h, g: as for slsht_forward on this plan.
 * Lets a caller reuse one coupling for several windows, and time the synthesis
 * kernels by themselves.  Asynchronous on `stream`; ENERGY plans and FULL plans with
 * L_h > 16 use the plan's workspace, so calls on one plan are issued on one stream. */
int slsht_synthesize(slsht_plan_t plan, const void* A, const void* h, void* g, void* stream);

/* Several forward transforms in few launches (continuous batching, Section IV-B's
 * separated form for each): the couplings of all n plans, then one synthesis grid per
 * group of up to 16 FULL plans that share a synthesis kernel (same precision, band-limit
 * bucket and phi-slot class), its blocks split between the transforms by a tile list;
 * ENERGY plans get their own launch.  Results equal n separate slsht_forward calls.
 *   plans: n distinct plans on one device (each plan's coupling scratch is used);
 *   f[i], h[i], g[i]: device pointers as for slsht_forward on plans[i].
 * n >= 1 (SLSHT_EINVAL otherwise, also for a repeated plan or a NULL entry).
 * Asynchronous on `stream`. */
int slsht_forward_batch(int n, const slsht_plan_t* plans, const void* const* f,
                        const void* const* h, void* const* g, void* stream);

/* Forward transform of one signal against several windows (remark on multiple
 * windows, Section IV-B): the coupling of f is computed once and shared; each
 * window then costs one synthesis.  Same plan rules as slsht_forward.
 *   f: device, complex128[L_f * L_f]
 *   h: device, complex128[n_windows][L_h * L_h]
 *   g: device, n_windows consecutive outputs of slsht_forward's layout, each
 *      out_bytes of slsht_footprint() long
 * n_windows >= 1 (SLSHT_EINVAL otherwise).  Asynchronous on `stream`. */
int slsht_forward_windows(slsht_plan_t plan, const void* f, const void* h, int n_windows,
                          void* g, void* stream);

/* Inverse through the spectral marginal (Section III-C): for every (l, m) of the
 * plan,  f_hat = (1/(n_phi^2 n_omega)) sum_{a,b,c} q(theta_b) g(phi_a, theta_b, omega_c; l, m)
 * (eq. Eq:sig_reconstruction_discrete with per-axis sizes), and
 * f_out[lm] = f_hat / (sqrt(16 pi^3) h_0^0)  (eq. Eq:inversion_2).  The result is
 * f_l^m for l < L_f and zero (to rounding) for l >= L_f.
 *   g: device, FULL layout of this plan;  h: device complex128[L_h * L_h] (only
 *   h_0^0 is read, by the kernel);
 *   f_out: device complex128[l_hi^2 - l_lo^2].
 * Requires a FULL plan over all theta rows with n_phi >= 2 L_h - 1 and
 * n_omega >= 2 n_az - 1 (n_az = L_h unless the window is steerable)
 * (SLSHT_EINVAL otherwise).  The inverse divides by h_0^0, which the library
 * does not read on the host: h_0^0 = 0 gives non-finite f_out, not an error
 * status.  Asynchronous on `stream`, kernels only. */
int slsht_inverse(slsht_plan_t plan, const void* g, const void* h, void* f_out, void* stream);

/* The paper's own route, for comparison (factoring of rotations, Section IV-B):
 * on its minimal grid E_{L_h} (n_phi = n_omega = 2 L_h - 1, n_theta = L_h), g is a
 * 3-D Fourier sum of
 *   C_{q,q'',q'}(l,m) = i^{q-q'} sum_p A^p_q h_p^{q'} Delta^p_{q'',q} Delta^p_{q'',q'},
 * Delta^p = d^p(pi/2) (eq. Eq:WignerD_expansion_new), evaluated on the fly by the
 * recursion of Trapani and Navaza as the paper does.  Computed in FP64 over a
 * caller-provided workspace: Delta, the window factor of C, then per (l, m) the C
 * slices with their omega and theta sums, then the phi sums.
 * slsht_factored_workspace(desc): bytes needed, or -1 (SLSHT_EINVAL in
 * slsht_last_error) unless desc is FULL, FP64, on that grid, over all theta rows,
 * without flags or a steerable limit, with n_lm * L_h <= 2^31 - 1.
 * slsht_forward_factored: same f, h, g as slsht_forward on such a plan (coupling by
 * slsht_coupling's 3j route, then the factored synthesis); work is device memory of at
 * least work_bytes >= slsht_factored_workspace(); asynchronous.
 * slsht_synthesize_factored: the factored synthesis alone from a given coupling
 *   A: device complex128[slsht_coupling_size()], layout of slsht_coupling
 * (the paper's tau_2 stage of its timing experiment, Section V); same rules. */
int64_t slsht_factored_workspace(const slsht_desc* desc);
int slsht_forward_factored(slsht_plan_t plan, const void* f, const void* h, void* g, void* work,
                           size_t work_bytes, void* stream);
int slsht_synthesize_factored(slsht_plan_t plan, const void* A, const void* h, void* g,
                              void* work, size_t work_bytes, void* stream);

/* Delta^p_{Q,Q'} = d^p_{Q,Q'}(pi/2) for p < L_h, 0 <= Q <= p, -Q <= Q' <= Q, by the
 * Trapani-Navaza recursion (Section IV-B): each column seeded on the edge Q = p by
 * Wigner's formula, then run down in Q by the three-term relation of d at pi/2.
 *   delta: device float64[L_h (L_h+1) (2 L_h+1) / 6], entry (p, Q, Q') at
 *          p (p+1) (2p+1) / 6 + Q^2 + Q + Q'; the other entries follow from
 *          Delta_{q,q'} = (-1)^{q-q'} Delta_{q',q} = Delta_{-q',-q}.
 * 1 <= L_h <= SLSHT_MAX_LH (SLSHT_EINVAL otherwise).  Asynchronous on `stream` of
 * `device`; the caller owns delta. */
int slsht_wigner_delta(int L_h, int device, void* delta, void* stream);

/* Coupling through the spherical harmonic transform of the modulated signal
 * conj(f) Y_l^m (Appendix A, eq. Eq:sht_sep_variable): the paper's tau_1 stage.  Same
 * result and layout as slsht_coupling (which uses 3j symbols instead):
 *   A[lm][p*p + p + q] = 2 pi sum_j w_j lam_l^m(theta_j) lam_p^q(theta_j) F_{m-q}(theta_j),
 *   F_mu(theta) = sum_{l'} f_{l'}^mu lam_{l'}^mu(theta),  lam_l^m Y_l^m's theta factor,
 * summed over n = ((L_f-1) + (l_hi-1) + (L_h-1)) / 2 + 1 Gauss-Legendre nodes in
 * cos(theta), exact for this integrand; FP64 for every plan precision.
 * slsht_modulated_workspace(desc): bytes of device workspace (nodes, weights, F and
 * the Legendre values of the l-window and of p < L_h), or -1 for an invalid desc.
 * slsht_coupling_modulated: f device complex128[L_f * L_f]; A device
 * complex128[slsht_coupling_size()]; work device memory of work_bytes >=
 * slsht_modulated_workspace() (SLSHT_EINVAL otherwise).  Asynchronous on `stream`;
 * the workspace may be reused once the call's work on the stream has finished. */
int64_t slsht_modulated_workspace(const slsht_desc* desc);
int slsht_coupling_modulated(slsht_plan_t plan, const void* f, void* A, void* work,
                             size_t work_bytes, void* stream);

/* Slepian eigenfunction window (Section III-D): among functions band-limited to
 * s < L_h, the one with the largest energy concentration in the elliptical region
 * R_(theta_c, a) = {x : dist(x, (theta_c, 0)) + dist(x, (theta_c, pi)) <= 2a}
 * (eq. Eq:region_def), 0 <= theta_c < a <= pi/2 (theta_c = 0: polar cap of radius a).
 * The concentration matrix is summed by quadrature on `device` in FP64, its top
 * eigenvector found on the host; synchronous.
 *   h_out: host complex128[L_h * L_h], unit energy, real-signal consistent
 *          (h_s^{-r} = (-1)^r conj(h_s^r)), sign fixed by a positive largest entry
 *   concentration: host, int_R |h|^2 (may be NULL)
 * SLSHT_EINVAL for arguments outside those ranges. */
int slsht_slepian_window(int L_h, double theta_c, double a, int device, void* h_out,
                         double* concentration);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of forward transforms of uneven size.
 *
 * A server owns one worker thread, device tables cached by descriptor, and an
 * HBM budget for request outputs and inputs.  Requests are admitted in arrival
 * order as budget frees up (a later, smaller request may pass a head that does
 * not fit yet).  The requests admitted in one scheduling round are launched
 * together: FULL transforms that share a synthesis kernel run in one grid of up
 * to 16 transforms (as slsht_forward_batch), each group on the next of the
 * server's streams, so the work of different requests overlaps on the device.
 * Results stay in server-owned device memory until released; each equals the
 * same transform run alone through slsht_forward, bit for bit.
 */
enum { SLSHT_REQ_QUEUED = 0, SLSHT_REQ_RUNNING = 1, SLSHT_REQ_DONE = 2, SLSHT_REQ_FAILED = 3 };

/* hbm_budget: bytes of device memory the server may hold for request inputs and
 * outputs together; n_streams: device streams used for concurrent requests (1..8). */
int slsht_server_create(int device, size_t hbm_budget, int n_streams, slsht_server_t* out);
/* Waits for in-flight work, then frees every buffer, plan and stream. */
int slsht_server_destroy(slsht_server_t server);
/* Copies f (complex128[L_f^2]) and h (complex128[L_h^2]) from host memory and
 * queues the request; returns a ticket.  SLSHT_ETOOBIG if the request alone
 * exceeds the budget, SLSHT_EINVAL for a bad descriptor. */
int slsht_submit(slsht_server_t server, const slsht_desc* desc, const void* f_host,
                 const void* h_host, uint64_t* ticket);
/* Non-blocking state query.  When DONE, *g_dev is the device output (layout of
 * slsht_forward) and *out_bytes its size; when FAILED, *err holds the status. */
int slsht_poll(slsht_server_t server, uint64_t ticket, int* state, const void** g_dev,
               size_t* out_bytes, int* err);
/* Blocks until the request is DONE or FAILED (or timeout_ms elapses: EBUSY). */
int slsht_wait(slsht_server_t server, uint64_t ticket, int timeout_ms);
/* Returns a finished request's output memory to the budget; the server may hand it to
 * the next admitted request at once, so any work of the caller that reads *g_dev
 * (copies, kernels, on any stream) must have completed before this call. */
int slsht_release(slsht_server_t server, uint64_t ticket);
/* Timestamps (seconds on the server's monotonic clock) of a finished request:
 * submit, admission (enqueue) and completion.  Any pointer may be NULL. */
int slsht_request_times(slsht_server_t server, uint64_t ticket, double* t_submit,
                        double* t_start, double* t_done);
/* Current server clock (same origin as slsht_request_times). */
double slsht_server_clock(slsht_server_t server);
/* Snapshot of the server: bytes of the HBM budget held by admitted requests (inputs,
 * scratch and unreleased outputs), the budget itself, and the number of queued and
 * running requests.  Any pointer may be NULL. */
int slsht_server_stats(slsht_server_t server, size_t* used_bytes, size_t* budget_bytes,
                       int* n_queued, int* n_running);

#ifdef __cplusplus
}
#endif

#endif /* SLSHT_H */
