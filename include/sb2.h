/* sb2 -- second-Born self-energy and GKBA collision integral on MI355X (gfx950).
 *
 * C ABI of the library libsb2.so.  Method: Tuovinen, Covito & Sentef,
 * "Efficient computation of the second-Born self-energy using tensor-contraction
 * operations" (arXiv:1905.01180).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Pointers named v, h, G*, S*, rho*, I*, g* are DEVICE pointers owned by the
 *    caller.  ws is a caller-owned device workspace of at least
 *    sb2_workspace_size(...) bytes, 256-byte aligned.  The library allocates no
 *    memory, creates no streams and never synchronises the device inside these
 *    calls: all work is enqueued on `stream` (a hipStream_t passed as void*;
 *    NULL is the default stream) and the call returns once it is enqueued.
 *  * Complex matrices are row-major, interleaved (re, im) float64 pairs (the
 *    layout of a C99 double complex / torch.complex128 tensor).  An N x N matrix
 *    X has X_ij at element i*N + j.  Stacks of matrices are contiguous.
 *  * v is the real two-body tensor v_ijkl of Eq. 3, float64, element
 *    ((i*N + j)*N + k)*N + l.  No permutation symmetry of v is assumed unless
 *    an entry point says so.
 *  * Time grid: past times t_k = k*dt for k = 0..T-1; "now" is t = T*dt.
 *    rho_hist[k] = rho(t_k), the one-particle density matrix -i G^<(t_k, t_k).
 *  * Return value: SB2_OK or a negative sb2_status.  Argument errors are
 *    detected on the host before anything is enqueued (outputs untouched).
 *    A HIP launch failure returns SB2_EHIP.  An error that an earlier
 *    asynchronous failure left in the HIP runtime (of this library's work or
 *    any other) is returned as SB2_EHIP by the next call that would enqueue
 *    work, and cleared; device faults also surface through the HIP runtime on
 *    the caller's next synchronisation.
 *  * Inputs are assumed Hermitian where the physics says so (h, rho_k); NaN or
 *    Inf inputs propagate to the outputs.  With the environment variable
 *    SB2_CHECK=1 every entry point that enqueues work first checks its inputs
 *    on the device (all values finite; h and every rho_k Hermitian to 1e-10
 *    relative to max(1, max |entry|)) and returns SB2_ECHECK, with nothing
 *    else enqueued, if one fails.  The check synchronises the stream (it
 *    copies three words to the host), so it is for debugging, not for timed
 *    runs or stream capture.
 *  * prec selects the arithmetic of the bulk tensor contractions only.  The
 *    propagators, GKBA two-time functions, the sum over past times and every
 *    output stay float64:
 *      SB2_FP64        complex float64 on the FP64 matrix cores,
 *      SB2_FP32        complex float32 on the FP32 matrix cores, float32 sums
 *                      folded into float64 along the long contraction,
 *      SB2_SPLIT_FP16  each float32 operand split into two scaled float16 pieces,
 *                      three float16 products per real product (hi*hi + hi*lo +
 *                      lo*hi) with float32 accumulation on the FP16 matrix cores,
 *      SB2_SPLIT_BF16  not built (SB2_EUNSUPPORTED): two bfloat16 pieces carry
 *                      16 significant bits (about 1e-5, short of the 1e-6 target)
 *                      and three pieces need six products per real product at
 *                      the FP16 rate, twice the cost of SB2_SPLIT_FP16 for the
 *                      same accuracy.
 *  * Calls that share a workspace must be ordered on one stream.
 */
#ifndef SB2_H
#define SB2_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SB2_OK = 0,
  SB2_EINVAL = -1,       /* null pointer, non-finite or non-positive dt, bad enum   */
  SB2_ESHAPE = -2,       /* N or T out of range                                     */
  SB2_EWORKSPACE = -3,   /* ws_bytes smaller than sb2_workspace_size(...)           */
  SB2_EHIP = -4,         /* a HIP runtime call or kernel launch failed              */
  SB2_EUNSUPPORTED = -5, /* precision not available for this entry point            */
  SB2_ESCRATCH = -6,     /* sb2_collision_noalloc: problem too large for its static
                            scratch buffer                                          */
  SB2_ECHECK = -7        /* SB2_CHECK=1 input check failed                          */
} sb2_status;

typedef enum {
  SB2_FP64 = 0,
  SB2_FP32 = 1,
  SB2_SPLIT_FP16 = 2,
  SB2_SPLIT_BF16 = 3     /* recognised, not built: every entry point returns SB2_EUNSUPPORTED */
} sb2_precision;

/* Operation codes for sb2_workspace_size. */
typedef enum {
  SB2_OP_SIGMA = 0,
  SB2_OP_COLLISION = 1,
  SB2_OP_COLLISION_BACKWARD = 2,
  SB2_OP_RHO_STEP = 3,
  SB2_OP_AUTOTUNE = 4,
  SB2_OP_PROPAGATE = 5,
  SB2_OP_COLLISION_DIAGONAL = 6,
  SB2_OP_COLLISION_SYMMETRIC = 7,
  SB2_OP_PROPAGATE_DIAGONAL = 8,
  SB2_OP_PROPAGATE_SYMMETRIC = 9,
  SB2_OP_PROPAGATE_LINEAR = 10
} sb2_op;

/* Largest basis size and history length accepted. */
#define SB2_MAX_N 128
#define SB2_MAX_T 65536

/* sb2_sigma -- second-Born self-energies for B pairs of times (Sec. III, Eq. 13).
 *
 *   Sigma_ij = sum_{mnpqrs} v_irpn (2 v_mqsj - v_qmsj) G_nm G_pq Gbar_sr,
 *
 * which is Eq. 13 with the exchange term's summation indices renamed; it holds
 * for any real v.  For pair b, Gl[b] = G^<(t, t'_b) and Gg[b] = G^>(t, t'_b)
 * (N x N complex each); the reversed-time functions are formed internally as
 * Gbar = G(t', t) = -G(t, t')^dagger (Sec. II), and
 *   Sl[b] = Sigma^<(t, t'_b) = Sigma(G = Gl[b], Gbar = -Gg[b]^dagger),
 *   Sg[b] = Sigma^>(t, t'_b) = Sigma(G = Gg[b], Gbar = -Gl[b]^dagger).
 * Outputs are B x N x N complex float64, overwritten.
 * Errors: SB2_ESHAPE for N < 1, N > SB2_MAX_N or B < 1; SB2_EINVAL for null
 * pointers or an unknown prec; SB2_EWORKSPACE.                                */
int sb2_sigma(int N, int B, const double* v, const void* Gl, const void* Gg,
              void* Sl, void* Sg, int prec, void* ws, size_t ws_bytes, void* stream);

/* sb2_collision -- GKBA collision integral (Sec. II, Eqs. 9-11).
 *
 *   I(t) = dt * sum_{k=0}^{T-1} [ Sigma^>(t, t_k) G^<(t_k, t) - Sigma^<(t, t_k) G^>(t_k, t) ]
 *
 * the first two terms of Eq. 9 on the left-rectangle grid (the last two terms
 * are the Hermitian conjugate of these, so Eq. 9's integral is I + I^dagger).
 * Two-time functions come from the GKBA (Eq. 10) with the HF propagator of
 * Eq. 11 for the frozen one-body matrix h: U_k = exp(-i h (T-k) dt),
 *   G^<(t,t_k) = i U_k rho_k,      G^>(t,t_k) = -i U_k (1 - rho_k),
 *   G^<(t_k,t) = i rho_k U_k^dag,  G^>(t_k,t) = -i (1 - rho_k) U_k^dag.
 * h: N x N complex; rho_hist: T x N x N complex; I_out: N x N complex (overwritten).
 * Sigma_out: optional (may be NULL) 2 x T x N x N complex receiving
 *   Sigma_out[0][k] = Sigma^<(t, t_k), Sigma_out[1][k] = Sigma^>(t, t_k).
 * Errors: SB2_ESHAPE (N, T out of range), SB2_EINVAL (null pointer, dt not
 * finite or <= 0, unknown prec), SB2_EWORKSPACE.                              */
int sb2_collision(int N, int T, const double* v, const void* h, const void* rho_hist, double dt,
                  void* I_out, void* Sigma_out, int prec, void* ws, size_t ws_bytes, void* stream);

/* sb2_collision_backward -- adjoint of sb2_collision (FP64 only).
 *
 * Given gI = dL/dI for a real scalar L in torch's convention
 * (gI = dL/dRe I + i dL/dIm I, N x N complex), writes
 *   gv   = dL/dv          N^4 float64 (v treated as an unconstrained real tensor),
 *   gh   = dL/dh          N x N complex (h treated as an unconstrained complex
 *                         matrix; the propagators' dependence on h goes through
 *                         the chain U_k = U_1^(T-k), U_1 = exp(-i h dt)),
 *   grho = dL/drho_hist   T x N x N complex,
 * all in the same convention and overwritten.  The GKBA functions and the
 * contraction intermediates are recomputed, not stored.
 * Errors: as sb2_collision; SB2_EUNSUPPORTED for prec != SB2_FP64.          */
int sb2_collision_backward(int N, int T, const double* v, const void* h, const void* rho_hist, double dt,
                           const void* gI, double* gv, void* gh, void* grho,
                           int prec, void* ws, size_t ws_bytes, void* stream);

/* sb2_collision_noalloc -- sb2_collision for callers that cannot allocate
 * device memory (code under HIP graph capture that must not allocate, tight
 * serving loops, harnesses that forbid hipMalloc): no workspace argument, no
 * allocation of any kind.  Its scratch memory is one static device buffer of
 * SB2_NOALLOC_SCRATCH_BYTES per device, held from the library's first use on
 * that device until the process ends; the chunk of past times one pass of the
 * contraction chain holds is the largest whose workspace fits it (results
 * equal sb2_collision's up to the order of float32 accumulation).
 * Arguments and outputs as for sb2_collision.  Every call on a device shares
 * that device's buffer: calls that overlap on one device (other streams,
 * other host threads) race and give wrong results; calls ordered on one
 * stream are safe (each call initialises what it reads).
 * Errors: as sb2_collision; SB2_ESCRATCH (nothing enqueued) when even one
 * past time per pass needs more than SB2_NOALLOC_SCRATCH_BYTES (about N > 40
 * for SB2_FP32 / SB2_SPLIT_FP16, N > 32 for SB2_FP64).                       */
#define SB2_NOALLOC_SCRATCH_BYTES (128u << 20)
int sb2_collision_noalloc(int N, int T, const double* v, const void* h, const void* rho_hist, double dt,
                          void* I_out, void* Sigma_out, int prec, void* stream);

/* sb2_collision_prop -- sb2_collision with the propagators supplied by the
 * caller: U_hist[k] = U(t, t_k), k = 0..T-1 (T x N x N complex), the HF
 * propagators of Eq. 11 for any (time-dependent) effective one-body matrix.
 * The GKBA functions (Eq. 10) and I(t) are formed from U_hist and rho_hist
 * exactly as in sb2_collision; with U_hist[k] = exp(-i h (T-k) dt) the two
 * calls agree up to the rounding of the propagators.  Workspace:
 * sb2_workspace_size(SB2_OP_COLLISION, N, T, prec).  Errors: as sb2_collision. */
int sb2_collision_prop(int N, int T, const double* v, const void* U_hist, const void* rho_hist, double dt,
                       void* I_out, void* Sigma_out, int prec, void* ws, size_t ws_bytes, void* stream);

/* Special interaction vertices of Sec. III. */
typedef enum {
  SB2_VERTEX_DIAGONAL = 1,   /* v_ijkl = U_i d_ij d_ik d_il (Hubbard-like), parameter U: N float64  */
  SB2_VERTEX_SYMMETRIC = 2   /* v_ijkl = V_ij d_il d_jk (density-density), parameter V: N x N float64 */
} sb2_vertex;

/* sb2_collision_vertex -- sb2_collision for a special vertex, float64 throughout.
 * The GKBA functions and the sum over past times are those of sb2_collision
 * (Eqs. 9-11); the self-energy is
 *   diagonal basis (Eq. 14):  Sigma_ij = U_i U_j G_ij Gbar_ji G_ij                         O(N^2)
 *   symmetric basis (Eq. 16): Sigma = 2 G o [(V x {[V x (Gbar^T o G)]}^T)^T]   (Eq. 17, bubble)
 *                             - sum_kl V_ik V_jl G_il Gbar_lk G_kj               (exchange) O(N^4)
 * with G, Gbar as in sb2_collision.  vparam: U (N float64) or V (N x N
 * float64, row-major, V[i][j] = V_ij), device pointer.  h, rho_hist, I_out,
 * Sigma_out as for sb2_collision.  Workspace: sb2_workspace_size(
 * SB2_OP_COLLISION_DIAGONAL or SB2_OP_COLLISION_SYMMETRIC, N, T, any prec).
 * Errors: as sb2_collision; SB2_EINVAL for an unknown vertex.                */
int sb2_collision_vertex(int N, int T, int vertex, const double* vparam, const void* h, const void* rho_hist,
                         double dt, void* I_out, void* Sigma_out, void* ws, size_t ws_bytes, void* stream);

/* 8-fold packed interaction tensor.  For real basis functions the Coulomb
 * integrals of Eq. 3 obey the 8-point symmetry of Eq. 4: v_ijkl depends only
 * on the unordered pairs {i, l} (both orbitals at r) and {j, k} (at r') and
 * is unchanged when the two pairs are exchanged.  Packed storage keeps one
 * float64 per orbit:
 *   pair(a, b) = max(a,b) (max(a,b) + 1) / 2 + min(a,b)
 *   packed[pair(pair(i, l), pair(j, k))] = v_ijkl
 * sb2_v8_count: number of packed values, P (P + 1) / 2 with P = N (N + 1) / 2
 * (about N^4 / 8); 0 for N out of range.
 * sb2_v8_expand: write the full N^4 tensor v (row-major v[i][j][k][l], as the
 * other entry points take it) from the packed values; device pointers,
 * enqueued on stream.  Errors: SB2_ESHAPE, SB2_EINVAL (null pointer).       */
size_t sb2_v8_count(int N);
int sb2_v8_expand(int N, const double* packed, double* v, void* stream);

/* sb2_collision_v8 -- sb2_collision with the interaction given as its 8-fold
 * packed values (vpacked: sb2_v8_count(N) float64, layout as above; the full
 * tensor is never formed: the layout kernels read the packed values
 * directly).  Only for v with the symmetry of Eq. 4.  Results are bit for bit
 * those of sb2_collision with v = sb2_v8_expand(vpacked).  Workspace:
 * sb2_workspace_size(SB2_OP_COLLISION, N, T, prec).  Errors: as sb2_collision. */
int sb2_collision_v8(int N, int T, const double* vpacked, const void* h, const void* rho_hist, double dt,
                     void* I_out, void* Sigma_out, int prec, void* ws, size_t ws_bytes, void* stream);

/* Terms of the equation of motion included by sb2_gkba_propagate. */
typedef enum {
  SB2_PROP_HF = 1,         /* Sigma_HF (Eq. 12) in the propagator and the commutator */
  SB2_PROP_COLLISION = 2   /* the second-Born collision integral (Eq. 9)             */
} sb2_prop_flags;

/* sb2_gkba_propagate -- advance the GKBA density-matrix propagation (Sec. II,
 * Eqs. 8-12; time-stepping without predictor-corrector as in Sec. IV) from
 * step n0 to step n0 + nsteps, on the device, without host synchronisation.
 * Time grid t_n = n dt.  Per step n:
 *   h_HF(t_n)  = h + Sigma_HF(rho_n),   (Sigma_HF)_ij = sum_kl (2 v_iklj - v_ikjl) rho_lk
 *   U_step     = exp(-i h_HF(t_n) dt)
 *   I_n        = sb2_collision_prop over the past times t_0 .. t_{n-1} with
 *                U(t_n, t_k) (I_0 = 0)
 *   rho_{n+1}  = U_step rho_n U_step^dag - dt (I_n + I_n^dag)
 *   U(t_{n+1}, t_k) = U_step U(t_n, t_k) for k < n,  U(t_{n+1}, t_n) = U_step,
 * i.e. the time-ordered exponential of Eq. 11 with h_HF sampled at the start of
 * each step.  Without SB2_PROP_HF the bare h is used; without
 * SB2_PROP_COLLISION I_n = 0.
 * State (caller-owned device memory, complex, row-major N x N slices):
 *   rho_hist  capacity >= n0 + nsteps + 1 slices; rho_hist[0..n0] are read,
 *             rho_hist[n0+1 .. n0+nsteps] are written;
 *   U_hist    capacity >= n0 + nsteps slices; on entry U_hist[k] = U(t_n0, t_k)
 *             for k < n0, on return U(t_{n0+nsteps}, t_k) for k < n0 + nsteps;
 *   I_hist    optional (may be NULL), capacity >= n0 + nsteps slices;
 *             I_hist[n] = I_n is written for n0 <= n < n0 + nsteps.
 * The state after a call is the input of the next (checkpoint = these three
 * arrays and n).  h: N x N complex, v: N^4 float64, as for sb2_collision.
 * Workspace: sb2_workspace_size(SB2_OP_PROPAGATE, N, n0 + nsteps, prec).
 * Errors: SB2_ESHAPE (N out of range, n0 < 0, nsteps < 1, n0 + nsteps >
 * SB2_MAX_T), SB2_EINVAL (null pointer, dt not finite or <= 0, unknown prec
 * or flags), SB2_EWORKSPACE.                                                  */
int sb2_gkba_propagate(int N, int n0, int nsteps, const double* v, const void* h, void* rho_hist, void* U_hist,
                       void* I_hist, double dt, int flags, int prec, void* ws, size_t ws_bytes, void* stream);

/* sb2_gkba_propagate_switched -- sb2_gkba_propagate with a time-dependent
 * interaction strength: the Hamiltonian is h + lambda(t) V, as in the
 * adiabatic switching by which Sec. II prepares a correlated state from an
 * uncorrelated one.  lambda: device array of n0 + nsteps float64 values,
 * lambda[m] = lambda(t_m).  The HF self-energy at t_n carries lambda(t_n) and
 * the second-Born self-energy Sigma(t_n, t_k), whose two interaction lines sit
 * at t_n and t_k, carries lambda(t_n) lambda(t_k):
 *   h_HF(t_n) = h + lambda_n Sigma_HF(rho_n),
 *   I_n = dt lambda_n sum_k lambda_k [Sigma^>_k G^<(t_k,t_n) - Sigma^<_k G^>(t_k,t_n)],
 * everything else as in sb2_gkba_propagate (same workspace size).
 * Errors: as sb2_gkba_propagate; SB2_EINVAL for lambda == NULL.            */
int sb2_gkba_propagate_switched(int N, int n0, int nsteps, const double* v, const void* h, void* rho_hist,
                                void* U_hist, void* I_hist, const double* lambda, double dt, int flags, int prec,
                                void* ws, size_t ws_bytes, void* stream);

/* sb2_gkba_propagate_linear -- the propagation of sb2_gkba_propagate
 * (HF propagators, float64 throughout) with the sum over past times of the
 * collision integral (Eq. 9) carried along instead of recomputed.  The step
 * propagators of Eq. 11 compose, U(t_n, t_k) = P_n P_k^dag with
 * P_n = U(t_n, t_0), so each GKBA function of Eq. 10 is P_n (or P_n^dag)
 * times a function of t_k alone, and P_n acts only on the three t-side legs
 * of the interaction in Eq. 13:
 *   I(t_n) = dt [sum_{(n,p,r)} vt_n[i][(n,p,r)] M_n[(n,p,r)][l]] P_n^dag,
 *   vt_n[i][(n,p,r)] = sum v_{i r' p' n'} P_{n' n} P_{p' p} conj(P_{r' r}),
 *   M_n = sum_{k<n} (Ct^>_k abar_k - Ct^<_k bbar_k),
 * with abar_k = i rho_k P_k, bbar_k = -i (1 - rho_k) P_k and Ct^<_k, Ct^>_k
 * the first three contractions of the chain on the functions of past time k
 * (a_k = i P_k^dag rho_k, b_k = -i P_k^dag (1 - rho_k)).  Each step adds one
 * past time to M and rotates v once: O(N^5) work per step instead of
 * O(n N^5), with I equal to that of sb2_gkba_propagate up to rounding.
 *   P        device, N x N complex, caller-owned state: P_{n0} on entry,
 *            P_{n0+nsteps} on return (set to 1 by the call when n0 = 0);
 *   M        device, N^4 complex, caller-owned state (row (p,r,n), column
 *            l: M[((p N + r) N + n) N + l]); M_{n0} on entry (zeroed by the
 *            call when n0 = 0), M_{n0+nsteps} on return;
 *   lambda   optional (NULL: constant coupling 1) device array of n0 + nsteps
 *            float64 values lambda(t_m), the interaction being lambda(t) v as
 *            in sb2_gkba_propagate_switched: past time k joins M weighted by
 *            lambda(t_k), I(t_n) and Sigma_HF(t_n) carry lambda(t_n);
 *   rho_hist, I_hist, flags: as sb2_gkba_propagate (a resumed propagation
 *            keeps the flags and the coupling history: past times join M
 *            only with SB2_PROP_COLLISION set).  No U history is kept.
 * Workspace: sb2_workspace_size(SB2_OP_PROPAGATE_LINEAR, N, any T, any prec)
 * (independent of the history length).  Errors: as sb2_gkba_propagate (no
 * prec argument); SB2_EINVAL for P or M == NULL.                          */
int sb2_gkba_propagate_linear(int N, int n0, int nsteps, const double* v, const void* h, void* rho_hist, void* P,
                              void* M, void* I_hist, const double* lambda, double dt, int flags, void* ws,
                              size_t ws_bytes, void* stream);

/* sb2_gkba_propagate_qp -- sb2_gkba_propagate with correlated (quasiparticle)
 * propagators in the GKBA, the extension the Conclusion names beside GW,
 * T-matrix and initial correlations: the propagators of Eq. 11 that build the
 * two-time functions of Eq. 10 are generated by h_HF(t) + sigma_qp instead of
 * h_HF(t), with sigma_qp a constant N x N complex matrix (device, row-major,
 * caller-owned), for example -i Gamma/2 with Gamma Hermitian positive
 * semidefinite (a quasiparticle damping); a Hermitian part shifts the
 * quasiparticle energies.  Per step n:
 *   U_step(n)   = exp(-i h_HF(t_n) dt)               advances the density (Eq. 8),
 *   Uqp_step(n) = exp(-i (h_HF(t_n) + sigma_qp) dt)  advances the history,
 *   U_hist[k]   = U_qp(t_n, t_k) = Uqp_step(n-1) ... Uqp_step(k),
 * and I_n is the collision integral of these propagators (sb2_collision_prop).
 * sigma_qp = 0 reproduces sb2_gkba_propagate bit for bit.  Everything else,
 * the workspace size and the errors as sb2_gkba_propagate; SB2_EINVAL for
 * sigma_qp == NULL.                                                         */
int sb2_gkba_propagate_qp(int N, int n0, int nsteps, const double* v, const void* h, const void* sigma_qp,
                          void* rho_hist, void* U_hist, void* I_hist, double dt, int flags, int prec, void* ws,
                          size_t ws_bytes, void* stream);

/* sb2_gkba_propagate_vertex -- sb2_gkba_propagate for a special vertex of
 * Sec. III (Sec. IV runs its chains this way), float64 throughout.  Per step
 * n exactly the scheme of sb2_gkba_propagate, with
 *   Sigma_HF (Eq. 12 for the vertex):  diagonal basis  diag(U_i rho_ii),
 *                                      symmetric basis 2 diag(sum_k V_ik rho_kk) - V o rho
 *   I_n: the collision integral of sb2_collision_vertex (self-energy of Eq. 14
 *        or Eqs. 16-17) with the supplied propagators U(t_n, t_k).
 * vertex, vparam as for sb2_collision_vertex; state arrays, flags and errors
 * as for sb2_gkba_propagate (no prec argument).  Workspace:
 * sb2_workspace_size(SB2_OP_PROPAGATE_DIAGONAL or SB2_OP_PROPAGATE_SYMMETRIC,
 * N, n0 + nsteps, any prec).  Errors: as sb2_gkba_propagate; SB2_EINVAL for
 * an unknown vertex.                                                          */
int sb2_gkba_propagate_vertex(int N, int n0, int nsteps, int vertex, const double* vparam, const void* h,
                              void* rho_hist, void* U_hist, void* I_hist, double dt, int flags, void* ws,
                              size_t ws_bytes, void* stream);

/* One system of a batched collision-integral evaluation. */
typedef struct {
  int N, T;
  double dt;
  const double* v;       /* N^4 float64            */
  const void* h;         /* N x N complex          */
  const void* rho_hist;  /* T x N x N complex      */
  void* I_out;           /* N x N complex (out)    */
} sb2_system;

/* sb2_collision_batched -- sb2_collision for nsys <= 64 independent systems
 * of uneven N and T in one enqueue (the descriptor array `sys` is read on the
 * host; every pointer in it is a device pointer).  Systems with less than
 * 10^12 flops of contraction work (48 T N^5) are grouped: those with the same
 * ceil(N/16) form a bucket, the buckets run one after the other, and within a
 * bucket the past times of all systems are processed in common rounds, every
 * contraction stage of a round being one launch over the work items of all
 * the bucket's systems.  Larger systems fill the chip with their own launches
 * and run as in sb2_collision, after the buckets.  Nothing is allocated or synchronised, so the call
 * can be captured in a HIP graph.  Results equal nsys calls of sb2_collision
 * with the same prec up to the order of float32 accumulation.  Errors: as
 * sb2_collision for any system; SB2_EINVAL for nsys < 1 or sys == NULL;
 * SB2_ESHAPE for nsys > 64.                                                  */
int sb2_collision_batched(int nsys, const sb2_system* sys, int prec, void* ws, size_t ws_bytes,
                          void* stream);
size_t sb2_batched_workspace_size(int nsys, const sb2_system* sys, int prec);

/* sb2_rho_step -- one exponential-Euler step of Eq. 8 for rho = -i G^<(t,t):
 *   rho_out = U rho U^dag - dt (I + I^dagger),  U = exp(-i h dt).
 * h, rho, I: N x N complex; rho_out: N x N complex (may alias rho).           */
int sb2_rho_step(int N, const void* h, const void* rho, const void* I, double dt, void* rho_out,
                 void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for op (an sb2_op) at basis size N, history length T
 * (T = number of pairs B for SB2_OP_SIGMA, ignored for SB2_OP_RHO_STEP) and
 * precision prec.  Returns 0 for invalid arguments.  The sizes do not depend
 * on tuned launch parameters.                                               */
size_t sb2_workspace_size(int op, int N, int T, int prec);

/* Static description of a status code. */
const char* sb2_status_string(int status);

/* sb2_autotune -- choose launch parameters for basis size N and precision
 * prec by timing sb2_collision on the first chunk of past times of the given
 * workload (v, h, rho_hist, dt as for sb2_collision; the chunk is the number
 * of past times one pass of the contraction chain holds).  ws must hold
 * sb2_workspace_size(SB2_OP_AUTOTUNE, N, T, prec) bytes; its contents are
 * scratch.  Searched, one after the other: the number of workgroups of the
 * single-slab contraction launches (256 .. 3072; default 3072 for
 * SB2_SPLIT_FP16, 768 otherwise), the split-K
 * factor of the last contraction (50 .. 200 % of the default count) and, for
 * SB2_SPLIT_FP16 with N <= 112, the number of workgroups of the fused second
 * and third contraction (256 .. 2048, default 512).  The winner goes into a
 * process-wide table (not thread-safe) consulted by every later call with
 * this (N, prec), and to *persist_out / *r4pct_out / *fused_out when
 * non-NULL.  Synchronises the stream: not for use under stream capture.  The
 * workspace sizes of the other operations do not depend on tuned values.
 * On error the previous entry for (N, prec) is restored.                    */
int sb2_autotune(int N, int T, const double* v, const void* h, const void* rho_hist, double dt, int prec,
                 void* ws, size_t ws_bytes, void* stream, int* persist_out, int* r4pct_out, int* fused_out);

/* sb2_set_tuning -- install launch parameters for (N, prec), e.g. values an
 * earlier sb2_autotune returned: persist >= 1, 10 <= r4pct <= 200,
 * fused_wgs >= 0 (0 runs the second and third contraction as two separate
 * launches, which is also what every case other than SB2_SPLIT_FP16 with
 * N <= 112 does); otherwise SB2_EINVAL.  Results do not depend on these values
 * beyond the order of float32 accumulation.                                  */
int sb2_set_tuning(int N, int prec, int persist, int r4pct, int fused_wgs);

/* Stage timing for measurement (not for use under stream capture).
 * sb2_profile_enable(1) makes later calls bracket each stage launch with HIP
 * events recorded on the caller's stream; sb2_profile_read waits for those
 * events and returns, per slot, the summed milliseconds and the number of
 * launches since the last read or enable, then clears them.  Slots: 0..3 the
 * four contractions R1..R4 of the self-energy chain, 4 the interaction
 * layout, 5 propagators and GKBA functions, 6 operand packing and the split-K
 * reduction, 7 the collision terms and the sum over past times.  The event
 * objects are created lazily by the library and reused.                     */
int sb2_profile_enable(int on);
int sb2_profile_read(double* ms, int* launches, int nslots);

/* Library version string. */
const char* sb2_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SB2_H */
