/*
 * cpmdp.h -- C ABI of the MI355X (gfx950) CP-structured Bellman backup.
 *
 * Problem (Kuinchtner, Sales & Meneguzzi, CP-MDP, Sec. 2.1 and Sec. 3):
 *   an MDP <S, A, P, R, gamma> over an n-dimensional grid whose state space
 *   is the Cartesian product of the per-dimension state sets (Def. 1), listed
 *   with the LAST dimension varying fastest (Def. 2): for sizes m_0..m_{n-1}
 *   the state with coordinates (i_0..i_{n-1}) has flat index
 *   s = sum_k i_k * prod_{j>k} m_j.
 *
 *   Each action's transition model is held in CP (sum of rank-one terms,
 *   Sec. 2.2) / Kronecker form and never expanded:
 *       P_a = sum_{r < R_a} lambda_{a,r} kron_k T^{(k)}_{a,r},
 *   with T^{(k)}_{a,r} an m_k x m_k row-stochastic matrix,
 *   T[i][j] = P(next coordinate j | current coordinate i) along dim k.
 *
 *   Backup (Eq. 1), with a per-state reward outside the max and a terminal
 *   mask tau (terminal states end the interaction, Sec. 3.2):
 *       Q_a(s) = R(s) + gamma * (1 - tau(s)) * (P_a V)(s)
 *       V'(s)  = max_a Q_a(s)
 *   Value iteration repeats the backup; policy iteration alternates
 *   evaluation of a fixed policy with greedy improvement and stops when the
 *   policy no longer changes (Sec. 2.1).
 *
 * Tie rule for reported policies: the lowest action index whose Q is within
 *   tol = 1e-12 * max(1, ||V||_inf) of the maximum; policy improvement keeps
 *   the incumbent action unless another beats it by more than tol.
 *
 * Conventions
 *   - Every call returns a status code (cpmdp_status); no C++ exception
 *     crosses this boundary.  The message of the last failure is available
 *     from cpmdp_last_error().
 *   - Host arrays passed in are copied; the library never keeps a caller's
 *     host pointer.
 *   - Device buffers (V, pi, workspace) are owned by the caller (allocated
 *     e.g. as torch tensors) and are never freed by the library.
 *   - All device work is enqueued on the stream given to cpmdp_bind (a
 *     hipStream_t passed as void*).  Calls that return host scalars
 *     synchronize that stream before returning.
 *   - A handle is not thread-safe: use it from one host thread, with one
 *     stream at a time.
 */
#ifndef CPMDP_H
#define CPMDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpmdp cpmdp_t;
typedef struct cpmdp_batch cpmdp_batch_t;

typedef enum cpmdp_status {
  CPMDP_OK = 0,
  CPMDP_NOT_CONVERGED = 1,     /* warning: max_iter reached, outputs valid */
  CPMDP_POLICY_UNSETTLED = 2,  /* warning (policy iteration): V certified, but
                                  the last improvements still swapped actions
                                  whose Q-values differ by less than the
                                  evaluation error; outputs valid          */
  CPMDP_E_ARG = -1,            /* bad argument (null, size, range)          */
  CPMDP_E_NOT_STOCHASTIC = -2, /* factor row or lambda sum != 1 (1e-12)     */
  CPMDP_E_DEVICE = -3,         /* a HIP runtime call failed                 */
  CPMDP_E_WORKSPACE = -4,      /* workspace missing or too small            */
  CPMDP_E_NONFINITE = -5,      /* NaN / Inf in inputs or produced values    */
  CPMDP_E_UNSUPPORTED = -6,    /* valid request this build does not do      */
  CPMDP_E_STATE = -7           /* call out of order (e.g. not bound)        */
} cpmdp_status;

typedef enum cpmdp_precision {
  CPMDP_FP64 = 0, /* mode products in FP64                                     */
  CPMDP_FP32 = 1, /* mode products in FP32 (FP64 master, residual, certificate
                     in the solvers)                                           */
  CPMDP_BF16 = 2  /* dense modes with m_k <= 16: mode products on the matrix
                     cores with BF16 operands (each value split into hi + lo
                     BF16 parts, products hi*hi + hi*lo + lo*hi) and FP32
                     accumulation, on V - c (c = midrange of V; exact since
                     P_a 1 = 1); other modes run as FP32                       */
} cpmdp_precision;

typedef enum cpmdp_path {
  CPMDP_PATH_STENCIL = 0, /* every rank term has at most one non-identity
                             factor and it is a clamped +-1 shift           */
  CPMDP_PATH_DENSE = 1,   /* general factors: mode-product chains           */
  CPMDP_PATH_LISTS = 2,   /* successor lists of Def. 3 (cpmdp_create_lists) */
  CPMDP_PATH_TT = 3       /* Tensor-Train cores (cpmdp_create_tt, and Tucker
                             models rewritten as Tensor-Trains by
                             cpmdp_create_tucker)                            */
} cpmdp_path;

/*
 * cpmdp_create -- validate and copy one MDP (Sec. 2.1 tuple; Def. 1-2 sizes).
 *   n_dims   : number of dimensions n, 1 <= n <= 8.
 *   sizes    : [n_dims] states per dimension m_k >= 1 (Def. 1); the product
 *              S must be < 2^31.
 *   n_actions: A, 1 <= A <= 255.
 *   ranks    : [A] rank R_a >= 1 of each action's CP form.
 *   factors  : FP64, for each term t = 0 .. sum_a R_a - 1 (all terms of
 *              action 0 first, then action 1, ...), for each dim k, the
 *              m_k x m_k matrix T^{(k)}_t row-major (row i = current
 *              coordinate, column j = next coordinate).  Entries must be
 *              finite and >= 0, every row must sum to 1 within 1e-12.
 *   lambdas  : FP64 [sum_a R_a], >= 0, summing to 1 within 1e-12 per action.
 *   rewards  : FP64 [S] per-state reward R(s) of Eq. 1, row-major (Def. 2).
 *   gamma    : discount, 0 <= gamma < 1 (the contraction needs gamma < 1).
 * Returns CPMDP_OK and *out, or an error (CPMDP_E_ARG, CPMDP_E_NONFINITE,
 * CPMDP_E_NOT_STOCHASTIC) with *out = NULL.  Nothing is sent to the device.
 */
int cpmdp_create(cpmdp_t** out, int32_t n_dims, const int64_t* sizes,
                 int32_t n_actions, const int32_t* ranks,
                 const double* factors, const double* lambdas,
                 const double* rewards, double gamma);

/*
 * cpmdp_create_lists -- an MDP given directly by the per-state successor
 * lists of Def. 3 (the components (s, s', P(s'|s,a)) of every state), for
 * transition models with no Kronecker / CP structure.  The backup is Eq. 1
 * over those lists.
 *
 *   n_states  S >= 1 (at most 2^30), states numbered 0..S-1
 *   n_actions A in [1, 255]
 *   row_ptr   [A*S + 1] int64, row r = a*S + s (action-major): the list of
 *             (s, a) is entries row_ptr[r] .. row_ptr[r+1]-1; row_ptr[0] = 0,
 *             non-decreasing
 *   succ      [row_ptr[A*S]] int64 successor states s' in [0, S)
 *   prob      [row_ptr[A*S]] FP64 P(s'|s,a) >= 0; every list sums to 1
 *             within 1e-9 (repeated successors are allowed and add up)
 *   rewards   [S] FP64 R(s);  gamma in [0, 1)
 *
 * Host arrays, read during the call (the library keeps its own copy, laid
 * out for the device: 64-state slices, one per wave, each action's entries
 * padded to the slice's longest list).  Terminal states are set with
 * cpmdp_set_terminal; obstacles are not taken (the lists express blocked
 * moves themselves).  Solvers run in FP64 or FP32 (BF16 returns
 * CPMDP_E_UNSUPPORTED); batched solves do not take such handles.
 * Returns CPMDP_OK and *out, or CPMDP_E_ARG (sizes, pointers, ranges),
 * CPMDP_E_NONFINITE, CPMDP_E_NOT_STOCHASTIC (negative probability, list sum)
 * or CPMDP_E_UNSUPPORTED (more than 2^31 padded entries), with *out = NULL.
 */
int cpmdp_create_lists(cpmdp_t** out, int64_t n_states, int32_t n_actions,
                       const int64_t* row_ptr, const int64_t* succ, const double* prob,
                       const double* rewards, double gamma);

/*
 * cpmdp_create_tt -- an MDP whose transition operators are Tensor-Trains
 * (matrix-product operators) over the dimensions, the first of the two
 * decompositions that Sec. 5 proposes beyond the CP form of Sec. 2.2.
 * Action a has cores G_k (k = 0..n-1) of shape [b_k][m_k][m_k][b_{k+1}]
 * with b_0 = b_n = 1, and
 *     P_a[s, s'] = G_0[:, s_0, s'_0, :] G_1[:, s_1, s'_1, :] ... G_{n-1}[:, s_{n-1}, s'_{n-1}, :]
 * (a product of b_k x b_{k+1} matrices; states in the order of Def. 2).  A
 * CP term with rank R is the special case of diagonal cores with bond R.
 * The backup is Eq. 1 with these operators (terminal masks as for
 * cpmdp_create).
 *
 *   n_dims, sizes, n_actions : as cpmdp_create, and every m_k <= 16
 *   bonds  : int32 [A][n_dims + 1]; bonds[a][0] = bonds[a][n] = 1, every
 *            bond in [1, 8]
 *   cores  : FP64, action-major, then k = 0..n-1, one block
 *            [b_k][m_k][m_k][b_{k+1}] row-major each (index i = current
 *            coordinate, j = next coordinate); entries finite and >= 0, and
 *            every row of every P_a must sum to 1 within 1e-9 (checked from
 *            the cores at create)
 *   rewards, gamma : as cpmdp_create
 * Returns CPMDP_OK and *out, or CPMDP_E_ARG, CPMDP_E_NONFINITE,
 * CPMDP_E_NOT_STOCHASTIC, or CPMDP_E_UNSUPPORTED (m_k > 16, bond > 8), with
 * *out = NULL.  Sweeps run in FP64 or FP32 (CPMDP_BF16: CPMDP_E_UNSUPPORTED);
 * obstacles and batched solves do not take such handles.  The workspace holds
 * two buffers of max-bond x S and one of A x S FP64 words besides the values.
 */
int cpmdp_create_tt(cpmdp_t** out, int32_t n_dims, const int64_t* sizes,
                    int32_t n_actions, const int32_t* bonds, const double* cores,
                    const double* rewards, double gamma);

/*
 * cpmdp_create_tucker -- an MDP whose transition operators are in Tucker
 * form over the dimensions (the second decomposition Sec. 5 proposes):
 *     P_a = sum_{r_0..r_{n-1}} C_a[r_0, .., r_{n-1}] kron_k U^{(k)}_{a, r_k}
 * with a core C_a of shape R_{a,0} x .. x R_{a,n-1} and R_{a,k} row-stochastic
 * m_k x m_k factors per dimension.  The CP form is the special case of a
 * diagonal core.  The library rewrites each action exactly as a Tensor-Train
 * (path CPMDP_PATH_TT): split at the dim mu that minimises the largest bond,
 * the bonds left of mu carry (r_0..r_{k-1}), those right of it
 * (r_k..r_{n-1}), and core mu contracts C_a.
 *
 *   n_dims, sizes, n_actions : as cpmdp_create_tt (m_k <= 16)
 *   core_ranks : int32 [A][n_dims], each in [1, 8]; the rewritten bonds must
 *                stay <= 8 (else CPMDP_E_UNSUPPORTED)
 *   cores      : FP64, action-major, C_a row-major (prod_k R_{a,k} entries),
 *                >= 0, summing to 1 per action
 *   factors    : FP64, action-major, then k, then r < R_{a,k}: one m_k x m_k
 *                row-major block U^{(k)}_{a,r} each, rows summing to 1
 *   rewards, gamma : as cpmdp_create
 * (the sum conditions are checked on the rewritten operator, every row
 * within 1e-9).  Returns as cpmdp_create_tt.
 */
int cpmdp_create_tucker(cpmdp_t** out, int32_t n_dims, const int64_t* sizes,
                        int32_t n_actions, const int32_t* core_ranks,
                        const double* cores, const double* factors,
                        const double* rewards, double gamma);

/*
 * cpmdp_cp_fit -- fit rank-R CP factors to one action's tabular transition
 * matrix (the decomposition step behind the CP form of Sec. 2.2 / Sec. 3,
 * whose method the paper leaves open): alternating least squares (Kolda &
 * Bader, SIAM Review 51(3), 2009, Sec. 3.4) on the n-way tensor
 *     X[u_0, .., u_{n-1}] = P(s' | s),   u_k = i_k m_k + j_k
 * (s = (i_0..i_{n-1}), s' = (j_0..j_{n-1}) in the order of Def. 2).  One
 * iteration updates k = 0..n-1 in turn: A^(k) = M V^+, with M the sparse
 * matricised tensor times the Khatri-Rao product of the other factors
 * (computed on the device over the entries) and V the Hadamard product of
 * their Gram matrices (R x R, on the host), then scales each column of
 * A^(k) to unit 2-norm; the norms of the last update are the weights.  The
 * result is the unconstrained least-squares model (factors may be negative
 * and rows need not sum to 1).
 *
 *   n_dims, sizes : the grid (Def. 1), 1 <= n <= 8, S < 2^31; every
 *                   m_k^2 * rank <= 8192 (else CPMDP_E_UNSUPPORTED)
 *   nnz, rows, cols, vals : DEVICE arrays of the nnz COO entries (s, s',
 *                   P(s'|s)), int32 / int32 / FP64, each 16-byte aligned,
 *                   distinct and sorted by (s, s') (row-major); coordinates
 *                   outside [0, S) or entries out of order give CPMDP_E_ARG
 *   rank          : R in [1, 32]
 *   max_iter, tol : stop after max_iter iterations, or when the relative error
 *                   ||X - X_hat|| / ||X|| changes by <= tol between iterations
 *   factors       : HOST FP64 [R * sum_k m_k^2], in: the starting factors,
 *                   out: the fitted ones, in the term layout of cpmdp_create
 *                   (term r, dim k, one m_k x m_k block row-major = u_k)
 *   lambdas       : HOST FP64 [R] out: the weights
 *   errors        : HOST FP64 [max_iter] out (may be NULL): the relative error
 *                   after every iteration
 *   iters_out     : iterations run (may be NULL)
 *   mttkrp_ms     : out (may be NULL): mean device time of one mode's
 *                   Khatri-Rao product (its kernel and partial-sum reduction)
 *   workspace, ws_bytes : device, 256-byte aligned, at least
 *                   cpmdp_cp_fit_workspace_bytes
 *   stream        : the HIP stream for every device step
 * Returns CPMDP_OK, or CPMDP_E_ARG, CPMDP_E_UNSUPPORTED, CPMDP_E_WORKSPACE,
 * CPMDP_E_NONFINITE (start factors, entries or the fit), CPMDP_E_DEVICE.
 * The call synchronises the stream once per mode update.
 */
int cpmdp_cp_fit_workspace_bytes(int32_t n_dims, const int64_t* sizes,
                                 int64_t nnz, int32_t rank, size_t* bytes);
int cpmdp_cp_fit(int32_t n_dims, const int64_t* sizes, int64_t nnz,
                 const int32_t* rows, const int32_t* cols, const double* vals,
                 int32_t rank, int32_t max_iter, double tol, double* factors,
                 double* lambdas, double* errors, int32_t* iters_out,
                 double* mttkrp_ms, void* workspace, size_t ws_bytes,
                 void* stream);

/* Terminal states (Sec. 3.2): mask [S], nonzero = terminal (V(s) = R(s), no
 * continuation).  Must be called before cpmdp_bind; default: none. */
int cpmdp_set_terminal(cpmdp_t* h, const uint8_t* mask);

/* Obstacles (Sec. 3.2: states the agent has no access to): mask [S], host
 * memory read during the call, nonzero = obstacle.  The paper does not say
 * what a move towards an obstacle does; here it is blocked and the agent
 * stays where it is, as at the grid edge, and an obstacle state is outside
 * the problem: its reward is taken as 0 and it has no continuation, so its
 * value is 0 and its reported action 0.  Supported for shift/identity
 * factors (path CPMDP_PATH_STENCIL): with dense factors the blocked moves
 * are no sparse correction of the Kronecker form, and a mask with any
 * obstacle returns CPMDP_E_UNSUPPORTED.  A state may not be both terminal
 * and an obstacle (cpmdp_bind returns CPMDP_E_ARG).  Must be called before
 * cpmdp_workspace_bytes and cpmdp_bind (obstacles add 2 bytes per state to
 * the workspace); CPMDP_E_STATE after bind.  An all-zero mask removes the
 * obstacles.  Batched solves do not take instances with obstacles. */
int cpmdp_set_obstacles(cpmdp_t* h, const uint8_t* mask);

/* Which kernel family the instance runs on (cpmdp_path), via *path. */
int cpmdp_get_path(const cpmdp_t* h, int32_t* path);

/* Device workspace size in bytes that cpmdp_bind needs for this instance
 * (all precisions). */
int cpmdp_workspace_bytes(const cpmdp_t* h, size_t* bytes);

/*
 * cpmdp_bind -- attach a caller-owned device workspace (>= workspace_bytes,
 * 256-byte aligned) and a stream, and upload the packed model to it (the only
 * bulk host-to-device copy).  May be called again to move to another
 * workspace or stream; the workspace must stay allocated while the handle
 * is used.
 */
int cpmdp_bind(cpmdp_t* h, void* dev_workspace, size_t bytes,
               void* hip_stream);

/* Switch the stream used by later calls (workspace unchanged). */
int cpmdp_set_stream(cpmdp_t* h, void* hip_stream);

/*
 * cpmdp_set_option -- execution options; results are the same with either
 * setting (each state's arithmetic is unchanged).
 *   CPMDP_OPT_MARCH (value 0 or 1, default 1): on the shift/identity path,
 *     walk large grids plane by plane along dimension 0 with the dim-0
 *     neighbours kept in registers (used when n >= 2, m_{n-1} % 4 == 0, at
 *     least 8 planes of at least 65,536 states); 0 forces the one-pass form.
 * Returns CPMDP_E_ARG for an unknown option or value.
 */
enum { CPMDP_OPT_MARCH = 1 };
int cpmdp_set_option(cpmdp_t* h, int option, int64_t value);

/*
 * cpmdp_backup -- one Bellman backup (Eq. 1) on the device.
 *   V_in, V_out : device [S]; FP64 for CPMDP_FP64, FP32 otherwise.  Must not
 *                 alias.
 *   pi_out      : device int32 [S] greedy actions (tie rule above, applied
 *                 in the backup's precision) or NULL.
 *   residual_host: if non-NULL, the stream is synchronized and
 *                 ||V_out - V_in||_inf is written there (as FP64).
 *   precision   : cpmdp_precision.
 */
int cpmdp_backup(cpmdp_t* h, const void* V_in, void* V_out, int32_t* pi_out,
                 double* residual_host, int precision);

/*
 * cpmdp_policy_backup -- one fixed-policy backup (policy evaluation step of
 * Sec. 2.1): V_out(s) = R(s) + gamma (1 - tau(s)) (P_{pi(s)} V_in)(s).
 *   pi : device int32 [S], each in [0, A).  Other arguments as cpmdp_backup.
 */
int cpmdp_policy_backup(cpmdp_t* h, const void* V_in, void* V_out,
                        const int32_t* pi, double* residual_host,
                        int precision);

/*
 * cpmdp_value_iteration -- repeat the backup until the Bellman residual
 * ||B V - V||_inf <= eps (Sec. 2.1), then certify in FP64.
 *   V_dev     : device FP64 [S]; in: V0 (warm start), out: the solution.
 *   pi_out    : device int32 [S] greedy policy of the returned V, or NULL.
 *   eps       : absolute residual target (> 0).
 *   max_iter  : cap on backup sweeps (>= 1).
 *   precision : sweep arithmetic; FP32/BF16 sweeps run until they reach their
 *               rounding floor (8 ulp of rmax / (1 - gamma); on instances
 *               with S * A >= 2^24 then 12 ulp of ||V|| + r / (1 - gamma)
 *               measured on the iterate) or eps / 2, then FP64 sweeps
 *               continue until the FP64 residual meets eps (when the FP32
 *               residual already lies 4 ulp below eps the FP64 certificate
 *               is tried first); on the dense path,
 *               whose FP64 chain runs on the vector ALUs, the tail instead
 *               refines the greedy policy's evaluation: FP64 residual, low-
 *               precision correction sweeps, V += e, FP64 certificate.
 *   sweeps_out, residual_out : nullable; sweeps run, and the FP64 residual
 *               ||B V - V||_inf of the returned V.
 * Returns CPMDP_OK, or CPMDP_NOT_CONVERGED (outputs valid, best iterate),
 * or an error.
 */
int cpmdp_value_iteration(cpmdp_t* h, double* V_dev, int32_t* pi_out,
                          double eps, int64_t max_iter, int precision,
                          int64_t* sweeps_out, double* residual_out);

/*
 * cpmdp_policy_iteration -- policy iteration (Sec. 2.1): evaluate pi, improve
 * greedily keeping the incumbent on ties, stop when pi is unchanged and the
 * FP64 residual ||B V - V||_inf <= eps.  Evaluation runs as FP64 residual
 * r = R + gamma P_pi V - V, correction sweeps e <- r + gamma P_pi e in the
 * requested precision, and V += e in FP64.
 *   V_dev  : device FP64 [S]; in: initial V (any), out: the solution.
 *   pi_dev : device int32 [S]; in: initial policy, out: the final policy.
 *   max_iter: cap on the total number of sweeps of any kind.
 *   outer_iters_out, sweeps_out, residual_out: nullable statistics.
 * Returns CPMDP_OK when an improvement left pi unchanged and V is certified;
 * CPMDP_POLICY_UNSETTLED when V was certified in three improvement rounds in
 * a row but each still changed the policy (the evaluation is iterative, so
 * actions whose Q-values differ by less than its error can keep swapping):
 * V is certified and every returned action is within the tie tolerance of
 * the best Q of the returned V; CPMDP_NOT_CONVERGED at max_iter; or an error.
 */
int cpmdp_policy_iteration(cpmdp_t* h, double* V_dev, int32_t* pi_dev,
                           double eps, int64_t max_iter, int precision,
                           int64_t* outer_iters_out, int64_t* sweeps_out,
                           double* residual_out);

/*
 * cpmdp_bound_shift -- one FP64 backup of V followed by the constant shift of
 * McQueen's error bounds (McQueen 1966, "A modified dynamic programming method
 * for Markovian decision problems"): with r = BV - V over the non-terminal
 * states, V* lies within BV + gamma/(1-gamma) [min r, max r] when every
 * factor row sums to 1; V is replaced by BV + gamma/(1-gamma) (min r + max r)/2
 * on non-terminal states and by BV = R on terminal ones.  Used to start value
 * iteration from a predicted V0 without its global offset.
 *   V      : device FP64 [S], in/out.
 *   lo_out, hi_out: nullable; gamma/(1-gamma) min r and gamma/(1-gamma) max r.
 */
int cpmdp_bound_shift(cpmdp_t* h, double* V, double* lo_out, double* hi_out);

/*
 * cpmdp_time_sweeps -- measurement helper: run n backup sweeps ping-ponging
 * between the device buffers V_a and V_b (dtype of the precision, starting
 * from V_a) on the bound stream, each launched with a HIP event pair that
 * records its kernels' own start and stop (hipExtLaunchKernelGGL; from the
 * first kernel of the sweep to the last), and return the mean time of one
 * sweep's kernels in milliseconds.
 *   mode: 0 = Bellman max sweep (Eq. 1), 1 = fixed-policy sweep with pi.
 */
int cpmdp_time_sweeps(cpmdp_t* h, void* V_a, void* V_b, int32_t n, int precision, int mode,
                      const int32_t* pi, double* mean_ms);

/* Release the handle (host memory only; device buffers stay the caller's). */
void cpmdp_destroy(cpmdp_t* h);

/* Message of the last failure on h (h == NULL: of the last failed create or
 * batch call in this thread).  Valid until the next call on h. */
const char* cpmdp_last_error(const cpmdp_t* h);

/* ------------------------------------------------------------ batched ---
 * Many independent instances (each a created handle, stencil path) solved
 * together: every sweep is one persistent launch over a table of tiles of
 * all still-active instances, chunks of sweeps are captured as HIP graphs,
 * and the tile size / sweeps per graph come from a small autotuner.
 */

/* Collect count >= 1 created handles (not necessarily bound) into *out;
 * the handles must outlive the batch, which cpmdp_batch_destroy frees.
 * Every handle must be on the stencil path (shift / identity factors) with
 * at most 4 dimensions and no obstacles, else CPMDP_E_UNSUPPORTED; count < 1
 * or a NULL handle: CPMDP_E_ARG. */
int cpmdp_batch_create(cpmdp_batch_t** out, cpmdp_t* const* handles,
                       int32_t count);
/* Device bytes cpmdp_batch_bind needs: the batch's own copy of every
 * instance (rows padded to a multiple of 4 states; rewards, terminal bits,
 * two FP32 and two FP64 value buffers) plus tile tables and residual slots. */
int cpmdp_batch_workspace_bytes(const cpmdp_batch_t* b, size_t* bytes);
/* Lay the batch out in dev_workspace (caller-owned device memory of at least
 * cpmdp_batch_workspace_bytes, 256-byte aligned, kept until the batch is
 * destroyed or bound again; else CPMDP_E_WORKSPACE) and fill it from the
 * handles' host-side rewards, terminal states and weights (the copies have
 * finished when the call returns).  hip_stream is the caller's stream (NULL:
 * the null stream): every later solve is ordered after the work enqueued on
 * it. */
int cpmdp_batch_bind(cpmdp_batch_t* b, void* dev_workspace, size_t bytes,
                     void* hip_stream);

/*
 * cpmdp_batch_solve -- solve every instance to ||B V - V||_inf <= eps.
 *   V_devs : [count] device FP64 [S_i] buffers; in: V0_i, out: solution.
 *   pi_devs: [count] device int32 [S_i] buffers (policy out; for PI also in)
 *            or NULL.
 *   eps    : > 0, the FP64 certificate each instance must meet.
 *   max_iter: >= 1, cap on each instance's sweeps of any kind.
 *   precision: CPMDP_FP64: FP64 sweeps only; CPMDP_FP32 (or CPMDP_BF16,
 *            which this stencil path runs as FP32): FP32 sweeps until they
 *            stop contracting, then FP64 sweeps; the certificate is FP64.
 *            Policy iteration runs FP32 correction sweeps: with CPMDP_FP64
 *            it returns CPMDP_E_UNSUPPORTED.
 *   method : 0 = value iteration, 1 = policy iteration.
 *   sweeps_out   : [count] int64 sweeps per instance (the certificate's
 *                  included), or NULL.
 *   residual_out : [count] FP64 certificate per instance, or NULL.
 * The work is ordered after everything enqueued on the bound stream so far
 * and has finished when the call returns.  Returns CPMDP_OK,
 * CPMDP_NOT_CONVERGED if any instance hit max_iter, else
 * CPMDP_POLICY_UNSETTLED if policy iteration stopped so on any instance (as
 * in cpmdp_policy_iteration), or an error.
 */
int cpmdp_batch_solve(cpmdp_batch_t* b, double* const* V_devs,
                      int32_t* const* pi_devs, double eps, int64_t max_iter,
                      int precision, int method, int64_t* sweeps_out,
                      double* residual_out);

/* Autotuner control: tune = 1 times candidate tile sizes, grid sizes, tile
 * forms (marching tiles where an instance allows them, or one-pass tiles
 * only) and tile schedules (a contiguous range of tiles per block, or a range
 * per XCD taken in turn by its blocks) on the bound batch, keeps the fastest
 * and sizes the sweeps per graph from the host round trip; cache_path
 * (nullable) is a text file of size class -> choice read before and written
 * after tuning. */
int cpmdp_batch_autotune(cpmdp_batch_t* b, int tune, const char* cache_path);
/* The current choice: states per one-pass tile and sweeps per graph. */
int cpmdp_batch_config(const cpmdp_batch_t* b, int32_t* tile_states,
                       int32_t* sweeps_per_graph);
/* Set the choice by hand (tests, measurements): states per one-pass tile (a
 * multiple of 1024 in [1024, 65536]), blocks per launch (a multiple of 8 in
 * [8, 2048]), marching tiles (1) or one-pass tiles only (0), tile schedule
 * (0: range per block, 1: range per XCD, interleaved); other values:
 * CPMDP_E_ARG.  Results do not depend on the choice. */
int cpmdp_batch_set_schedule(cpmdp_batch_t* b, int32_t tile_states, int32_t grid, int32_t march,
                             int32_t sched);
/* The current choice: blocks per launch, marching tiles on (1) / off (0),
 * tile schedule (0: range per block, 1: range per XCD, interleaved). */
int cpmdp_batch_schedule(const cpmdp_batch_t* b, int32_t* grid, int32_t* march,
                         int32_t* sched);
/* Measurement helper: n FP32 value-iteration sweeps over the whole bound
 * batch (every instance active, values in the internal FP32 buffers, so the
 * results are meaningless), each launched with events that record the sweep
 * kernel's own start and stop; *mean_ms = mean kernel time of one sweep.
 * A later cpmdp_batch_solve starts from the caller's V as usual. */
int cpmdp_batch_time_sweeps(cpmdp_batch_t* b, int32_t n, double* mean_ms);
/* Free the batch, its private streams, graphs and pinned staging buffers
 * (not the handles, nor the caller's workspace); NULL is a no-op. */
void cpmdp_batch_destroy(cpmdp_batch_t* b);

/* ------------------------------------------------------- learned warm start
 * A 130 -> 256 -> 256 -> 1 ReLU MLP for 3-D GridWorlds (m^3 states) whose
 * output y predicts (1 - gamma) V(s) = 0.2 + 0.05 y from per-state features;
 * V0 = (0.2 + 0.05 y) / (1 - gamma) starts value iteration, whose FP64
 * certificate is unchanged (plain VI from V0 = 0 stays the fallback).  All
 * buffers are device buffers owned by the caller; work goes to `stream`.
 *
 * Parameters (FP32, 99,585): W1 [130][256] (input-major), b1 [256],
 * W2 [256][256], b2 [256], w3 [256], b3 [1], in that order.
 * Features of state s = (i0, i1, i2) (last index fastest, Def. 2):
 *   [0..2]   i_k / (m - 1)
 *   [3..127] 10 * R(clamp(i + d)), d in {-2..2}^3, d_0 slowest, each
 *            coordinate clamped to [0, m - 1]
 *   [128]    (gamma - 0.945) / 0.026
 *   [129]    (slip - 0.175) / 0.072
 * Random numbers: SplitMix64 (Steele, Lea & Flood 2014); normals by
 * Box-Muller.  Loss: mean squared error of y against
 * ((1 - gamma) V* - 0.2) / 0.05.
 */
int cpmdp_mlp_param_count(int64_t* count);
/* Workspace bytes for `batch` rows (train step, loss_grad, forward) or for
 * a predict chunk of that many states. */
int cpmdp_mlp_workspace_bytes(int32_t batch, size_t* bytes);
/* He-normal hidden weights from `seed`; zero biases and output layer. */
int cpmdp_mlp_init(float* params, uint64_t seed, void* stream);
/* X [count][130] for states s0 .. s0+count-1 of an m^3 grid with rewards R
 * [m^3] (FP32).  m^3 >= 2^31 or a range past m^3: CPMDP_E_ARG. */
int cpmdp_mlp_features(const float* R, int32_t m, double gamma, double slip, int32_t s0,
                       int32_t count, float* X, void* stream);
/* y [count] = MLP(X).  precision: CPMDP_FP32 (every product in FP32) or
 * CPMDP_BF16 (the two hidden-layer products take BF16 operands, rounded to
 * nearest even, on the matrix cores with FP32 accumulation, bias and ReLU;
 * the output layer stays FP32); other values: CPMDP_E_ARG. */
int cpmdp_mlp_forward(const float* params, const float* X, int32_t count, float* y,
                      int32_t precision, void* ws, size_t ws_bytes, void* stream);
/* Gradient of mean((MLP(X) - t)^2) into grad [99,585]; loss_out (nullable,
 * synchronizes the stream). */
int cpmdp_mlp_loss_grad(const float* params, const float* X, const float* t, int32_t count,
                        float* grad, double* loss_out, void* ws, size_t ws_bytes, void* stream);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) at step >= 1. */
int cpmdp_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t step, double lr,
                   void* stream);
/* One training step on `batch` samples drawn from n_inst solved instances:
 * R_ptrs / Vstar_ptrs are DEVICE arrays of n_inst device pointers (FP32
 * rewards, FP64 solutions), gammas / slips device FP64 [n_inst]; sample i
 * of step k is SplitMix64(seed ^ SplitMix64(k * 0x100000001B3 + i)) ->
 * (instance = high 32 bits mod n_inst, state = low 32 bits mod m^3).
 * Then forward, backward and Adam.  loss_out nullable (synchronizes).
 * Every R_ptrs[i] must hold m^3 floats and every Vstar_ptrs[i] m^3 doubles
 * (the kernels index them up to m^3 - 1 and cannot check their extent);
 * m^3 >= 2^31: CPMDP_E_ARG. */
int cpmdp_mlp_train_step(float* params, float* adam_m, float* adam_v, float* grad, int64_t step,
                         const float* const* R_ptrs, const double* const* Vstar_ptrs,
                         const double* gammas, const double* slips, int32_t n_inst, int32_t m,
                         int32_t batch, uint64_t seed, double lr, void* ws, size_t ws_bytes,
                         void* stream, double* loss_out);
/* V0 [m^3] (FP64) = MLP prediction / (1 - gamma), in chunks of `chunk`
 * states (workspace sized for chunk); precision as in cpmdp_mlp_forward.
 * level = 1: the network runs on n = min(m^3, chunk, 4096) states spread
 * evenly over the grid (state floor(j m^3 / n) for j < n) and every entry of
 * V0 is set to the mean of their predicted values (summed in a fixed order),
 * the instance's predicted value level; level = 0: the per-state
 * predictions.  R must hold m^3 floats and V0 m^3
 * doubles (not checkable here: the caller's extents are unknown to the
 * library); m^3 >= 2^31 or level outside {0, 1}: CPMDP_E_ARG. */
int cpmdp_mlp_predict(const float* params, const float* R, int32_t m, double gamma, double slip,
                      double* V0, int32_t chunk, int32_t precision, int32_t level, void* ws,
                      size_t ws_bytes, void* stream);
/* The value levels of n_inst instances of one grid size in one pass (the
 * level = 1 prediction of cpmdp_mlp_predict, each instance on its
 * n = min(m^3, 4096) spread states, one forward pass over all n_inst * n
 * rows): V0[i] (m^3 doubles) is set to instance i's level.  R and V0 are
 * HOST arrays of n_inst device pointers (m^3 floats / m^3 doubles each; their
 * extents cannot be checked), gammas and slips host arrays of n_inst.  The
 * workspace is sized for n_inst * n rows (cpmdp_mlp_workspace_bytes).
 * Levels agree with per-instance calls to FP32 rounding (the forward pass
 * may group its sums differently for more rows).  n_inst * n > 2^24, a null
 * pointer or gamma >= 1: CPMDP_E_ARG. */
int cpmdp_mlp_predict_levels(const float* params, const float* const* R, const double* gammas,
                             const double* slips, int32_t n_inst, int32_t m, double* const* V0,
                             int32_t precision, void* ws, size_t ws_bytes, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * prediction as cpmdp_mlp_predict, with the workspace in the library's own
 * static device array (30.3 MiB per GPU, the workspace of 4096 rows, held
 * until the process ends) instead of an argument.  No allocation of any
 * kind.  chunk must be in [1, 4096], else CPMDP_E_ARG; other arguments and
 * results as in cpmdp_mlp_predict.  Every call on one GPU uses that GPU's one
 * array: calls that overlap on one GPU (other threads, other streams) race
 * and must be serialized by the caller. */
int cpmdp_mlp_predict_noalloc(const float* params, const float* R, int32_t m, double gamma,
                              double slip, double* V0, int32_t chunk, int32_t precision,
                              int32_t level, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CPMDP_H */
