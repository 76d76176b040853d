/*
 * pmx.h - Kronecker-structured payoff-matrix gradients for poker endgames on
 * AMD Instinct MI355X (gfx950).  C ABI of libpmx.so.
 *
 * What it computes (Farina & Sandholm, "Fast Payoff Matrix Sparsification
 * Techniques for Structured Extensive-Form Games", AAAI 2022):
 *
 *   - Section 2: the payoff matrix A of Player 1 has rows indexed by Player
 *     1's sequences and columns by Player 2's; a terminal z contributes its
 *     payoff times the probability of the chance events leading to it.
 *     First-order solvers need the gradients A y and A^T x every iteration
 *     (Section 2, application 3).
 *   - Section 3 (Prop. 1): for a river endgame with deal distribution pi and
 *     outcome gamma,  A = C (x) F + (L1 W L2) (x) S : every hand pair plays the
 *     same betting skeleton, so A is a sum of Kronecker products of a small
 *     betting factor and a hand-comparison factor.  A turn endgame is
 *     block-diagonal over the river card (Section 3, last paragraph).
 *   - Section 4 (eq. cf and Technique B): the compatibility term is a rank-one
 *     product minus a card-collision correction, and the win/lose term,
 *     with hands sorted by strength, is the inverse of a bidiagonal
 *     difference operator, i.e. a prefix sum.  The library never forms A: it
 *     applies each hand factor as a strength-sorted prefix scan with per-card
 *     inclusion-exclusion corrections.
 *   - Section 5 (first-order methods): a regret-based solver (here regret
 *     matching+, alternating, linear averaging) updates all hands in
 *     parallel; exploitability = half the saddle gap over the initial pot.
 *
 * Conventions shared by every call
 * --------------------------------
 *  * Players are 0 (Player 1, small blind, acts first, maximizes x^T A y) and
 *    1 (Player 2).
 *  * Sequences of each player are numbered in depth-first preorder of the
 *    betting tree: when a decision node is first visited all its actions get
 *    consecutive ids in the order fold, check/call, bets and raises by
 *    ascending size, all-in; children are then visited in action order; a
 *    chance node (turn + river endgames) visits river cards in the order
 *    given.  The empty sequence has no id (parent -1).
 *  * Vectors are sequence-major and hand-contiguous: element (s, h) of player
 *    p's vector is at [s * stride + h], h indexing the player's hand list in
 *    the order it was given.  Entries h >= n_hands of a row are padding: they
 *    are ignored on input and written as 0 on output.
 *  * A game may hold several independent instances (a batch).  Instance i's
 *    vector block of player p starts at element vec_offset (game_layout) and
 *    spans n_seq * stride elements; a batched buffer is the concatenation.
 *  * Device pointers are caller-owned HIP device allocations; host pointers
 *    are plain host memory.  Streams are hipStream_t passed as void*
 *    (NULL = the default stream).  Asynchronous calls only enqueue work.
 *  * Every call returns PMX_OK (0) or a negative PMX_E* code; on error no
 *    out-parameter is written and pmx_last_error() describes the failure.
 *    No C++ exception crosses the ABI.
 */
#ifndef PMX_H
#define PMX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PMX_OK = 0,
  PMX_EINVAL = -1,    /* invalid argument or descriptor                        */
  PMX_ENOMEM = -2,    /* host or device allocation failed                      */
  PMX_EDEVICE = -3,   /* a HIP call failed (message carries hipGetErrorString)  */
  PMX_ESTATE = -4,    /* call not valid in the handle's state (e.g. host-only)  */
  PMX_ENUMERIC = -5   /* NaN/Inf detected in a solver quantity                 */
};

/* Terminal kinds (Section 3: F collects fold payoffs, S showdown stakes). */
enum { PMX_FOLD_P1 = 0, PMX_FOLD_P2 = 1, PMX_SHOWDOWN = 2 };

typedef struct Game Game;   /* opaque; owns host and device state */

/*
 * GameDesc - one endgame instance (Section 3: board B, stacks (s1, s2), pot
 * contribution c, beliefs mu_1, mu_2; betting abstraction of Appendix A).
 * All arrays are read during game_create and copied; the caller keeps them.
 *
 *  deck_size        cards are 0 .. deck_size-1 (deck_size <= 64)
 *  cards_per_hand   1 or 2
 *  n_board, board   public cards already dealt (none may repeat)
 *  n_river, river_cards
 *                   0 for a river endgame.  Otherwise a turn + river endgame:
 *                   after the first betting round one more card is dealt
 *                   uniformly from the cards not on the board and not in
 *                   either hand; river_cards must list exactly the cards not
 *                   on the board.
 *  n_hands[p], hand_cards[p]
 *                   player p's hand list, [n_hands][cards_per_hand] card ids;
 *                   no hand may repeat a card or use a board card.
 *                   1 <= n_hands <= 1280.
 *  strength[p]      [max(1, n_river)][n_hands[p]]: hand strength on each final
 *                   board; higher wins, equal ties.  A hand that appears in
 *                   both lists must have equal strengths.  Entries of hands
 *                   holding that board's river card are ignored.
 *  range[p]         [n_hands[p]] belief weights mu_p >= 0, finite, any scale
 *                   (beta normalizes); sum over compatible pairs must be > 0.
 *  contrib          each player's pot contribution before the endgame (> 0)
 *  stack[p]         chips behind (>= 0)
 *  n_bet_fracs, bet_fracs
 *                   bet / raise sizes: match the opponent, then add fraction
 *                   x the pot after matching (Fig. 1 caption); each > 0.
 *  max_raises       raises allowed after the opening bet of a round (>= 0)
 *  allow_allin      nonzero: offer all-in (also past the raise cap)
 *  bet_menu_len, bet_menu
 *                   optional asymmetric betting abstraction (the paper's
 *                   appendix on the betting abstraction): NULL, or
 *                   bet_menu_len[5 p + k] fractions of player p in situation
 *                   k (0 opening the round, 1 answering a check, 2 facing a
 *                   bet, 3 facing one raise, 4 facing two or more raises),
 *                   read in that order from bet_menu, each > 0 and at most 64
 *                   per list; they replace bet_fracs.  A zeroed descriptor
 *                   tail (both NULL) keeps bet_fracs everywhere.
 */
typedef struct {
  int32_t deck_size, cards_per_hand;
  int32_t n_board;
  const uint8_t* board;
  int32_t n_river;
  const uint8_t* river_cards;
  int32_t n_hands[2];
  const uint8_t* hand_cards[2];
  const int32_t* strength[2];
  const double* range[2];
  double contrib;
  double stack[2];
  int32_t n_bet_fracs;
  const double* bet_fracs;
  int32_t max_raises;
  int32_t allow_allin;
  const int32_t* bet_menu_len;
  const double* bet_menu;
} GameDesc;

/*
 * Layout - shape of one instance for one player.  The pointed-to arrays are
 * owned by the Game and stay valid until game_destroy.
 *   infoset_parent[i]  parent sequence id of infoset i (-1 = empty sequence)
 *   infoset_first[i]   first action's sequence id (actions are consecutive)
 *   infoset_nact[i]    number of actions
 *   infoset_board[i]   -1 first betting round, r >= 0 river card index
 */
typedef struct {
  int32_t n_seq;
  int32_t n_hands;
  int32_t stride;          /* row stride of vectors (>= n_hands, multiple of 4) */
  int64_t vec_offset;      /* element offset of this instance's block           */
  int64_t vec_elems;       /* total elements of the batched buffer (all instances) */
  int32_t n_infosets;
  const int32_t* infoset_parent;
  const int32_t* infoset_first;
  const int32_t* infoset_nact;
  const int32_t* infoset_board;
} Layout;

/*
 * Terminals of one instance (Section 2 / 3: the leaves of the skeleton).
 * seq[0], seq[1]: last sequence of each player; kind: PMX_FOLD_P1 / _P2 /
 * PMX_SHOWDOWN; c1, c2: pot contributions; board: -1 first round, else river
 * card index; runout: showdown reached all-in before the river card.
 */
typedef struct {
  int32_t n_terminals;
  const int32_t* seq1;
  const int32_t* seq2;
  const int32_t* kind;
  const int32_t* board;
  const int32_t* runout;
  const double* c1;
  const double* c2;
} Terminals;

/*
 * HandMeta - integer hand metadata of one (instance, board context, player)
 * used by the hand operators; exported so tests can check it bit-exactly.
 * Board context 0 is the first-round board; context 1 + r is river card r
 * (turn + river endgames only).  Hands are ordered by (strength, index).
 *   rank[h]     position of hand h in that order among live hands, -1 dead
 *   n_live      live hands
 *   lt[h], le[h]  number of live opponent hands strictly weaker / not
 *               stronger than h (-1 if h is dead)
 *   self_[h]    rank of the opponent's hand with the same cards (-1 none)
 *   beta        sum of mu1 mu2 over compatible pairs (same for all contexts)
 */
typedef struct {
  int32_t n_hands;
  int32_t n_live;
  const int32_t* rank;
  const int32_t* lt;
  const int32_t* le;
  const int32_t* self_;
  double beta;
} HandMeta;

/* ---- lifetime ------------------------------------------------------------ */

/* Validate and build one instance (host) and upload it to the current HIP
 * device.  Synchronous.  PMX_EINVAL names the offending field. */
int game_create(const GameDesc* desc, Game** out);

/* Build n instances as one batched game (Section 5's solver applied to many
 * endgames at once); each instance keeps its own vectors (game_layout). */
int game_create_batch(const GameDesc* descs, int32_t n, Game** out);

/* Host-only build: layout, terminals and hand metadata are available, but no
 * device memory is touched; device calls return PMX_ESTATE.  Usable on
 * machines without a GPU. */
int game_create_host(const GameDesc* descs, int32_t n, Game** out);

/* Free host and device state.  NULL is accepted.  Synchronizes the device. */
void game_destroy(Game* g);

int game_num_instances(const Game* g, int32_t* n);
int game_layout(const Game* g, int32_t instance, int32_t player, Layout* out);
int game_terminals(const Game* g, int32_t instance, Terminals* out);
int game_hand_meta(const Game* g, int32_t instance, int32_t ctx, int32_t player, HandMeta* out);

/* Matvec schedule of the FP32 products (results agree to the FP32 rounding
 * of the data): kernels 2 and 3 = one workgroup of 256 / 512 threads per
 * chunk of output rows on the chunk-aligned scan layout, launched per
 * hands-per-thread class (prefix sums accumulated in FP64 and stored once
 * rounded to FP32); kernel 4 (the default) = one workgroup per chunk of
 * groups, a group scanning up to four input rows of one board context at
 * once (Technique B's solve and the inclusion-exclusion of eq. cf applied to
 * all of them).  rows_per_chunk in [1, 64]: output rows per chunk (2, 3) or
 * groups per chunk (4).  The FP64 products always run the chunk-aligned
 * layout.  Synchronizes the device; drops the captured solver graph.  The
 * defaults depend on the game's size; an autotuner may override them.
 * PMX_EINVAL for a kernel outside [2, 4]. */
int game_tune(Game* g, int32_t kernel, int32_t rows_per_chunk);
int game_get_tuning(const Game* g, int32_t* kernel, int32_t* rows_per_chunk);

/* Regret-update schedule: each player's treeplex is cut into pieces of at
 * most `rows` sequences (default and maximum 64) and 64 infosets whose rows
 * stay in LDS for 64 hands at a time; pieces hanging below other pieces
 * exchange root values and parent weights through a stage buffer.  Results
 * do not depend on the cut (same arithmetic per infoset).  PMX_EINVAL if rows
 * is outside [1, 64] or below the largest action count of an infoset (the
 * previous cut stays).
 * Synchronizes the device; drops the captured solver graph. */
int solver_set_task_rows(Game* g, int32_t rows);

/* Regret-update kernel choice: a launch of at most `max_records` block
 * records (64 hands of one piece each) runs with four lanes per hand and 16
 * hands per workgroup (its walk is latency-bound: few workgroups), a larger
 * one with one lane per hand (it is bound by HBM bytes).  Default 256; 0
 * selects the one-lane form everywhere, INT32_MAX the four-lane form.  Both
 * compute the same update (sums over an infoset's actions in another
 * order).  PMX_EINVAL if max_records < 0.  Synchronizes the device; drops the
 * captured solver graph. */
int solver_set_rm_quad(Game* g, int32_t max_records);

/* ---- gradients (Section 2 app. 3; Prop. 1; eq. cf; Technique B) ----------- */

/* out = A y (Player 1's gradient).  y: player 1's vectors (all instances),
 * out: player 0's.  FP32 in and out; hand scans accumulate in FP64.  Both
 * device pointers, sizes vec_elems of the respective player; must not alias.
 * Asynchronous on `stream`. */
int matvec_A(Game* g, const float* y_dev, float* out_dev, void* stream);

/* out = A^T x.  x: player 0's vectors, out: player 1's.  As matvec_A. */
int matvec_AT(Game* g, const float* x_dev, float* out_dev, void* stream);

/* FP64 forms (used for the saddle gap and for precision checks). */
int matvec_A_f64(Game* g, const double* y_dev, double* out_dev, void* stream);
int matvec_AT_f64(Game* g, const double* x_dev, double* out_dev, void* stream);

/* Both products of one matvec pair in a single launch (x and y independent):
 * out_x = A y, out_y = A^T x. */
int matvec_pair(Game* g, const float* y_dev, const float* x_dev, float* Ay_dev,
                float* ATx_dev, void* stream);

/* ---- Technique B's explicit factors (Section 4; a cross-check) ----------- */
/* Sizes of the explicit sparsification A = Ahat + U M^-1 V^T of a
 * one-instance river endgame (Technique B with the Postprocessing
 * subsection's removal of V's zero columns), as stored nonzeros (Table 1's
 * size metric), and the solve's dimension. */
typedef struct {
  int64_t nnz_A;                          /* nonzeros of A itself                  */
  int64_t nnz_ahat, nnz_u, nnz_m, nnz_v;  /* before postprocessing                  */
  int64_t nnz_u_pp, nnz_m_pp, nnz_v_pp;   /* after (Ahat is unchanged)              */
  int64_t m_dim, m_dim_pp;                /* unknowns of M before / after            */
  int32_t chain_depth;                    /* longest chain of M after postprocessing */
} TbSizes;
/* Build the explicit factors on the host (and, for a device game, their CSR
 * forms and M's chains on the device; the device path needs every row and
 * column of the postprocessed M to hold at most one off-diagonal entry).
 * PMX_EINVAL for a batch or a turn + river game.  sizes may be NULL.
 * Synchronous. */
int tb_build(Game* g, TbSizes* sizes);
/* The factors after postprocessing as CSR (library-owned host arrays, valid
 * until the next tb_build or game_destroy): which = 0 Ahat (rows: Player 1's
 * vector elements, columns: Player 2's), 1 U (rows: Player 1's elements,
 * columns: the solve's unknowns), 2 M (unknowns x unknowns, unit lower
 * triangular, diagonal included), 3 V (rows: Player 2's elements, columns:
 * the unknowns); so that A = Ahat + U M^-1 V^T over the vector layout of
 * game_layout.  PMX_ESTATE before tb_build, PMX_EINVAL for another which. */
typedef struct {
  int64_t rows, cols, nnz;
  const int64_t* ptr;                     /* rows + 1 */
  const int32_t* idx;                     /* nnz column indices */
  const double* val;                      /* nnz values */
} TbMatrix;
int tb_matrix(const Game* g, int32_t which, TbMatrix* out);
/* A y and A^T x through the explicit factors, FP64, on the device: CSR
 * products for Ahat, U and V (one wavefront per row) and M's unit triangular
 * solve by pointer jumping along its chains (ceil(log2 depth) rounds).  Same
 * vectors as matvec_A_f64 / matvec_AT_f64.  PMX_ESTATE before tb_build.
 * Asynchronous. */
int matvec_A_tb(Game* g, const double* y_dev, double* out_dev, void* stream);
int matvec_AT_tb(Game* g, const double* x_dev, double* out_dev, void* stream);

/* ---- regret matching+ solver (Section 5; per hand, all hands in parallel) -- */

/* Reset to t = 0: zero regrets and averages, uniform current strategies.
 * Asynchronous. */
int solver_reset(Game* g, void* stream);

/* Solver rule: kind 0 = regret matching+ (default); kind 1 = discounted CFR,
 * the family of the paper's GPU solver (Section 5): regrets scaled by
 * t^alpha/(t^alpha+1) when positive and t^beta/(t^beta+1) otherwise before
 * the instantaneous regret is added, strategies from the positive part, and
 * iterate t weighted t^gamma in the average (gamma in {1, 2, 3}).  Takes
 * effect from the next iteration; averages already accumulated are kept.
 * Synchronizes the device. */
int solver_set_params(Game* g, int32_t kind, double alpha, double beta, int32_t gamma);

/* Run n_iters alternating RM+ iterations: g1 = A y_t, update Player 1;
 * g2 = -A^T x_{t+1}, update Player 2; averages += t * (x_t, y_t).
 * Asynchronous. */
int solver_step(Game* g, int32_t n_iters, void* stream);

/* Retire or revive instances of a batch: active_host[i] = 0 makes
 * solver_step skip instance i (its regrets, plans and averages stay frozen,
 * and so does its averaging weight total, see solver_get_weights);
 * saddle_gap and get_average_strategy still report every instance, each
 * normalized by its own weight total.  When the active set has halved since the
 * solver's launch lists were built, or a revived instance is missing from
 * them, the lists are rebuilt without the retired instances (their
 * workgroups are then not dispatched); this synchronizes the device and
 * drops the captured solver graph.  solver_reset revives all (and restores
 * the lists the same way).  Synchronizes `stream`. */
int solver_set_active(Game* g, const int32_t* active_host, void* stream);

/* FP64 saddle gap of the average strategies (exploitability = gap / 2, over
 * the initial pot 2 * contrib).  An instance's average is its weighted sum
 * divided by its own weight total; one with no weight yet (retired before
 * its first iteration) stands at its current plan.  Values are kept per
 * instance: one not iterated since the last call (a retired instance)
 * reuses them, until solver_reset, solver_set_state, solver_set_weights,
 * set_initial_strategy or warm_apply changes the state.  gap, br1, br2 are host arrays with one
 * entry per instance: br1 = max_x x^T A ybar, br2 = min_y xbar^T A y,
 * gap = br1 - br2 >= 0 (chips).  Synchronizes `stream`. */
int saddle_gap(Game* g, double* gap, double* br1, double* br2, void* stream);

/* Divergence guard of saddle_gap (failure detection): PMX_ENUMERIC, naming
 * the instance, once an instance's computed gap has grown (by more than
 * 1e-12 of its pot) over k computations in a row; the out arrays of that
 * call are then left untouched.  The count restarts whenever the gap does
 * not grow and at solver_reset, solver_set_state, set_initial_strategy and
 * warm_apply (not at solver_set_weights: new weight totals rescale the
 * averages of the same run).  k = 0 disables the guard; the
 * default is 16.  A non-finite best response is PMX_ENUMERIC whatever k. */
int solver_set_gap_guard(Game* g, int32_t k);

/* The same for given sequence-form strategies (device FP64 vectors of each
 * player, vec_elems each).  Synchronizes `stream`. */
int saddle_gap_of(Game* g, const double* x_dev, const double* y_dev, double* gap,
                  double* br1, double* br2, void* stream);

/* saddle_gap_of for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels, with the FP64 gradients, stage rows, per-hand values and
 * per-instance sums in one static device array of 32 MiB per GPU (set up at
 * game_create on the game's device, held until the process ends).  The
 * call allocates nothing, on the device or the host: br1 and br2 (host
 * arrays, one entry per instance) are required and receive the sums; gap
 * may be NULL.  PMX_EINVAL when the game needs more scratch than the array
 * holds (8 bytes per element of both players' vectors, deep-piece stage
 * rows and hands, each part rounded up to 256 bytes; about 4 M elements:
 * single river endgames and small batches fit, the batch of 512 and the
 * turn + river game do not).  Calls on one GPU share its array: calls that
 * overlap on one GPU (other streams or threads) race.  Synchronizes
 * `stream`. */
int saddle_gap_of_static(Game* g, const double* x_dev, const double* y_dev, double* gap,
                         double* br1, double* br2, void* stream);

/* Copy solver state to / from host arrays (NULL skips a field).  Regrets and
 * current plans are FP32, averages FP64 (weighted sums).  t = iterations
 * done; wsum = sum of the averaging weights of all iterations, which is each
 * instance's own total unless it was retired for some (solver_get_weights).
 * solver_set_state gives every instance the weight total wsum. */
int solver_get_state(Game* g, int32_t player, float* regret, float* plan,
                     double* avg_sum, int32_t* t, double* wsum);
int solver_set_state(Game* g, int32_t player, const float* regret, const float* plan,
                     const double* avg_sum, int32_t t, double wsum);

/* Averaging weight totals, one per instance (host FP64 arrays): the sum of
 * the weights of the iterations the instance took part in (DCFR: t^gamma;
 * RM+: t), by which its averages are divided.  solver_set_weights restores
 * them after solver_set_state; PMX_EINVAL on a negative or non-finite
 * total.  Host-side only. */
int solver_get_weights(Game* g, double* wsum_host);
int solver_set_weights(Game* g, const double* wsum_host);

/* A device-side copy of the solver state (both players' regrets, plans and
 * average sums, the per-instance weight totals and the iteration count),
 * kept by the game (allocated at the first call: 16 B per vector element);
 * asynchronous on `stream`.  solver_restore_instances copies the snapshot's
 * state back for every instance i with restore[i] != 0 (host array, one flag
 * per instance) and leaves the others as they are: the per-instance choice
 * between two runs of the same length, e.g. the uniform start as the
 * fallback of a warm start judged by the FP64 gap.  PMX_ESTATE without a
 * snapshot or when the iteration count differs from the snapshot's. */
int solver_snapshot(Game* g, void* stream);
int solver_restore_instances(Game* g, const int32_t* restore, void* stream);

/* Average strategy in sequence form (FP64 host array, vec_elems): each
 * instance's weighted sums over its own weight total, or its current plan if
 * it has none. */
int get_average_strategy(Game* g, int32_t player, double* x_host);

/* Warm start: behavioural strategy b(a|I) per sequence (device FP32,
 * vec_elems), used as the current strategy (regrets = scale * b). */
int set_initial_strategy(Game* g, int32_t player, const float* behav_dev, float scale,
                         void* stream);

/* ---- learned warm start (not in the paper; a prior for the solver) -------- */
/* The network sees one row per (infoset I, hand h) of a player, rows ordered
 * instance by instance, infosets in layout order, hands in list order.  Row
 * features (64, BF16): 59 betting features of I (pot, stacks and amount to
 * call relative to the pot, raises, depth, round, and per action slot its
 * kind and added chips; 8 slots) followed by 5 range features of h (belief
 * weight relative to the mean, strength quantile, share of the opponent's
 * range it blocks, compatible opponent mass it beats / loses to).  Infosets
 * with more than 8 actions make the warm start unavailable (PMX_EINVAL). */
int warm_num_rows(const Game* g, int32_t player, int64_t* rows);
/* x_dev: device BF16 [rows][64]. Asynchronous. */
int warm_features(Game* g, int32_t player, uint16_t* x_dev, void* stream);
/* Training targets from the solver's average strategy: target_dev [rows][8]
 * holds xbar[Ia] / xbar[parent(I)] for valid slots (uniform if unreached) and
 * -1 for invalid slots; weight_dev [rows] = relative belief weight x average
 * reach of I (0 for an instance with no weight total).  Needs at least one
 * solver iteration.  Synchronizes `stream`. */
int warm_targets(Game* g, int32_t player, float* target_dev, float* weight_dev, void* stream);
/* Reset the solver to the prior given by network logits (device FP32
 * [rows][ldz] per player): masked softmax per row -> behavioural prior b0;
 * regrets = regret_scale * lambda(h) * pot * b0 (the units of that hand's
 * gradients), current plans = realization of b0, averages
 * seeded as avg_weight iterations of b0.  Asynchronous. */
int warm_apply(Game* g, const float* logits0_dev, const float* logits1_dev, int32_t ldz,
               float regret_scale, double avg_weight, void* stream);

/* ---- network kernels (device buffers, asynchronous) ----------------------- */
/* C[M x N] = op(A) op(B) on the BF16 matrix cores with FP32 accumulation;
 * op(A)(m,k) = transA ? A[k*lda + m] : A[m*lda + k], op(B)(k,n) = transB ?
 * B[n*ldb + k] : B[k*ldb + n].  Epilogue: + bias[n] (if bias), ReLU (if relu),
 * zero where mask[m*ldm + n] <= 0 (if mask); stored as FP32 C and / or BF16 Cb
 * (either may be NULL, not both).  work: optional caller-owned device FP32
 * workspace of work_elems elements (NULL / 0: none).  When M x N gives few
 * 64 x 64 tiles and K is long (weight gradients), K is split into ranges
 * whose partial products go to work (at most work_elems / (M*N) ranges, up
 * to 64) and are added in range order, so the result does not depend on
 * timing; it does depend on the number of ranges.  Must not alias C or Cb. */
int mlp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, int32_t lda, int32_t transA,
                  const uint16_t* B, int32_t ldb, int32_t transB, const float* bias, int32_t relu,
                  const float* mask, int32_t ldm, float* C, int32_t ldc, uint16_t* Cb, int32_t ldcb,
                  float* work, int64_t work_elems, void* stream);
/* Masked softmax cross-entropy over K <= 64 slots (target < 0 = invalid):
 * dlogits[r][a] = weight[r] (softmax - target) (FP32 and / or BF16, stride K);
 * loss_partial[b] = sum of weight[r] * cross-entropy over block b's 256 rows. */
int mlp_softmax_xent(int32_t rows, int32_t K, const float* logits, int32_t ldl, const float* target,
                     const float* weight, float* dlogits, uint16_t* dlogits_bf16, float* loss_partial,
                     void* stream);
/* db[n] = sum_m dz[m][n] (bias gradient), in a fixed order.  work: optional
 * device FP32 workspace of ceil(rows / 64) * cols elements (NULL, or too
 * small: one thread per column walks every row). */
int mlp_colsum(int32_t rows, int32_t cols, const float* dz, float* db, float* work, int64_t work_elems,
               void* stream);
/* Adam with bias correction and decoupled-free L2 weight decay; writes the
 * BF16 copy of the weights when w_bf16 is not NULL. */
int mlp_adam(int64_t n, float* w, const float* g, float* m, float* v, uint16_t* w_bf16, float lr,
             float beta1, float beta2, float eps, float weight_decay, int32_t step, void* stream);
/* dst[i][:] = src[idx[i]][:] for rows of `width` elements. */
int mlp_gather_bf16(int64_t n, int32_t width, const int64_t* idx, const uint16_t* src, uint16_t* dst,
                    void* stream);
int mlp_gather_f32(int64_t n, int32_t width, const int64_t* idx, const float* src, float* dst,
                   void* stream);
/* dst = BF16(src), round to nearest even. */
int mlp_cast_bf16(int64_t n, const float* src, uint16_t* dst, void* stream);

/* Thread-local description of the last error ("" if none). */
const char* pmx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMX_H */
