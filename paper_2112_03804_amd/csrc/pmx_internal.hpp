// Internal host-side structures of libpmx: validated instances, the betting
// skeleton and its sequence form, hand metadata for the structured hand
// operators, and the work plans consumed by the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "pmx.h"

namespace pmx {

constexpr int kMaxHands = 1280;   // per player and instance
constexpr int kMaxDeck = 64;
constexpr double kEps = 1e-9;      // chip arithmetic: snapping and de-duplication

struct Error {
  int code;
  std::string msg;
};

// ---------------------------------------------------------------------------
// validated copy of one GameDesc
// ---------------------------------------------------------------------------
struct Instance {
  int deck = 0, cph = 0;
  std::vector<uint8_t> board, rivers;
  int n[2] = {0, 0};
  std::vector<uint8_t> cards[2];        // n x cph
  std::vector<int32_t> strength[2];     // nb x n
  std::vector<double> mu[2];
  double contrib = 0, stack[2] = {0, 0};
  std::vector<double> fracs;            // ascending
  bool has_menu = false;                // per-player, per-situation sizes replace fracs
  std::vector<double> menu[2][5];       // ascending; situations as in bet_situation
  int max_raises = 0;
  bool allin = false;
  int nb = 1;                           // final boards (max(1, n_river))
  bool two_rounds() const { return !rivers.empty(); }
  int remaining() const { return deck - (int)board.size() - 2 * cph; }
};

// ---------------------------------------------------------------------------
// sequence form
// ---------------------------------------------------------------------------
struct Infoset {
  int parent, first, nact, board;
};
struct Terminal {
  int seq[2];
  int kind;
  int board;
  int runout;
  double c1, c2;
};
struct RiverTask {      // one (chance node, river card) subtree
  int board;
  int parent_seq[2];    // each player's last first-round sequence
  int inf_begin[2], inf_end[2];
};
constexpr int kWarmActions = 8;        // action slots of the warm-start network
constexpr int kInfFeat = 11 + 6 * kWarmActions;   // betting features per infoset (59)
constexpr int kHandFeat = 5;           // range features per hand
constexpr int kWarmIn = 64;            // network input width (kInfFeat + kHandFeat)

struct SeqForm {
  int n_seq[2] = {0, 0};
  std::vector<Infoset> inf[2];
  std::vector<Terminal> terms;
  std::vector<RiverTask> rivers;        // empty for a river endgame
  std::vector<float> inf_feat[2];       // kInfFeat per infoset (warm-start inputs)
};

// ---------------------------------------------------------------------------
// hand metadata of one (board context, player)
// ---------------------------------------------------------------------------
// Scan side: the player's live hands sorted by (strength, index) and the
// entry list of the segmented scan: segment 0 = all live hands, segment 1+c =
// live hands holding card c, each in sorted order and closed by a sentinel.
// An entry holds the sorted position of its hand, or -1-seg for a sentinel.
// Query side: positions in the *opponent's* scan side that bracket a hand.
struct QueryRec {                       // 8 x int32, the kernel's record
  int32_t lt, le;                       // global: opp live hands weaker / not stronger
  int32_t lt0, le0, lt1, le1;           // same inside each own card's segment (absolute entry index)
  int32_t cards;                        // c0 | c1 << 8 (c1 = 255 for one-card hands)
  int32_t self;                         // sorted position of the identical opp hand, -1 none
};
// The kernel's packed form of a QueryRec (16 bytes): x = lt | le << 16,
// y = lt0 | le0 << 16, z = lt1 | le1 << 16, w = c0 | c1 << 8 | self << 16.
struct QueryRec16 {
  uint32_t x, y, z, w;
};
struct CtxMeta {
  // scan side of this player
  int n_live = 0;
  std::vector<int32_t> rank;            // n
  std::vector<int32_t> seg_src;         // entries
  std::vector<int32_t> seg_end;         // 1 + deck: sentinel entry index of each segment
  std::vector<int32_t> sorted_strength; // n_live, ascending
  // query side of this player against the opponent's scan side
  std::vector<QueryRec> q;              // n
};

// ---------------------------------------------------------------------------
// per-instance build result
// ---------------------------------------------------------------------------
struct Built {
  Instance inst;
  SeqForm sf;
  double beta = 0;
  std::vector<double> lam[2];
  int n_ctx = 1;
  std::vector<CtxMeta> ctx[2];          // [player][ctx]
  int stride[2] = {0, 0};
  int64_t vec_off[2] = {0, 0};
  // exported layout arrays
  std::vector<int32_t> inf_parent[2], inf_first[2], inf_nact[2], inf_board[2];
  std::vector<int32_t> t_seq1, t_seq2, t_kind, t_board, t_runout;
  std::vector<double> t_c1, t_c2;
  std::vector<float> hand_feat[2];      // kHandFeat per hand (warm-start inputs)
};

// ---------------------------------------------------------------------------
// kernel plans (plain structs, copied to the device verbatim)
// ---------------------------------------------------------------------------
struct MvCtx {                          // (instance, context) as seen by one direction
  int32_t n_own, n_opp, n_live, n_ent;
  int32_t n_seg, cph, stride_own, pad;
  int64_t q_off;                        // QueryRec offset (own)
  int64_t rank_off;                     // opp rank offset
  int64_t seg_off;                      // opp entries offset
  int64_t segend_off;                   // opp seg_end offset
  int64_t lam_own_off, lam_opp_off;
};
struct MvItem {
  int64_t out, in_f, in_s;              // element offsets (in_* = -1: absent)
  int32_t ctx;                          // -1: the row has no terminal, write zeros
  int32_t last;                         // 1: last item of its output row; 2: last item of a
                                        //    partial row (out indexes the direction's partial buffer)
  int32_t n_own, stride;                // output row length and padded stride
  double kf, ks;                        // coefficients (payoff x chance)
  int32_t run_end;                      // one past the last item of this chunk with the same ctx
  int32_t n_opp;                        // opponent hands of the context (0 without one)
};
// An output row whose terms span many board contexts (a turn all-in run-out
// sums over every river card) is cut into parts of a few contexts each; the
// parts run as chunks of their own and write partial rows, which one more
// launch sums in part order into the output row.
struct MvRed {
  int64_t out;                          // element offset of the output row
  int64_t part;                         // element offset of its first partial row (rows `stride` apart)
  int32_t n_parts, stride;              // partial rows; row length incl. padding
  int32_t inst, pad;                    // instance (skipped when retired)
};
struct MvDir {                          // host copy of one direction's plan
  std::vector<MvCtx> ctx;
  std::vector<MvItem> items;
  std::vector<MvRed> red;               // rows summed from partial rows
  int64_t part_elems = 0;               // length of the partial buffer
  std::vector<int32_t> blk;             // item ranges: blk[b] .. blk[b+1]
  std::vector<int32_t> blk_inst;        // instance of each chunk
  std::vector<QueryRec16> q;
  std::vector<int16_t> rank, seg;
  std::vector<int32_t> segend;
  int max_ent = 0, max_seg = 0, max_n = 0;
  // wave kernel: chunks grouped by hand-count class (LDS sized per class)
  static constexpr int kClasses = 3;
  std::vector<int32_t> cls_chunks[kClasses];
  int cls_ent[kClasses] = {0, 0, 0}, cls_n[kClasses] = {0, 0, 0};
};
constexpr int kClassN[MvDir::kClasses] = {512, 1024, 1280};   // hands per player, upper bounds

// Chunk-aligned matvec layout (kernels 2 and 3).  The opponent's scan side
// is laid out segment by segment (segment 0: all live hands by strength;
// segment 1 + c: live hands holding card c), each segment starting at a
// thread chunk of KE entries and owning ceil((len + 1) / KE) chunks, so the
// slot after its last entry (its total) lies in its own last chunk.  Entry i
// of a chunk sits at LDS slot chunk * SK + i (SK = KE plus padding that keeps
// the 16-byte chunk reads of a wavefront free of bank conflicts).
constexpr int kMcClasses = 5;            // hands per thread: 1..5
constexpr int kMcSegMax = 1 + kMaxDeck;
inline int mc_ke(int block, int kh) { return block == 512 ? 4 * kh : 4 * kh + 4; }
inline int mc_sk(int ke) { return ke + (ke % 8 == 0 ? 4 : 0); }
struct McCtx {                           // (instance, context) as seen by one direction
  int32_t n_own, n_opp, cph, n_chunk;
  int64_t q_off;                         // own query records (uint4)
  int64_t pos_off;                       // opponent hands' three slots (uint2)
  int64_t meta_off;                      // per-thread chunk descriptors (block entries)
  int64_t lam_own_off, lam_opp_off;
};
// Chunk descriptor bits: 0-7 valid entries, 8 first chunk of a segment,
// 16-23 (segment + 1) when the chunk is the last of its segment.
// Slots are stored as byte offsets of 4-byte values (int16; -1 = none).
struct McDir {
  int block = 256;                       // threads per workgroup the layout is built for
  std::vector<McCtx> ctx;                // same indexing as MvDir::ctx
  std::vector<QueryRec16> q;             // x: lt|le (global), y: lt0|le0, z: lt1|le1 (card slots),
                                         // w: c0 | c1 << 8 | self slot << 16
  std::vector<uint32_t> pos;             // pairs: (global | card0 << 16, card1 | 0xffff << 16)
  std::vector<uint32_t> meta;
  std::vector<int32_t> chunks[kMcClasses];   // per class: 4 ints per row chunk (it0, it1, inst, ctx)
};

// Grouped matvec layout (kernel 4, FP32).  A group applies the hand
// operators to up to kGrpComps input rows of one board context at once: each
// component is one opponent row u = lambda_opp * v; the fold operator of eq.
// (cf) and the showdown operator (Technique B) are linear, so one segmented
// scan of u serves every terminal that reads that row, and the payoff
// coefficients enter when the own hands combine the prefix sums.  Output o
// of a group takes the showdown operator of component o and the fold
// operator of component fc(o).  Per context, the workgroup stages the
// components' weighted opponent values as one 16-byte row per live hand in
// strength order (row pu(i) = i + i / 16 for sorted position i; the zero row
// follows the last hand and a trash row takes the hands dead in the
// context), gathers each thread's chunk of the segmented entry list from
// those rows, scans, and stores the exclusive prefix sums of entry i of chunk
// t at slot i * BLOCK + t of the same LDS region.
constexpr int kGrpComps = 4;
constexpr int kGrpBlock = 256;                  // threads per workgroup
constexpr int kGrpClasses = 5;                  // hands per thread 1..5
constexpr int kGrpTwoWideMinRows = 1024;        // output rows of a product from which two-wide launches are used
constexpr int kGrpKE[kGrpClasses] = {4, 8, 12, 16, 18};   // scan entries per thread per class
inline int grp_urow(int i) { return i + (i >> 4); }
struct GCtx {                           // (instance, context) as seen by one direction
  int32_t n_own, n_opp, cph, n_chunk;
  int32_t zrow, trash;                  // LDS byte offsets of the zero row and the trash row
  int32_t pad0, pad1;
  int64_t q_off;                        // own hands' query records (uint4)
  int64_t rk_off;                       // opponent hands' staging rows (uint16 LDS byte offsets)
  int64_t src_off;                      // entry sources: pairs of uint16 LDS byte offsets, entry-pair major
                                        // (pair j of thread t at src_off + j * kGrpBlock + t)
  int64_t meta_off;                     // per-thread chunk descriptors (kGrpBlock entries)
  int64_t lam_own_off, lam_opp_off;
};
struct GGroup {
  int32_t in[kGrpComps];                // component input rows (element offsets; -1: none)
  int32_t out[kGrpComps];               // output rows (element offsets; -1: none)
  double ks[kGrpComps];                 // output o: coefficient of the showdown operator on component sc(o)
  double kf[kGrpComps];                 // output o: coefficient of the fold operator on component fc(o)
  int32_t ctx;                          // -1: the group only writes rows without terminals (zeros)
  int32_t fc;                           // fold component of output o in bits 2o, 2o + 1
  int32_t acc;                          // bit o: output o starts its sum here; bit 4 + o: it ends here (stored)
  int32_t n_own, stride;                // row length and stride of the outputs
  int32_t n_in;                         // row length of the inputs (opponent hands)
  int32_t sc;                           // showdown component of output o in bits 2o, 2o + 1: o itself,
                                        // except in two-wide groups (components compacted to 0 and 1)
  int32_t pad;
};   // element offsets are 32-bit: the layout builder rejects vectors of 2^31 elements or more
// Group query record (uint4): x = prefix slot of lt | slot of le << 16 (global
// segment), y = the same in card c0's segment, z = in card c1's segment,
// w = c0 | c1 << 6 | (identical opponent hand present) << 12 | (its global
// entry is the last of its chunk) << 13 | (prefix slot of that entry) << 14;
// a hand dead in the context has x = 0xffffffff.
// Chunk descriptor bits: 8 first chunk of a segment, 16-23 (segment + 1)
// when the chunk is the last of its segment.
struct GrpDir {
  std::vector<GCtx> ctx;
  std::vector<GGroup> groups;
  std::vector<uint32_t> q, src, meta;
  std::vector<uint16_t> rk;
  // per kind (0: every sequence one group, 1: sequences carrying sums over
  // several groups, 2: as 0 for groups of at most two components, whose
  // launches use two-wide slots, 3: as 0 for groups whose showdown terms
  // read at most two of their components, which alone get prefix slots) and
  // class: 4 ints per chunk (g0, g1, inst, ctx of g0)
  static constexpr int kKinds = 4;
  std::vector<int32_t> chunks[kKinds][kGrpClasses];
  int max_chunk[kGrpClasses] = {0, 0, 0, 0, 0};
};

// Technique B's explicit factors of a one-instance river endgame (host and
// the GPU cross-check path; see host_sparsify.cpp).
struct TbCsr {
  int64_t rows = 0, cols = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> idx;
  std::vector<double> val;
};
struct TbHost {
  int64_t nnz_A = 0;
  int64_t nnz[4] = {0, 0, 0, 0};        // Ahat, U, M, V before postprocessing
  int64_t nnz_pp[4] = {0, 0, 0, 0};     // after postprocessing
  int64_t m_dim = 0, m_dim_pp = 0;      // the solve's dimension before / after
  TbCsr ahat, ahat_t, u, u_t, v, v_t;   // over vector elements (rows x cols as named)
  std::vector<int32_t> par, chi;        // M's chains: parent / child of each unknown (-1: none)
  std::vector<double> cpar, cchi;       // z_k = r_k + cpar_k z_par(k);  w_i = r_i + cchi_i w_chi(i)
  int depth = 0;                        // longest chain
};

struct TpTask {                         // treeplex task: one subtree of one instance
  int64_t vec_base;
  int32_t stride, n_hands;
  int32_t inf_begin, inf_end;           // range into the task's infoset id list
  int32_t stage;                        // deep task: row of the stage buffer, else -1
  int32_t pull_begin, pull_end;         // top task: stage rows to pull
  int32_t inst;
  int32_t hand_base;                    // offset of this instance's hands in per-hand outputs
  int32_t ext_parent;                   // deep task: the first-round sequence its roots hang from
  int32_t seq_begin, seq_end;           // contiguous sequences owned by the task (-1: not contiguous)
};
struct TpPull {
  int32_t seq;                          // instance-relative sequence receiving the value
  int32_t stage;
};
struct TpPlan {                         // one player
  std::vector<int32_t> inf_parent, inf_first, inf_nact;   // global infoset table (seq ids relative)
  std::vector<int32_t> order;           // infoset ids of each task, DFS order
  std::vector<TpTask> tasks;
  std::vector<TpPull> pulls;
  std::vector<int32_t> deep, top, single;                 // task ids per phase
  int n_stage = 0, stage_stride = 0;
  int64_t hands_total = 0;
};

// Regret-update tasks.  Each player's treeplex is cut into pieces of at most
// `task_rows` sequences and kTaskInfMax infosets, so that a piece's rows for
// 64 hands stay resident in LDS during the bottom-up and top-down passes.
// A piece is a forest of whole
// infoset subtrees of what remains of the treeplex once the deeper pieces are
// cut away.  A piece whose roots hang from a sequence of another piece (a
// "deep" piece) passes its root values up through a stage buffer and reads
// the parent sequence's realization weight back in its top-down pass.
constexpr int kTaskRowsMax = 64;        // rows per piece (one per lane of a wavefront)
constexpr int kTaskInfMax = 64;         // infosets per piece (one per lane)
// A game whose every treeplex fits one piece of at most kTaskRowsWhole rows
// (and kTaskInfMax infosets), with few hand blocks in all, takes one piece per
// treeplex: one fused launch per player, four lanes per hand (16 hands per
// workgroup keep the rows in LDS; LDS row numbers stay below 256).
constexpr int kTaskRowsWhole = 192;
constexpr int kTaskExtMax = 15;         // distinct external parents per piece
constexpr int kRmGroups = 4;            // subtree groups walked concurrently (wavefronts per block)
constexpr int kRmGroupSlots = 4;        // distinct parent targets of one group's roots
// Group table of a split piece (64 ints): [kRmGBeg + w] / [kRmGEnd + w] the
// infoset range of group w, [kRmGTop] / [kRmGTop + 1] the range of the top
// part, [kRmGCnt + w] the number of accumulator slots of group w, and
// kRmMergeMax merge entries, two per int from [kRmGMrg] (entry 2i in bits
// 0-15, 2i+1 in bits 16-31): the LDS row of a group-root slot (bits 0-7) and
// of its target (bits 8-15).  Entries are sorted by target, the slots of one
// target in group order; the list is filled up at its front with entries
// whose slot and target are the root sink row (nothing reads it before the
// top-down pass sets it to 1).
constexpr int kRmMergeMax = kRmGroups * kRmGroupSlots;
constexpr int kRmGBeg = 1;
constexpr int kRmGEnd = kRmGBeg + kRmGroups;
constexpr int kRmGTop = kRmGEnd + kRmGroups;
constexpr int kRmGCnt = kRmGTop + 2;
constexpr int kRmGMrg = kRmGCnt + kRmGroups;
static_assert(kRmMergeMax % 2 == 0 && kRmGMrg + kRmMergeMax / 2 <= 64,
              "the group table is read one entry per lane");
// LDS rows of a regret-update workgroup in one index space (a row holds one
// value per hand of the workgroup): the root sink / root weight, the
// group-root accumulator slots (kRmGroupSlots per wavefront), the external
// parents, then the piece's rows.  With a 64-row piece the values (g, then
// the new x) and the regrets take 2 * 64 rows after these 32, 40 KiB per
// workgroup, so four workgroups share a CU's 160 KiB.
constexpr int kRmRowOne = 0;
constexpr int kRmRowSlot = 1;
constexpr int kRmRowExt = kRmRowSlot + kRmGroups * kRmGroupSlots;
constexpr int kRmRowLocal = kRmRowExt + kTaskExtMax;
struct RmTask {
  int64_t vec_base;
  int32_t stride, n_hands;
  int32_t rows_off, n_rows;             // sorted instance-relative sequence ids of the piece
  int32_t inf_off, n_inf;               // packed local infosets, depth-first order
  int32_t pull_off, n_pull;             // stage rows added into local rows before the walk
  int32_t ext_off, n_ext;               // external parents: sequence and stage row
  int32_t inst, depth;
  int32_t grp_off;                      // 64-int group table, -1: one wavefront walks the piece
  int32_t row0;                         // rows are row0 .. row0 + n_rows - 1, or -1: use the table
};
// Packed local infoset: first local row (bits 0-7) | actions (bits 8-15) |
// LDS row that receives the infoset's value in the bottom-up pass (bits
// 16-23: the group-root slot for a group root, else the parent sequence's
// row, the external parent's row, or the sink) | LDS row holding the parent
// sequence's realization weight in the top-down pass (bits 24-31: the
// parent's row, the external parent's row, or the root-weight row).  LDS
// rows as numbered by kRmRow*.  Pulls of a piece (when it has any): kRmGroups
// counts, then wavefront w's pulls (local rows r with r % kRmGroups == w),
// each local row (bits 0-7) | stage row << 8, in row order.
// Group table: as described at kRmGBeg.  Infosets are listed group by group,
// then the top part, each in depth-first order.
struct RmPlan {                         // one player
  std::vector<RmTask> tasks;
  std::vector<int32_t> rows, infs, pulls, ext_seq, ext_slot, grp;
  std::vector<std::vector<int32_t>> by_depth;   // task ids per depth (0: no external parent)
  int n_slot = 0, stage_stride = 0;
  int max_rows[2] = {0, 0}, max_ext[2] = {0, 0};   // [depth 0, deeper] LDS sizing
};

struct HostGame {
  std::vector<Built> inst;
  int64_t elems[2] = {0, 0};
  int mv_kernel = 4;                    // FP32 products: 2 / 3 chunk-aligned layout with 256 / 512
                                        // threads, 4 grouped layout
  int rows_per_block = 1;               // chunk-aligned layout (also the FP64 products): rows per chunk
  int mc_block = 256;                   // chunk-aligned layout: threads per workgroup
  int groups_per_chunk = 1;             // kernel 4: groups per workgroup
  MvDir dir[2];
  McDir mc[2];
  GrpDir grp[2];
  TpPlan tp[2];
  RmPlan rm[2];
  int task_rows = kTaskRowsMax;
  int rm_quad_max = 256;                // regret launches of at most this many block records use k_rmq
  bool rm_whole = false;                // one piece per treeplex (kTaskRowsWhole; see above)
  int max_stride = 0;
};

// host_build.cpp
int validate(const GameDesc& d, Instance& out, std::string& msg);
void build_seqform(const Instance& in, SeqForm& sf);
void build_hand_meta(Built& b);
int build_game(const GameDesc* descs, int n, HostGame& hg, std::string& msg);
int default_rows_per_block(int64_t rows, int kernel);
int default_mv_kernel(int64_t mean_hands);
void build_matvec_plan(HostGame& hg, int d, int rows_per_block);
int build_rm_plan(HostGame& hg, int p, int task_rows, std::string& msg);
int build_mc_layout(HostGame& hg, int d, int block, std::string& msg);
int build_grp_layout(HostGame& hg, int d, int groups_per_chunk, std::string& msg);
// host_sparsify.cpp
int build_tb_factors(const HostGame& hg, TbHost& out, std::string& msg);

}  // namespace pmx
