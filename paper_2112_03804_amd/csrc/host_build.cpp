// Host-side game construction for libpmx: descriptor validation, the betting
// skeleton and its sequence form, hand metadata for the structured hand
// operators, and the kernels' work plans.
//
// Betting rules (paper, Appendix A and the caption of Fig. 1): check or bet
// when not facing a bet; fold, call or raise when facing one; a bet or raise
// matches the opponent and then adds a fraction of the pot after matching;
// nobody puts in more than the opponent can match (that maximum is the
// all-in); the round ends on a fold, a call or two checks.  Raises after the
// opening bet are capped at max_raises; the all-in stays available past the
// cap (Fig. 1, nodes K and O).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <utility>

#include "pmx_internal.hpp"

namespace pmx {

namespace {

int hand_key(const uint8_t* c, int cph) {
  if (cph == 1) return c[0];
  int a = c[0], b = c[1];
  if (a > b) std::swap(a, b);
  return a * kMaxDeck + b;
}

bool holds(const Instance& in, int p, int h, int card) {
  for (int k = 0; k < in.cph; ++k)
    if (in.cards[p][h * in.cph + k] == card) return true;
  return false;
}

}  // namespace

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
int validate(const GameDesc& d, Instance& o, std::string& msg) {
  auto bad = [&](const std::string& m) {
    msg = m;
    return PMX_EINVAL;
  };
  if (d.deck_size < 2 || d.deck_size > kMaxDeck) return bad("deck_size must be in [2, 64]");
  if (d.cards_per_hand != 1 && d.cards_per_hand != 2) return bad("cards_per_hand must be 1 or 2");
  if (d.n_board < 0 || d.n_board > d.deck_size) return bad("n_board out of range");
  if (d.n_board > 0 && !d.board) return bad("board is NULL");
  o.deck = d.deck_size;
  o.cph = d.cards_per_hand;
  std::vector<int> on_board(o.deck, 0);
  for (int i = 0; i < d.n_board; ++i) {
    int c = d.board[i];
    if (c >= o.deck) return bad("board card out of range");
    if (on_board[c]) return bad("board card repeated");
    on_board[c] = 1;
    o.board.push_back((uint8_t)c);
  }
  if (d.n_river < 0) return bad("n_river must be >= 0");
  if (d.n_river > 0) {
    if (!d.river_cards) return bad("river_cards is NULL");
    if (d.n_river != o.deck - d.n_board)
      return bad("river_cards must list every card not on the board");
    std::vector<int> seen(o.deck, 0);
    for (int i = 0; i < d.n_river; ++i) {
      int c = d.river_cards[i];
      if (c >= o.deck || on_board[c] || seen[c])
        return bad("river_cards must list every card not on the board exactly once");
      seen[c] = 1;
      o.rivers.push_back((uint8_t)c);
    }
    if (o.remaining() < 1) return bad("no card left for the river");
  }
  o.nb = std::max(1, d.n_river);
  std::vector<int> key_strength_seen;
  for (int p = 0; p < 2; ++p) {
    int n = d.n_hands[p];
    if (n < 1 || n > kMaxHands) return bad("n_hands must be in [1, 1280]");
    if (!d.hand_cards[p] || !d.strength[p] || !d.range[p]) return bad("hand arrays must not be NULL");
    o.n[p] = n;
    o.cards[p].assign(d.hand_cards[p], d.hand_cards[p] + (size_t)n * o.cph);
    o.strength[p].assign(d.strength[p], d.strength[p] + (size_t)n * o.nb);
    o.mu[p].assign(d.range[p], d.range[p] + n);
    std::vector<char> seen_key((size_t)kMaxDeck * kMaxDeck, 0);
    for (int h = 0; h < n; ++h) {
      const uint8_t* c = &o.cards[p][(size_t)h * o.cph];
      for (int k = 0; k < o.cph; ++k) {
        if (c[k] >= o.deck) return bad("hand card out of range");
        if (on_board[c[k]]) return bad("hand uses a board card");
      }
      if (o.cph == 2 && c[0] == c[1]) return bad("hand repeats a card");
      int key = hand_key(c, o.cph);
      if (seen_key[key]) return bad("hand listed twice");
      seen_key[key] = 1;
      double m = o.mu[p][h];
      if (!std::isfinite(m) || m < 0) return bad("range weights must be finite and >= 0");
    }
  }
  // equal strength for a hand present in both lists
  {
    std::vector<int> idx1((size_t)kMaxDeck * kMaxDeck, -1);
    for (int h = 0; h < o.n[1]; ++h) idx1[hand_key(&o.cards[1][(size_t)h * o.cph], o.cph)] = h;
    for (int h = 0; h < o.n[0]; ++h) {
      int j = idx1[hand_key(&o.cards[0][(size_t)h * o.cph], o.cph)];
      if (j < 0) continue;
      for (int b = 0; b < o.nb; ++b) {
        if (!o.rivers.empty() && holds(o, 0, h, o.rivers[b])) continue;
        if (o.strength[0][(size_t)b * o.n[0] + h] != o.strength[1][(size_t)b * o.n[1] + j])
          return bad("a hand in both lists has two different strengths");
      }
    }
  }
  if (!std::isfinite(d.contrib) || d.contrib <= 0) return bad("contrib must be finite and > 0");
  o.contrib = d.contrib;
  for (int p = 0; p < 2; ++p) {
    if (!std::isfinite(d.stack[p]) || d.stack[p] < 0) return bad("stacks must be finite and >= 0");
    o.stack[p] = d.stack[p];
  }
  if (d.n_bet_fracs < 0 || (d.n_bet_fracs > 0 && !d.bet_fracs)) return bad("bad bet_fracs");
  for (int i = 0; i < d.n_bet_fracs; ++i) {
    double f = d.bet_fracs[i];
    if (!std::isfinite(f) || f <= 0) return bad("bet fractions must be finite and > 0");
    o.fracs.push_back(f);
  }
  std::sort(o.fracs.begin(), o.fracs.end());
  if (d.bet_menu_len) {
    o.has_menu = true;
    size_t at = 0;
    for (int p = 0; p < 2; ++p)
      for (int k = 0; k < 5; ++k) {
        const int len = d.bet_menu_len[5 * p + k];
        if (len < 0 || len > 64) return bad("bet_menu_len entries must be in [0, 64]");
        if (len > 0 && !d.bet_menu) return bad("bet_menu is NULL");
        for (int i = 0; i < len; ++i) {
          const double f = d.bet_menu[at++];
          if (!std::isfinite(f) || f <= 0) return bad("bet fractions must be finite and > 0");
          o.menu[p][k].push_back(f);
        }
        std::sort(o.menu[p][k].begin(), o.menu[p][k].end());
      }
  } else if (d.bet_menu) {
    return bad("bet_menu without bet_menu_len");
  }
  if (d.max_raises < 0 || d.max_raises > 64) return bad("max_raises must be in [0, 64]");
  o.max_raises = d.max_raises;
  o.allin = d.allow_allin != 0;
  return PMX_OK;
}

// ---------------------------------------------------------------------------
// betting skeleton
// ---------------------------------------------------------------------------
namespace {

enum { K_P0 = 0, K_P1 = 1, K_LEAF = 2, K_CHANCE = 3 };

struct TNode {
  int kind;
  double c[2], s[2];
  int term = -1, runout = 0;
  int raises = 0, facing = 0;
  std::vector<int> kids;
};

struct TreeBuilder {
  const Instance& in;
  std::vector<TNode> nodes;
  size_t limit = 4u << 20;
  bool overflow = false;
  explicit TreeBuilder(const Instance& i) : in(i) {}

  int add(TNode n) {
    if (nodes.size() >= limit) {
      overflow = true;
      return 0;
    }
    nodes.push_back(std::move(n));
    return (int)nodes.size() - 1;
  }

  int leaf(const double c[2], const double s[2], int term, int runout) {
    TNode n;
    n.kind = K_LEAF;
    n.c[0] = c[0]; n.c[1] = c[1]; n.s[0] = s[0]; n.s[1] = s[1];
    n.term = term;
    n.runout = runout;
    return add(std::move(n));
  }

  int end_round(const double c[2], const double s[2], bool last) {
    if (last) return leaf(c, s, PMX_SHOWDOWN, 0);
    if (s[0] <= kEps || s[1] <= kEps) return leaf(c, s, PMX_SHOWDOWN, 1);
    TNode n;
    n.kind = K_CHANCE;
    n.c[0] = c[0]; n.c[1] = c[1]; n.s[0] = s[0]; n.s[1] = s[1];
    return add(std::move(n));
  }

  int decision(int p, const double c[2], const double s[2], bool facing, int raises, bool checked,
               bool last) {
    if (overflow) return 0;
    const int o = 1 - p;
    const double allin_to = std::min(c[p] + s[p], c[o] + s[o]);
    std::vector<int> kids;
    auto put = [&](double target, double nc[2], double ns[2]) {
      nc[0] = c[0]; nc[1] = c[1]; ns[0] = s[0]; ns[1] = s[1];
      nc[p] = target;
      double rest = s[p] - (target - c[p]);
      ns[p] = std::fabs(rest) < kEps ? 0.0 : rest;
    };
    if (facing) {
      kids.push_back(leaf(c, s, p == 0 ? PMX_FOLD_P1 : PMX_FOLD_P2, 0));
      double nc[2], ns[2];
      put(c[o], nc, ns);
      kids.push_back(end_round(nc, ns, last));
    } else if (checked) {
      kids.push_back(end_round(c, s, last));
    } else {
      kids.push_back(decision(o, c, s, false, raises, true, last));
    }
    const bool grow = allin_to > c[o] + kEps;
    std::vector<double> targets;
    // bet sizes: one list, or the acting player's list for the situation
    // (opening, after a check, facing a bet, one raise, more raises)
    const int sit = facing ? 2 + std::min(raises, 2) : (checked ? 1 : 0);
    const std::vector<double>& sizes = in.has_menu ? in.menu[p][sit] : in.fracs;
    if (grow && (!facing || raises < in.max_raises)) {
      for (double f : sizes) {
        double t = c[o] + f * 2.0 * c[o];
        if (t >= allin_to - kEps) t = allin_to;
        if (!targets.empty() && std::fabs(targets.back() - t) <= kEps) continue;
        targets.push_back(t);
      }
    }
    if (grow && in.allin && (targets.empty() || std::fabs(targets.back() - allin_to) > kEps))
      targets.push_back(allin_to);
    for (double t : targets) {
      double nc[2], ns[2];
      put(std::fabs(t - allin_to) <= kEps ? allin_to : t, nc, ns);
      kids.push_back(decision(o, nc, ns, true, raises + (facing ? 1 : 0), false, last));
    }
    TNode n;
    n.kind = p;
    n.c[0] = c[0]; n.c[1] = c[1]; n.s[0] = s[0]; n.s[1] = s[1];
    n.raises = raises;
    n.facing = facing ? 1 : 0;
    n.kids = std::move(kids);
    return add(std::move(n));
  }

  int round(const double c[2], const double s[2], bool last) {
    return decision(0, c, s, false, 0, false, last);
  }

  int build() {
    double c[2] = {in.contrib, in.contrib};
    double s[2] = {in.stack[0], in.stack[1]};
    int root = round(c, s, !in.two_rounds());
    if (in.two_rounds()) {
      size_t n0 = nodes.size();
      for (size_t i = 0; i < n0 && !overflow; ++i) {
        if (nodes[i].kind != K_CHANCE) continue;
        double cc[2] = {nodes[i].c[0], nodes[i].c[1]};
        double ss[2] = {nodes[i].s[0], nodes[i].s[1]};
        int r = round(cc, ss, true);
        nodes[i].kids.assign(1, r);
      }
    }
    return root;
  }
};

struct SfBuilder {
  const Instance& in;
  const std::vector<TNode>& nodes;
  SeqForm& sf;
  // Betting features of a decision node (inputs of the warm-start network):
  // pot and stacks relative to the pot, the amount to call, raise count,
  // depth, round, and per action slot its kind and the chips it adds.
  void infoset_features(const TNode& n, int p, int depth, int board) {
    const int o = 1 - p;
    const double pot = n.c[0] + n.c[1];
    float f[kInfFeat] = {0};
    f[0] = (float)p;
    f[1] = (float)(pot / (2.0 * in.contrib));
    f[2] = (float)(n.c[p] / pot);
    f[3] = (float)((n.c[o] - n.c[p]) / pot);
    f[4] = (float)(std::min(n.s[p] / pot, 20.0) / 20.0);
    f[5] = (float)(std::min(n.s[o] / pot, 20.0) / 20.0);
    f[6] = (float)n.facing;
    f[7] = (float)n.raises / 4.f;
    f[8] = (float)n.kids.size() / (float)kWarmActions;
    f[9] = (float)depth / 8.f;
    f[10] = board >= 0 ? 1.f : 0.f;
    for (int a = 0; a < (int)n.kids.size() && a < kWarmActions; ++a) {
      const TNode& k = nodes[n.kids[a]];
      float* q = f + 11 + 6 * a;
      q[0] = 1.f;
      if (a == 0 && n.facing) {
        q[1] = 1.f;                                   // fold
      } else if (a == 0 || (a == 1 && n.facing)) {
        q[2] = 1.f;                                   // check / call
      } else {
        q[3] = 1.f;                                   // bet / raise
        if (k.s[p] <= kEps) q[4] = 1.f;               // all-in
      }
      q[5] = (float)((k.c[p] - n.c[p]) / pot);
    }
    sf.inf_feat[p].insert(sf.inf_feat[p].end(), f, f + kInfFeat);
  }

  void visit(int id, int l0, int l1, int board, int depth = 0) {
    const TNode& n = nodes[id];
    if (n.kind == K_LEAF) {
      Terminal t;
      t.seq[0] = l0; t.seq[1] = l1;
      t.kind = n.term;
      t.board = board;
      t.runout = n.runout;
      t.c1 = n.c[0]; t.c2 = n.c[1];
      sf.terms.push_back(t);
      return;
    }
    if (n.kind == K_CHANCE) {
      for (int r = 0; r < (int)in.rivers.size(); ++r) {
        RiverTask rt;
        rt.board = r;
        rt.parent_seq[0] = l0; rt.parent_seq[1] = l1;
        rt.inf_begin[0] = (int)sf.inf[0].size(); rt.inf_begin[1] = (int)sf.inf[1].size();
        visit(n.kids[0], l0, l1, r, depth + 1);
        rt.inf_end[0] = (int)sf.inf[0].size(); rt.inf_end[1] = (int)sf.inf[1].size();
        sf.rivers.push_back(rt);
      }
      return;
    }
    const int p = n.kind;
    const int first = sf.n_seq[p];
    const int na = (int)n.kids.size();
    sf.inf[p].push_back(Infoset{p == 0 ? l0 : l1, first, na, board});
    infoset_features(n, p, depth, board);
    sf.n_seq[p] += na;
    for (int a = 0; a < na; ++a)
      visit(n.kids[a], p == 0 ? first + a : l0, p == 1 ? first + a : l1, board, depth + 1);
  }
};

}  // namespace

void build_seqform(const Instance& in, SeqForm& sf) {
  TreeBuilder tb(in);
  int root = tb.build();
  sf = SeqForm();
  if (tb.overflow) {
    sf.n_seq[0] = sf.n_seq[1] = -1;
    return;
  }
  SfBuilder sb{in, tb.nodes, sf};
  sb.visit(root, -1, -1, -1);
}

// ---------------------------------------------------------------------------
// hand metadata
// ---------------------------------------------------------------------------
void build_hand_meta(Built& b) {
  const Instance& in = b.inst;
  // beta = sum of mu1 mu2 over pairs sharing no card, by inclusion-exclusion
  // over cards (eq. cf: the all-pairs product minus the collision term).
  double tot[2] = {0, 0};
  std::vector<double> mc[2];
  for (int p = 0; p < 2; ++p) {
    mc[p].assign(in.deck, 0.0);
    for (int h = 0; h < in.n[p]; ++h) {
      tot[p] += in.mu[p][h];
      for (int k = 0; k < in.cph; ++k) mc[p][in.cards[p][(size_t)h * in.cph + k]] += in.mu[p][h];
    }
  }
  double collide = 0;
  for (int c = 0; c < in.deck; ++c) collide += mc[0][c] * mc[1][c];
  double same = 0;
  std::vector<int> idx1((size_t)kMaxDeck * kMaxDeck, -1);
  for (int h = 0; h < in.n[1]; ++h) idx1[hand_key(&in.cards[1][(size_t)h * in.cph], in.cph)] = h;
  std::vector<int> twin0(in.n[0], -1), twin1(in.n[1], -1);
  for (int h = 0; h < in.n[0]; ++h) {
    int j = idx1[hand_key(&in.cards[0][(size_t)h * in.cph], in.cph)];
    if (j >= 0) {
      twin0[h] = j;
      twin1[j] = h;
      same += in.mu[0][h] * in.mu[1][j];
    }
  }
  b.beta = tot[0] * tot[1] - collide + (in.cph == 2 ? same : 0.0);
  const double rs = b.beta > 0 ? 1.0 / std::sqrt(b.beta) : 0.0;
  for (int p = 0; p < 2; ++p) {
    b.lam[p].resize(in.n[p]);
    for (int h = 0; h < in.n[p]; ++h) b.lam[p][h] = in.mu[p][h] * rs;
  }
  b.n_ctx = in.two_rounds() ? 1 + (int)in.rivers.size() : 1;
  for (int p = 0; p < 2; ++p) b.ctx[p].assign(b.n_ctx, CtxMeta());

  // per-card sorted strengths of each scan side (for the query positions)
  std::vector<std::vector<std::vector<int32_t>>> card_str(2);
  std::vector<std::vector<int32_t>> card_start(2);
  auto key_of = [&](int p, int ctx, int h) -> int32_t {
    if (in.two_rounds()) return ctx == 0 ? 0 : in.strength[p][(size_t)(ctx - 1) * in.n[p] + h];
    return in.strength[p][h];
  };
  auto live_in = [&](int p, int ctx, int h) {
    return ctx == 0 || !holds(in, p, h, in.rivers[ctx - 1]);
  };
  for (int ctx = 0; ctx < b.n_ctx; ++ctx) {
    for (int p = 0; p < 2; ++p) {
      CtxMeta& m = b.ctx[p][ctx];
      const int n = in.n[p];
      std::vector<int> order;
      order.reserve(n);
      for (int h = 0; h < n; ++h)
        if (live_in(p, ctx, h)) order.push_back(h);
      std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        int32_t ka = key_of(p, ctx, a), kc = key_of(p, ctx, c);
        return ka < kc || (ka == kc && a < c);
      });
      m.n_live = (int)order.size();
      m.rank.assign(n, -1);
      m.sorted_strength.resize(order.size());
      for (int i = 0; i < (int)order.size(); ++i) {
        m.rank[order[i]] = i;
        m.sorted_strength[i] = key_of(p, ctx, order[i]);
      }
      m.seg_src.clear();
      m.seg_end.assign(1 + in.deck, 0);
      for (int i = 0; i < m.n_live; ++i) m.seg_src.push_back(i);
      m.seg_end[0] = (int)m.seg_src.size();
      m.seg_src.push_back(-1);
      card_str[p].assign(in.deck, {});
      card_start[p].assign(in.deck, 0);
      for (int c = 0; c < in.deck; ++c) {
        card_start[p][c] = (int)m.seg_src.size();
        for (int i = 0; i < m.n_live; ++i) {
          if (holds(in, p, order[i], c)) {
            m.seg_src.push_back(i);
            card_str[p][c].push_back(m.sorted_strength[i]);
          }
        }
        m.seg_end[1 + c] = (int)m.seg_src.size();
        m.seg_src.push_back(-1 - (1 + c));
      }
    }
    // queries of p against the opponent's scan side
    for (int p = 0; p < 2; ++p) {
      const int q = 1 - p;
      CtxMeta& m = b.ctx[p][ctx];
      const CtxMeta& o = b.ctx[q][ctx];
      m.q.assign(in.n[p], QueryRec{});
      for (int h = 0; h < in.n[p]; ++h) {
        QueryRec r{};
        if (!live_in(p, ctx, h)) {
          r.lt = -1;
          r.le = -1;
          r.cards = 255 | (255 << 8);
          r.self = -1;
          m.q[h] = r;
          continue;
        }
        const int32_t s = key_of(p, ctx, h);
        const auto& gs = o.sorted_strength;
        r.lt = (int32_t)(std::lower_bound(gs.begin(), gs.end(), s) - gs.begin());
        r.le = (int32_t)(std::upper_bound(gs.begin(), gs.end(), s) - gs.begin());
        int32_t lts[2] = {0, 0}, les[2] = {0, 0};
        int cs[2] = {255, 255};
        for (int k = 0; k < in.cph; ++k) {
          int c = in.cards[p][(size_t)h * in.cph + k];
          const auto& v = card_str[q][c];
          cs[k] = c;
          lts[k] = card_start[q][c] + (int32_t)(std::lower_bound(v.begin(), v.end(), s) - v.begin());
          les[k] = card_start[q][c] + (int32_t)(std::upper_bound(v.begin(), v.end(), s) - v.begin());
        }
        r.lt0 = lts[0]; r.le0 = les[0]; r.lt1 = lts[1]; r.le1 = les[1];
        r.cards = cs[0] | (cs[1] << 8);
        int tw = p == 0 ? twin0[h] : twin1[h];
        r.self = tw >= 0 ? o.rank[tw] : -1;
        m.q[h] = r;
      }
    }
  }
  // Range features of each hand on the first board context (warm-start
  // inputs): belief weight relative to the mean, strength quantile, share of
  // the opponent's range it blocks, and the compatible opponent mass it beats
  // and loses to (prefix sums over the sorted opponent list with per-card
  // inclusion-exclusion, the hand operators of eq. cf and Technique B).
  for (int p = 0; p < 2; ++p) {
    const int q = 1 - p;
    const CtxMeta& own = b.ctx[p][0];
    const CtxMeta& opp = b.ctx[q][0];
    std::vector<double> pre(opp.seg_src.size() + 1, 0.0);   // exclusive prefix of mu_q per entry
    {
      std::vector<int> order(opp.n_live);
      for (int h = 0; h < in.n[q]; ++h)
        if (opp.rank[h] >= 0) order[opp.rank[h]] = h;
      double run = 0.0;
      for (size_t e = 0; e < opp.seg_src.size(); ++e) {
        pre[e] = run;
        int sidx = opp.seg_src[e];
        if (sidx >= 0) run += in.mu[q][order[sidx]];
        else run = 0.0;
      }
    }
    const double T = pre[opp.seg_end[0]];
    double meanp = 0;
    for (int h = 0; h < in.n[p]; ++h) meanp += in.mu[p][h];
    meanp = meanp > 0 ? meanp / in.n[p] : 1.0;
    b.hand_feat[p].assign((size_t)in.n[p] * kHandFeat, 0.f);
    for (int h = 0; h < in.n[p]; ++h) {
      float* f = &b.hand_feat[p][(size_t)h * kHandFeat];
      f[0] = (float)(std::min(in.mu[p][h] / meanp, 8.0) / 8.0);
      const QueryRec& r = own.q[h];
      if (r.lt < 0 || !(T > 0)) continue;
      f[1] = own.n_live > 1 ? (float)own.rank[h] / (float)(own.n_live - 1) : 0.5f;
      double blocked = 0, weaker = pre[r.lt], stronger = T - pre[r.le];
      for (int k = 0; k < in.cph; ++k) {
        const int c = in.cards[p][(size_t)h * in.cph + k];
        const double tc = pre[opp.seg_end[1 + c]];
        blocked += tc;
        weaker -= pre[k == 0 ? r.lt0 : r.lt1];
        stronger -= tc - pre[k == 0 ? r.le0 : r.le1];
      }
      const int tw = p == 0 ? twin0[h] : twin1[h];
      if (in.cph == 2 && tw >= 0) blocked -= in.mu[q][tw];
      const double compat = T - blocked;
      f[2] = (float)(blocked / T);
      if (compat > 0) {
        f[3] = (float)(weaker / compat);
        f[4] = (float)(stronger / compat);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
// One output row per workgroup while rows are few (latency: every row in
// flight at once); more rows per workgroup once the grid has several
// workgroups per compute unit, so context metadata is loaded once per chunk.
int default_rows_per_block(int64_t rows, int kernel) {
  if (rows <= 2048) return 1;
  return kernel == 3 ? 8 : 2;
}

// The FP64 products (the gap) run the chunk-aligned layout: 512-thread
// workgroups (fewer entries per thread, shorter serial passes) when instances
// hold many hands on average, 256-thread workgroups for batches of smaller
// instances.  The FP32 products default to the grouped kernel (4), one group
// per workgroup.
int default_mv_kernel(int64_t mean_hands) { return mean_hands > 800 ? 3 : 2; }

namespace {

struct Contrib {
  int ctx;
  bool fold;
  int in_seq;
  double coef;
};

}  // namespace

void build_matvec_plan(HostGame& hg, int d, int rows_per_block) {
  const int p = d, q = 1 - d;
  MvDir& D = hg.dir[d];
  D = MvDir();
  D.blk.push_back(0);
  for (size_t ii = 0; ii < hg.inst.size(); ++ii) {
    const Built& b = hg.inst[ii];
    const Instance& in = b.inst;
    // contexts of this instance
    const int ctx_base = (int)D.ctx.size();
    for (int c = 0; c < b.n_ctx; ++c) {
      const CtxMeta& own = b.ctx[p][c];
      const CtxMeta& opp = b.ctx[q][c];
      MvCtx m{};
      m.n_own = in.n[p];
      m.n_opp = in.n[q];
      m.n_live = opp.n_live;
      m.n_ent = (int)opp.seg_src.size();
      m.n_seg = 1 + in.deck;
      m.cph = in.cph;
      m.stride_own = b.stride[p];
      m.q_off = (int64_t)D.q.size();
      for (const QueryRec& r : own.q) {
        auto lohi = [](int32_t lo, int32_t hi) {
          return (uint32_t)(uint16_t)(int16_t)lo | ((uint32_t)(uint16_t)(int16_t)hi << 16);
        };
        QueryRec16 k;
        k.x = lohi(r.lt, r.le);
        k.y = lohi(r.lt0, r.le0);
        k.z = lohi(r.lt1, r.le1);
        k.w = (uint32_t)(r.cards & 0xffff) | ((uint32_t)(uint16_t)(int16_t)r.self << 16);
        D.q.push_back(k);
      }
      m.rank_off = (int64_t)D.rank.size();
      for (int32_t v : opp.rank) D.rank.push_back((int16_t)v);
      m.seg_off = (int64_t)D.seg.size();
      for (int32_t v : opp.seg_src) D.seg.push_back((int16_t)v);
      // pad each context's entry list to a multiple of 8 (aligned vector loads)
      while (D.seg.size() % 8) D.seg.push_back(0);
      while (D.rank.size() % 8) D.rank.push_back(-1);
      m.segend_off = (int64_t)D.segend.size();
      D.segend.insert(D.segend.end(), opp.seg_end.begin(), opp.seg_end.end());
      m.lam_own_off = -1;   // filled by the ABI layer (lambda arrays are per player)
      m.lam_opp_off = -1;
      D.max_ent = std::max(D.max_ent, m.n_ent);
      D.max_seg = std::max(D.max_seg, m.n_seg);
      D.max_n = std::max(D.max_n, std::max(m.n_own, m.n_opp));
      D.ctx.push_back(m);
    }
    // contributions per own sequence
    const int S = b.sf.n_seq[p];
    std::vector<std::vector<Contrib>> rows(S);
    const double rem = in.two_rounds() ? (double)in.remaining() : 1.0;
    for (const Terminal& t : b.sf.terms) {
      const int sg = t.seq[p], other = t.seq[q];
      if (t.kind != PMX_SHOWDOWN) {
        const double u1 = t.kind == PMX_FOLD_P1 ? -t.c1 : t.c2;
        if (t.board < 0) rows[sg].push_back({0, true, other, u1});
        else rows[sg].push_back({1 + t.board, true, other, u1 / rem});
      } else {
        const double st = (d == 0 ? 1.0 : -1.0) * t.c1;
        if (t.runout) {
          for (int r = 0; r < (int)in.rivers.size(); ++r) rows[sg].push_back({1 + r, false, other, st / rem});
        } else if (t.board < 0) {
          rows[sg].push_back({0, false, other, st});
        } else {
          rows[sg].push_back({1 + t.board, false, other, st / rem});
        }
      }
    }
    const int64_t out_base = b.vec_off[p], in_base = b.vec_off[q];
    const int64_t sp = b.stride[p], sq = b.stride[q];
    // the items of contributions cl[c0, c1) (sorted by context) of row sg,
    // written to element offset `out` of the output (last = 1) or of the
    // partial buffer (last = 2)
    auto emit_items = [&](int sg, size_t c0, size_t c1, int64_t out, int last) {
      // group this row's contributions by context; pair a fold and a showdown input per item
      const std::vector<Contrib>& cl = rows[sg];
      size_t i = c0;
      const size_t first_item = D.items.size();
      while (i < c1) {
        size_t j = i;
        std::vector<const Contrib*> fs, ss;
        while (j < c1 && cl[j].ctx == cl[i].ctx) {
          (cl[j].fold ? fs : ss).push_back(&cl[j]);
          ++j;
        }
        size_t k = std::max(fs.size(), ss.size());
        for (size_t t = 0; t < k; ++t) {
          MvItem it{};
          it.out = out;
          it.n_own = in.n[p];
          it.stride = b.stride[p];
          it.ctx = ctx_base + cl[i].ctx;
          it.in_f = t < fs.size() ? in_base + fs[t]->in_seq * sq : -1;
          it.kf = t < fs.size() ? fs[t]->coef : 0.0;
          it.in_s = t < ss.size() ? in_base + ss[t]->in_seq * sq : -1;
          it.ks = t < ss.size() ? ss[t]->coef : 0.0;
          it.last = 0;
          D.items.push_back(it);
        }
        i = j;
      }
      if (D.items.size() == first_item) {
        MvItem it{};
        it.out = out_base + sg * sp;
        it.n_own = in.n[p];
        it.stride = b.stride[p];
        it.ctx = -1;
        it.in_f = it.in_s = -1;
        D.items.push_back(it);
      }
      D.items.back().last = last;
    };
    auto emit_row = [&](int sg) {
      std::vector<Contrib>& cl = rows[sg];
      std::stable_sort(cl.begin(), cl.end(), [](const Contrib& a, const Contrib& c) { return a.ctx < c.ctx; });
      emit_items(sg, 0, cl.size(), out_base + sg * sp, 1);
    };
    auto n_ctx_of = [&](int sg) {
      int prev = -2, cnt = 0;
      std::vector<int> cs;
      for (auto& c : rows[sg]) cs.push_back(c.ctx);
      std::sort(cs.begin(), cs.end());
      for (int c : cs)
        if (c != prev) { ++cnt; prev = c; }
      return cnt;
    };
    // single-context rows grouped by context, then multi-context rows, then empty rows
    std::vector<std::vector<int>> by_ctx(b.n_ctx);
    std::vector<int> multi, empty;
    for (int sg = 0; sg < S; ++sg) {
      int nc = n_ctx_of(sg);
      if (nc == 0) empty.push_back(sg);
      else if (nc == 1) by_ctx[rows[sg][0].ctx].push_back(sg);
      else multi.push_back(sg);
    }
    for (int c = 0; c < b.n_ctx; ++c) {
      int cnt = 0;
      for (int sg : by_ctx[c]) {
        emit_row(sg);
        if (++cnt == rows_per_block) {
          { D.blk.push_back((int32_t)D.items.size()); D.blk_inst.push_back((int32_t)ii); }
          cnt = 0;
        }
      }
      if (cnt) { D.blk.push_back((int32_t)D.items.size()); D.blk_inst.push_back((int32_t)ii); }
    }
    // a row over more contexts than a chunk's rows: parts of about that many
    // contexts, each a chunk writing a partial row (one workgroup would
    // otherwise walk every context in turn, the product's longest chain)
    const int per_part = std::max(1, rows_per_block);
    for (int sg : multi) {
      std::vector<Contrib>& cl = rows[sg];
      std::stable_sort(cl.begin(), cl.end(), [](const Contrib& a, const Contrib& c) { return a.ctx < c.ctx; });
      std::vector<size_t> cut{0};   // first contribution of each context
      for (size_t i = 1; i < cl.size(); ++i)
        if (cl[i].ctx != cl[i - 1].ctx) cut.push_back(i);
      const int nc = (int)cut.size();
      cut.push_back(cl.size());
      if (nc <= per_part) {
        emit_items(sg, 0, cl.size(), out_base + sg * sp, 1);
        D.blk.push_back((int32_t)D.items.size());
        D.blk_inst.push_back((int32_t)ii);
        continue;
      }
      const int n_parts = (nc + per_part - 1) / per_part;
      MvRed r{};
      r.out = out_base + sg * sp;
      r.part = D.part_elems;
      r.n_parts = n_parts;
      r.stride = (int32_t)sp;
      r.inst = (int32_t)ii;
      for (int j = 0; j < n_parts; ++j) {
        // contexts [j nc / n_parts, (j + 1) nc / n_parts): parts differ by at most one context
        const int k0 = (int)((int64_t)j * nc / n_parts), k1 = (int)((int64_t)(j + 1) * nc / n_parts);
        emit_items(sg, cut[k0], cut[k1], r.part + (int64_t)j * sp, 2);
        D.blk.push_back((int32_t)D.items.size());
        D.blk_inst.push_back((int32_t)ii);
      }
      D.part_elems += (int64_t)n_parts * sp;
      D.red.push_back(r);
    }
    {
      int cnt = 0;
      for (int sg : empty) {
        emit_row(sg);
        if (++cnt == 4 * rows_per_block) {
          { D.blk.push_back((int32_t)D.items.size()); D.blk_inst.push_back((int32_t)ii); }
          cnt = 0;
        }
      }
      if (cnt) { D.blk.push_back((int32_t)D.items.size()); D.blk_inst.push_back((int32_t)ii); }
    }
  }
  // runs of consecutive items of a chunk that share a context
  for (size_t b = 0; b + 1 < D.blk.size(); ++b) {
    for (int it = D.blk[b + 1] - 1; it >= D.blk[b]; --it) {
      MvItem& m = D.items[it];
      const bool joins = it + 1 < D.blk[b + 1] && m.ctx >= 0 && D.items[it + 1].ctx == m.ctx;
      m.run_end = joins ? D.items[it + 1].run_end : it + 1;
      m.n_opp = m.ctx >= 0 ? D.ctx[m.ctx].n_opp : 0;
    }
  }
}

// Chunk-aligned layout of one direction for workgroups of `block` threads
// (see McCtx): slots of every opponent hand, the own hands' query slots, the
// per-thread chunk descriptors of each context, and the row chunks grouped by
// hands-per-thread class.  Uses the contexts and row chunks of hg.dir[d].
int build_mc_layout(HostGame& hg, int d, int block, std::string& msg) {
  const int p = d, q = 1 - d;
  McDir& M = hg.mc[d];
  M = McDir();
  M.block = block;
  const MvDir& D = hg.dir[d];
  const int kh_max = block == 512 ? 3 : 5;
  std::vector<int> inst_class(hg.inst.size(), 0);
  auto lohi = [](int32_t lo, int32_t hi) {
    return (uint32_t)(uint16_t)(int16_t)lo | ((uint32_t)(uint16_t)(int16_t)hi << 16);
  };
  size_t ci = 0;
  for (size_t ii = 0; ii < hg.inst.size(); ++ii) {
    const Built& b = hg.inst[ii];
    const Instance& in = b.inst;
    const int nmax = std::max(in.n[p], in.n[q]);
    const int kh = std::max(1, (nmax + block - 1) / block);
    if (kh > kh_max) {
      msg = "instance " + std::to_string(ii) + " has too many hands for this matvec schedule";
      return PMX_EINVAL;
    }
    inst_class[ii] = kh - 1;
    const int ke = mc_ke(block, kh), sk = mc_sk(ke);
    for (int c = 0; c < b.n_ctx; ++c, ++ci) {
      const CtxMeta& own = b.ctx[p][c];
      const CtxMeta& opp = b.ctx[q][c];
      const int n_seg = 1 + in.deck;
      // opponent scan side: sorted live hands and, per card, its holders in that order
      std::vector<int> order(opp.n_live);
      for (int h = 0; h < in.n[q]; ++h)
        if (opp.rank[h] >= 0) order[opp.rank[h]] = h;
      std::vector<int> len(n_seg, 0);
      len[0] = opp.n_live;
      std::vector<std::array<int, 2>> idx_in_card(in.n[q], std::array<int, 2>{-1, -1});
      for (int i = 0; i < opp.n_live; ++i) {
        const int h = order[i];
        for (int k = 0; k < in.cph; ++k) {
          const int card = in.cards[q][(size_t)h * in.cph + k];
          idx_in_card[h][k] = len[1 + card]++;
        }
      }
      std::vector<int> cstart(n_seg + 1, 0);
      for (int sg = 0; sg < n_seg; ++sg) cstart[sg + 1] = cstart[sg] + (len[sg] + 1 + ke - 1) / ke;
      const int n_chunk = cstart[n_seg];
      if (n_chunk > block) {
        msg = "instance " + std::to_string(ii) + ": scan entries exceed the workgroup";
        return PMX_EINVAL;
      }
      // byte offset of a slot for 4-byte values (the FP64 kernels double it)
      auto slot = [&](int sg, int i) { return 4 * ((cstart[sg] + i / ke) * sk + i % ke); };
      McCtx m{};
      m.n_own = in.n[p];
      m.n_opp = in.n[q];
      m.cph = in.cph;
      m.n_chunk = n_chunk;
      m.lam_own_off = m.lam_opp_off = -1;   // filled by the ABI layer
      m.pos_off = (int64_t)M.pos.size() / 2;
      for (int h = 0; h < in.n[q]; ++h) {
        if (opp.rank[h] < 0) {
          M.pos.push_back(0xffffffffu);
          M.pos.push_back(0xffffffffu);
          continue;
        }
        int cs[2] = {-1, -1};
        for (int k = 0; k < in.cph; ++k) {
          const int card = in.cards[q][(size_t)h * in.cph + k];
          cs[k] = slot(1 + card, idx_in_card[h][k]);
        }
        M.pos.push_back(lohi(slot(0, opp.rank[h]), cs[0]));
        M.pos.push_back(lohi(cs[1], -1));
      }
      m.meta_off = (int64_t)M.meta.size();
      std::vector<uint32_t> meta(block, 0u);
      for (int sg = 0; sg < n_seg; ++sg) {
        const int nch = cstart[sg + 1] - cstart[sg];
        for (int j = 0; j < nch; ++j) {
          const int nv = std::max(0, std::min(ke, len[sg] - j * ke));
          uint32_t v = (uint32_t)nv;
          if (j == 0) v |= 1u << 8;
          if (j == nch - 1) v |= (uint32_t)(sg + 1) << 16;
          meta[cstart[sg] + j] = v;
        }
      }
      M.meta.insert(M.meta.end(), meta.begin(), meta.end());
      m.q_off = (int64_t)M.q.size();
      for (int h = 0; h < in.n[p]; ++h) {
        const QueryRec& r = own.q[h];
        QueryRec16 k{};
        if (r.lt < 0) {
          k.x = lohi(-1, -1);
          k.w = 255u | (255u << 8) | (0xffffu << 16);
          M.q.push_back(k);
          continue;
        }
        k.x = lohi(slot(0, r.lt), slot(0, r.le));
        int cards[2] = {255, 255};
        uint32_t cw[2] = {0, 0};
        for (int kk = 0; kk < in.cph; ++kk) {
          const int card = in.cards[p][(size_t)h * in.cph + kk];
          const int base_old = opp.seg_end[card] + 1;   // old entry list: segment 1 + card starts here
          const int lt = (kk == 0 ? r.lt0 : r.lt1) - base_old, le = (kk == 0 ? r.le0 : r.le1) - base_old;
          cards[kk] = card;
          cw[kk] = lohi(slot(1 + card, lt), slot(1 + card, le));
        }
        k.y = cw[0];
        k.z = cw[1];
        const int self = r.self >= 0 ? slot(0, r.self) : -1;
        k.w = (uint32_t)cards[0] | ((uint32_t)cards[1] << 8) | ((uint32_t)(uint16_t)(int16_t)self << 16);
        M.q.push_back(k);
      }
      M.ctx.push_back(m);
    }
  }
  const int nch = (int)D.blk.size() - 1;
  for (int bch = 0; bch < nch; ++bch) {
    const int it0 = D.blk[bch], it1 = D.blk[bch + 1], ii = D.blk_inst[bch];
    int ctx = -1;
    for (int it = it0; it < it1 && ctx < 0; ++it) ctx = D.items[it].ctx;
    std::vector<int32_t>& L = M.chunks[inst_class[ii]];
    L.push_back(it0);
    L.push_back(it1);
    L.push_back(ii);
    L.push_back(ctx);
  }
  return PMX_OK;
}

// ---------------------------------------------------------------------------
// grouped matvec layout (kernel 4)
// ---------------------------------------------------------------------------
namespace {

struct GTerm {
  int out;        // own sequence (output row)
  int ctx;        // board context
  bool fold;
  int in;         // opponent sequence (input row)
  double coef;    // payoff x chance probability (sign of the direction included)
};

struct GroupH {   // a group before offsets: rows as sequence ids
  int ctx = -1;
  int in[kGrpComps] = {-1, -1, -1, -1};
  int fc[kGrpComps] = {0, 0, 0, 0};        // component of output o's fold term
  double ks[kGrpComps] = {0, 0, 0, 0}, kf[kGrpComps] = {0, 0, 0, 0};
  bool sd[kGrpComps] = {false, false, false, false}, f[kGrpComps] = {false, false, false, false};
};
using Slots = std::array<int, kGrpComps>;   // output row of each slot, -1: empty

// Places the terms of one context, for outputs in fixed slots, into as many
// groups as they need: a showdown term of the output in slot o takes
// component o, a fold term a component holding its input row or a free one.
// Terms that do not fit wait for the next group.
void place_terms(const Slots& slots, int ctx, std::vector<GTerm> pending, std::vector<GroupH>& res) {
  auto slot_of = [&](int row) {
    for (int o = 0; o < kGrpComps; ++o)
      if (slots[o] == row) return o;
    return -1;
  };
  while (!pending.empty()) {
    GroupH G;
    G.ctx = ctx;
    std::vector<GTerm> next;
    for (const GTerm& t : pending) {
      if (t.fold) continue;
      const int o = slot_of(t.out);
      if (!G.sd[o] && (G.in[o] < 0 || G.in[o] == t.in)) {
        G.in[o] = t.in;
        G.ks[o] = t.coef;
        G.sd[o] = true;
      } else if (G.sd[o] && G.in[o] == t.in) {
        G.ks[o] += t.coef;
      } else {
        next.push_back(t);
      }
    }
    for (const GTerm& t : pending) {
      if (!t.fold) continue;
      const int o = slot_of(t.out);
      if (G.f[o]) {
        if (G.in[G.fc[o]] == t.in) G.kf[o] += t.coef;
        else next.push_back(t);
        continue;
      }
      int pick = -1;
      for (int c = 0; c < kGrpComps && pick < 0; ++c)
        if (G.in[c] == t.in) pick = c;
      for (int c = 0; c < kGrpComps && pick < 0; ++c)
        if (G.in[c] < 0) pick = c;
      if (pick < 0) {
        next.push_back(t);
        continue;
      }
      G.in[pick] = t.in;
      G.fc[o] = pick;
      G.kf[o] = t.coef;
      G.f[o] = true;
    }
    res.push_back(G);
    pending.swap(next);
  }
}

}  // namespace

// Grouped layout of one direction (kernel 4): per instance, the terms of each
// board context are joined into connected sets of output and input rows
// (each output row reads at most one fold and one showdown input per context
// in these games, so the sets are small) and packed into groups of at most
// kGrpComps outputs and components; rows with terms in several contexts (the
// turn's all-in runouts) form sequences of groups over their contexts that
// carry each row's sum; rows without terms are written as zeros.  Groups are
// cut into workgroup chunks of about `gpc` groups at sequence boundaries.
int build_grp_layout(HostGame& hg, int d, int gpc, std::string& msg) {
  const int p = d, q = 1 - d;
  GrpDir& M = hg.grp[d];
  M = GrpDir();
  if (hg.elems[0] >= ((int64_t)1 << 31) || hg.elems[1] >= ((int64_t)1 << 31)) {
    msg = "vectors of 2^31 elements or more: matvec kernel 4 takes 32-bit offsets";
    return PMX_EINVAL;
  }
  const int BLK = kGrpBlock;
  auto lohi = [](uint32_t lo, uint32_t hi) { return (lo & 0xffffu) | ((hi & 0xffffu) << 16); };
  // two-wide launches pay when the product has many groups; a small one (a
  // single river endgame) keeps one launch per class
  int64_t out_rows = 0;
  for (const Built& b : hg.inst) out_rows += b.sf.n_seq[d];
  const bool two_wide = out_rows >= kGrpTwoWideMinRows;
  for (size_t ii = 0; ii < hg.inst.size(); ++ii) {
    const Built& b = hg.inst[ii];
    const Instance& in = b.inst;
    // hands-per-thread class: the smallest whose entry chunks fit every context
    const int nmax = std::max(in.n[p], in.n[q]);
    int cls = std::max(1, (nmax + BLK - 1) / BLK) - 1;
    std::vector<int> len_all;
    auto chunks_needed = [&](int ke) {
      int worst = 0;
      for (int c = 0; c < b.n_ctx; ++c) {
        const CtxMeta& opp = b.ctx[q][c];
        std::vector<int> len(1 + in.deck, 0);
        len[0] = opp.n_live;
        for (int h = 0; h < in.n[q]; ++h)
          if (opp.rank[h] >= 0)
            for (int k = 0; k < in.cph; ++k) ++len[1 + in.cards[q][(size_t)h * in.cph + k]];
        int n = 0;
        for (int l : len) n += (l + 1 + ke - 1) / ke;
        worst = std::max(worst, n);
      }
      return worst;
    };
    while (cls < kGrpClasses && chunks_needed(kGrpKE[cls]) > BLK) ++cls;
    if (cls >= kGrpClasses) {
      msg = "instance " + std::to_string(ii) + " has too many hands for matvec kernel 4";
      return PMX_EINVAL;
    }
    const int KE = kGrpKE[cls];
    const int ctx_base = (int)M.ctx.size();
    for (int c = 0; c < b.n_ctx; ++c) {
      const CtxMeta& own = b.ctx[p][c];
      const CtxMeta& opp = b.ctx[q][c];
      const int n_seg = 1 + in.deck;
      std::vector<int> order(opp.n_live);
      for (int h = 0; h < in.n[q]; ++h)
        if (opp.rank[h] >= 0) order[opp.rank[h]] = h;
      std::vector<std::vector<int>> card_list(in.deck);   // sorted positions of each card's holders
      for (int i = 0; i < opp.n_live; ++i)
        for (int k = 0; k < in.cph; ++k) card_list[in.cards[q][(size_t)order[i] * in.cph + k]].push_back(i);
      std::vector<int> len(n_seg), cstart(n_seg + 1, 0);
      len[0] = opp.n_live;
      for (int cd = 0; cd < in.deck; ++cd) len[1 + cd] = (int)card_list[cd].size();
      for (int sg = 0; sg < n_seg; ++sg) cstart[sg + 1] = cstart[sg] + (len[sg] + 1 + KE - 1) / KE;
      const int n_chunk = cstart[n_seg];
      auto slot = [&](int sg, int i) { return (uint32_t)((i % KE) * BLK + cstart[sg] + i / KE); };
      auto urow = [&](int pos) { return (uint32_t)(16 * grp_urow(pos)); };
      GCtx m{};
      m.n_own = in.n[p];
      m.n_opp = in.n[q];
      m.cph = in.cph;
      m.n_chunk = n_chunk;
      m.zrow = (int32_t)urow(opp.n_live);
      m.trash = m.zrow + 16;
      m.lam_own_off = m.lam_opp_off = -1;   // filled by the ABI layer
      // staging rows of the opponent's hands
      m.rk_off = (int64_t)M.rk.size();
      for (int h = 0; h < in.n[q]; ++h)
        M.rk.push_back((uint16_t)(opp.rank[h] >= 0 ? urow(opp.rank[h]) : (uint32_t)m.trash));
      while (M.rk.size() % 8) M.rk.push_back(0);
      // entry sources and chunk descriptors
      std::vector<uint32_t> ent((size_t)BLK * KE, (uint32_t)m.zrow);
      std::vector<uint32_t> meta(BLK, 0u);
      for (int sg = 0; sg < n_seg; ++sg) {
        const int nch = cstart[sg + 1] - cstart[sg];
        for (int j = 0; j < nch; ++j) {
          const int t = cstart[sg] + j;
          for (int i = 0; i < KE; ++i) {
            const int idx = j * KE + i;
            if (idx < len[sg]) ent[(size_t)t * KE + i] = urow(sg == 0 ? idx : card_list[sg - 1][idx]);
          }
          uint32_t v = 0;
          if (j == 0) v |= 1u << 8;
          if (j == nch - 1) v |= (uint32_t)(sg + 1) << 16;
          meta[t] = v;
        }
      }
      m.src_off = (int64_t)M.src.size();
      for (int j = 0; j < KE / 2; ++j)
        for (int t = 0; t < BLK; ++t)
          M.src.push_back(lohi(ent[(size_t)t * KE + 2 * j], ent[(size_t)t * KE + 2 * j + 1]));
      m.meta_off = (int64_t)M.meta.size();
      M.meta.insert(M.meta.end(), meta.begin(), meta.end());
      // query records of the own hands
      m.q_off = (int64_t)M.q.size() / 4;
      for (int h = 0; h < in.n[p]; ++h) {
        const QueryRec& r = own.q[h];
        if (r.lt < 0) {
          M.q.insert(M.q.end(), {0xffffffffu, 0u, 0u, 0u});
          continue;
        }
        uint32_t cw[2] = {0, 0};
        int cards[2] = {255, 255};
        for (int k = 0; k < in.cph; ++k) {
          const int card = in.cards[p][(size_t)h * in.cph + k];
          const int base_old = opp.seg_end[card] + 1;   // the card's list in the sentinel entry list
          const int lt = (k == 0 ? r.lt0 : r.lt1) - base_old, le = (k == 0 ? r.le0 : r.le1) - base_old;
          cards[k] = card;
          cw[k] = lohi(slot(1 + card, lt), slot(1 + card, le));
        }
        uint32_t w = (uint32_t)cards[0] | ((uint32_t)(in.cph == 2 ? cards[1] : 0) << 6);
        if (r.self >= 0)
          w |= (1u << 12) | ((uint32_t)(r.self % KE == KE - 1) << 13) | (slot(0, r.self) << 14);
        M.q.push_back(lohi(slot(0, r.lt), slot(0, r.le)));
        M.q.push_back(cw[0]);
        M.q.push_back(cw[1]);
        M.q.push_back(w);
      }
      M.ctx.push_back(m);
    }

    // terms of this direction: output = own sequence, input = opponent sequence
    const int S = b.sf.n_seq[p];
    std::vector<GTerm> terms;
    const double rem = in.two_rounds() ? (double)in.remaining() : 1.0;
    for (const Terminal& t : b.sf.terms) {
      const int sg = t.seq[p], other = t.seq[q];
      if (t.kind != PMX_SHOWDOWN) {
        const double u1 = t.kind == PMX_FOLD_P1 ? -t.c1 : t.c2;
        if (t.board < 0) terms.push_back({sg, 0, true, other, u1});
        else terms.push_back({sg, 1 + t.board, true, other, u1 / rem});
      } else {
        const double st = (d == 0 ? 1.0 : -1.0) * t.c1;
        if (t.runout) {
          for (int r = 0; r < (int)in.rivers.size(); ++r) terms.push_back({sg, 1 + r, false, other, st / rem});
        } else if (t.board < 0) {
          terms.push_back({sg, 0, false, other, st});
        } else {
          terms.push_back({sg, 1 + t.board, false, other, st / rem});
        }
      }
    }
    std::vector<std::vector<int>> row_terms(S);
    for (size_t i = 0; i < terms.size(); ++i) row_terms[terms[i].out].push_back((int)i);
    std::vector<int> empty, multi;
    std::vector<std::vector<int>> single(b.n_ctx);
    for (int sg = 0; sg < S; ++sg) {
      std::vector<int> cs;
      for (int i : row_terms[sg]) cs.push_back(terms[i].ctx);
      std::sort(cs.begin(), cs.end());
      cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
      if (cs.empty()) empty.push_back(sg);
      else if (cs.size() == 1) single[cs[0]].push_back(sg);
      else multi.push_back(sg);
    }
    const int64_t out_base = b.vec_off[p], in_base = b.vec_off[q];
    const int64_t sp = b.stride[p], sq = b.stride[q];
    // a sequence of groups over fixed output slots: offsets and carry flags
    std::vector<std::pair<int, int>> seqs;   // group ranges
    auto emit = [&](const Slots& slots, const std::vector<GroupH>& gs) {
      const int g0 = (int)M.groups.size();
      for (size_t k = 0; k < gs.size(); ++k) {
        const GroupH& H = gs[k];
        GGroup G{};
        G.ctx = H.ctx < 0 ? -1 : ctx_base + H.ctx;
        G.n_own = in.n[p];
        G.stride = b.stride[p];
        G.n_in = in.n[q];
        G.fc = 0;
        G.sc = 0xe4;   // output o: showdown component o
        G.acc = 0;
        for (int o = 0; o < kGrpComps; ++o) {
          G.in[o] = H.in[o] >= 0 ? (int32_t)(in_base + H.in[o] * sq) : -1;
          G.out[o] = slots[o] >= 0 ? (int32_t)(out_base + slots[o] * sp) : -1;
          G.ks[o] = H.ks[o];
          G.kf[o] = H.kf[o];
          G.fc |= (H.fc[o] & 3) << (2 * o);
          if (slots[o] >= 0) {
            if (k == 0) G.acc |= 1 << o;
            if (k + 1 == gs.size()) G.acc |= 1 << (4 + o);
          }
        }
        M.groups.push_back(G);
      }
      seqs.push_back({g0, (int)M.groups.size()});
    };
    // the groups of a set of rows over their contexts, for a slot assignment
    auto place_slots = [&](const Slots& slots, const std::vector<int>& tids) {
      std::vector<int> cs;
      for (int i : tids) cs.push_back(terms[i].ctx);
      std::sort(cs.begin(), cs.end());
      cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
      std::vector<GroupH> gs;
      for (int c : cs) {
        std::vector<GTerm> tl;
        for (int i : tids)
          if (terms[i].ctx == c) tl.push_back(terms[i]);
        place_terms(slots, c, tl, gs);
      }
      return gs;
    };
    // rows in slot order
    auto place_all = [&](const std::vector<int>& outs, const std::vector<int>& tids, Slots* used) {
      Slots sl = {-1, -1, -1, -1};
      for (size_t k = 0; k < outs.size(); ++k) sl[k] = outs[k];
      if (used) *used = sl;
      return place_slots(sl, tids);
    };
    // single-context rows: connected sets of rows (through shared input
    // rows) packed into groups while they fit in one
    for (int c = 0; c < b.n_ctx; ++c) {
      const std::vector<int>& rows = single[c];
      if (rows.empty()) continue;
      std::vector<int> parent(rows.size());
      std::iota(parent.begin(), parent.end(), 0);
      std::function<int(int)> find = [&](int a) { return parent[a] == a ? a : parent[a] = find(parent[a]); };
      std::vector<int> first_user(b.sf.n_seq[q], -1);
      for (size_t k = 0; k < rows.size(); ++k)
        for (int i : row_terms[rows[k]]) {
          int& fu = first_user[terms[i].in];
          if (fu < 0) fu = (int)k;
          else parent[find((int)k)] = find(fu);
        }
      std::vector<std::vector<int>> comps;
      std::vector<int> comp_of(rows.size(), -1);
      for (size_t k = 0; k < rows.size(); ++k) {
        const int r = find((int)k);
        if (comp_of[r] < 0) {
          comp_of[r] = (int)comps.size();
          comps.push_back({});
        }
        comps[comp_of[r]].push_back((int)k);
      }
      // first fit, larger sets first, into groups that stay one group
      std::stable_sort(comps.begin(), comps.end(),
                       [](const std::vector<int>& x, const std::vector<int>& y) { return x.size() > y.size(); });
      std::vector<std::pair<std::vector<int>, std::vector<int>>> open;   // (outputs, terms)
      for (const auto& cm : comps) {
        std::vector<int> co, ct;
        for (int k : cm) {
          co.push_back(rows[k]);
          for (int i : row_terms[rows[k]]) ct.push_back(i);
        }
        // best fit: the open group left with the fewest free output and component slots
        int best = -1, best_free = 1 << 30;
        for (size_t oi = 0; oi < open.size(); ++oi) {
          auto& os = open[oi];
          if (os.first.size() + co.size() > (size_t)kGrpComps) continue;
          std::vector<int> o2 = os.first, t2 = os.second;
          o2.insert(o2.end(), co.begin(), co.end());
          t2.insert(t2.end(), ct.begin(), ct.end());
          const std::vector<GroupH> gs = place_all(o2, t2, nullptr);
          if (gs.size() != 1) continue;
          int used = 0;
          for (int j = 0; j < kGrpComps; ++j) used += gs[0].in[j] >= 0;
          const int free_slots = (kGrpComps - (int)o2.size()) + (kGrpComps - used);
          if (free_slots < best_free) {
            best_free = free_slots;
            best = (int)oi;
          }
        }
        if (best >= 0) {
          open[best].first.insert(open[best].first.end(), co.begin(), co.end());
          open[best].second.insert(open[best].second.end(), ct.begin(), ct.end());
          continue;
        }
        if (co.size() <= (size_t)kGrpComps && place_all(co, ct, nullptr).size() == 1) {
          open.push_back({co, ct});
          continue;
        }
        // a set that needs several groups: slices of kGrpComps rows, each its own sequence
        for (size_t a2 = 0; a2 < cm.size(); a2 += kGrpComps) {
          std::vector<int> o2, t2;
          for (size_t k = a2; k < std::min(cm.size(), a2 + kGrpComps); ++k) {
            o2.push_back(rows[cm[k]]);
            for (int i : row_terms[rows[cm[k]]]) t2.push_back(i);
          }
          Slots sl;
          std::vector<GroupH> gs = place_all(o2, t2, &sl);
          emit(sl, gs);
        }
      }
      for (auto& os : open) {
        Slots sl;
        std::vector<GroupH> gs = place_all(os.first, os.second, &sl);
        emit(sl, gs);
      }
    }
    // rows over several contexts: kGrpComps at a time, context by context
    for (size_t a = 0; a < multi.size(); a += kGrpComps) {
      std::vector<int> outs, tids;
      for (size_t k = a; k < std::min(multi.size(), a + kGrpComps); ++k) {
        outs.push_back(multi[k]);
        for (int i : row_terms[multi[k]]) tids.push_back(i);
      }
      Slots sl;
      std::vector<GroupH> gs = place_all(outs, tids, &sl);
      emit(sl, gs);
    }
    // rows without terms
    for (size_t a = 0; a < empty.size(); a += kGrpComps) {
      Slots sl = {-1, -1, -1, -1};
      for (size_t k = a; k < std::min(empty.size(), a + kGrpComps); ++k) sl[k - a] = empty[k];
      emit(sl, {GroupH()});
    }
    // workgroup chunks: about gpc groups, cut at sequence boundaries.  A
    // single group that reads at most two input rows (often four outputs,
    // each a fold or a showdown term of one of two rows) runs two-wide: its
    // components move to 0 and 1 and each output names the component of its
    // showdown term (sc) as it names that of its fold term (fc)
    auto narrow = [&](int gi) {
      const GGroup& G = M.groups[gi];
      if (!two_wide || G.ctx < 0) return false;
      int used = 0;
      for (int j = 0; j < kGrpComps; ++j) used += G.in[j] >= 0;
      return used <= 2;
    };
    auto compact = [&](int gi) {
      GGroup& G = M.groups[gi];
      int to[kGrpComps] = {0, 0, 0, 0}, in2[kGrpComps] = {-1, -1, -1, -1}, n = 0;
      for (int j = 0; j < kGrpComps; ++j)
        if (G.in[j] >= 0) {
          to[j] = n;
          in2[n++] = G.in[j];
        }
      int fc = 0, sc = 0;
      for (int o = 0; o < kGrpComps; ++o) {
        const int fj = (G.fc >> (2 * o)) & 3;
        fc |= (G.in[fj] >= 0 ? to[fj] : 0) << (2 * o);
        sc |= (G.in[o] >= 0 ? to[o] : 0) << (2 * o);   // no row there: no showdown term (ks = 0)
      }
      for (int j = 0; j < kGrpComps; ++j) G.in[j] = in2[j];
      G.fc = fc;
      G.sc = sc;
    };
    // a single group of more components whose showdown terms read at most
    // two of them: those move to 0 and 1 (the only ones given prefix slots),
    // the fold-only ones to 2 and 3
    auto sd_comps = [&](int gi) {
      const GGroup& G = M.groups[gi];
      int m = 0;
      for (int o = 0; o < kGrpComps; ++o)
        if (G.out[o] >= 0 && G.ks[o] != 0.0) m |= 1 << o;   // a plain group's output o: showdown on component o
      return m;
    };
    auto split = [&](int gi) {
      if (!two_wide || M.groups[gi].ctx < 0) return false;
      return __builtin_popcount(sd_comps(gi)) <= 2;
    };
    auto split_order = [&](int gi) {
      const int m = sd_comps(gi);
      GGroup& G = M.groups[gi];
      int to[kGrpComps], in2[kGrpComps], n = 0;
      for (int pass = 0; pass < 2; ++pass)
        for (int j = 0; j < kGrpComps; ++j)
          if (((m >> j) & 1) == (pass == 0 ? 1 : 0)) {
            to[j] = n;
            in2[n++] = G.in[j];
          }
      int fc = 0, sc = 0;
      for (int o = 0; o < kGrpComps; ++o) {
        fc |= to[(G.fc >> (2 * o)) & 3] << (2 * o);
        sc |= (((m >> o) & 1) ? to[o] : 0) << (2 * o);   // no showdown term: ks = 0
      }
      for (int j = 0; j < kGrpComps; ++j) G.in[j] = in2[j];
      G.fc = fc;
      G.sc = sc;
    };
    // with two-wide launches, a single group whose showdown terms read more
    // than two components gives the outputs of all but two of them to a new
    // group (each output's value comes from one group either way), so that
    // both are two-wide or split and no four-wide launch is left
    if (two_wide) {
      const size_t n_seq_before = seqs.size();
      for (size_t q = 0; q < n_seq_before; ++q) {
        if (seqs[q].second - seqs[q].first != 1) continue;
        const int gi = seqs[q].first;
        const int m = sd_comps(gi);
        if (M.groups[gi].ctx < 0 || __builtin_popcount(m) <= 2) continue;
        GGroup G = M.groups[gi], H = M.groups[gi];
        int kept = 0;
        for (int o = 0; o < kGrpComps; ++o) {
          if (G.out[o] < 0) continue;
          const bool move = ((m >> o) & 1) && kept++ >= 2;
          GGroup& drop = move ? G : H;     // the group that loses output o
          drop.out[o] = -1;
          drop.ks[o] = drop.kf[o] = 0.0;
          drop.acc &= ~((1 << o) | (1 << (4 + o)));
        }
        for (GGroup* X : {&G, &H})
          for (int j = 0; j < kGrpComps; ++j) {
            bool used = false;
            for (int o = 0; o < kGrpComps; ++o)
              if (X->out[o] >= 0 && ((o == j && X->ks[o] != 0.0) || (((X->fc >> (2 * o)) & 3) == j && X->kf[o] != 0.0)))
                used = true;
            if (!used) X->in[j] = -1;
          }
        M.groups[gi] = G;
        M.groups.push_back(H);
        seqs.push_back({(int)M.groups.size() - 1, (int)M.groups.size()});
      }
    }
    auto kind_of = [&](const std::pair<int, int>& sq) {
      if (sq.second - sq.first > 1) return 1;
      return narrow(sq.first) ? 2 : split(sq.first) ? 3 : 0;
    };
    for (const auto& sq : seqs) {
      const int kd = kind_of(sq);
      if (kd == 2) compact(sq.first);
      else if (kd == 3) split_order(sq.first);
    }
    size_t k = 0;
    while (k < seqs.size()) {
      const int g0 = seqs[k].first;
      int g1 = seqs[k].second;
      const int kind = kind_of(seqs[k]);
      ++k;
      // rows without terms take chunks of their own (a separate path of the
      // kernel), and every chunk holds sequences of one kind
      while (k < seqs.size() && seqs[k].second - g0 <= gpc &&
             (M.groups[seqs[k].first].ctx < 0) == (M.groups[g0].ctx < 0) && kind_of(seqs[k]) == kind) {
        g1 = seqs[k].second;
        ++k;
      }
      std::vector<int32_t>& L = M.chunks[kind][cls];
      L.push_back(g0);
      L.push_back(g1);
      L.push_back((int32_t)ii);
      L.push_back(M.groups[g0].ctx);
    }
    int mc = 0;
    for (int c = 0; c < b.n_ctx; ++c) mc = std::max(mc, M.ctx[ctx_base + c].n_chunk);
    M.max_chunk[cls] = std::max(M.max_chunk[cls], mc);
  }
  return PMX_OK;
}


// Cut one player's treeplex of every instance into regret-update pieces of
// at most `cap` rows.  Repeatedly: take the maximal infoset subtrees of the
// remaining treeplex that have at most `cap` rows, pack consecutive ones
// (depth-first order) into pieces, and remove them; once what remains fits,
// it becomes the last piece.  Pieces made earlier hang below pieces made
// later, so the bottom-up pass runs them in creation order and the top-down
// pass in reverse; `depth` groups pieces that can run in one launch.
int build_rm_plan(HostGame& hg, int p, int cap, std::string& msg) {
  RmPlan& P = hg.rm[p];
  P = RmPlan();
  if (cap < 1 || cap > (hg.rm_whole ? kTaskRowsWhole : kTaskRowsMax)) {
    msg = "task_rows must be in [1, " + std::to_string(kTaskRowsMax) + "]";
    return PMX_EINVAL;
  }
  std::vector<int32_t> depth_of;        // per task
  for (size_t ii = 0; ii < hg.inst.size(); ++ii) {
    const Built& b = hg.inst[ii];
    const std::vector<Infoset>& inf = b.sf.inf[p];
    const int ni = (int)inf.size(), S = b.sf.n_seq[p];
    P.stage_stride = std::max(P.stage_stride, b.stride[p]);
    std::vector<int> owner(S, -1);
    for (int i = 0; i < ni; ++i) {
      if (inf[i].nact > cap) {
        msg = "an infoset has more actions than task_rows";
        return PMX_EINVAL;
      }
      for (int a = 0; a < inf[i].nact; ++a) owner[inf[i].first + a] = i;
    }
    std::vector<std::vector<int>> kids(S);   // child infosets of each sequence
    for (int i = 0; i < ni; ++i)
      if (inf[i].parent >= 0) kids[inf[i].parent].push_back(i);
    std::vector<char> alive(ni, 1);
    std::vector<int> rows(ni, 0), nis(ni, 0);   // alive subtree rows and infosets
    std::vector<std::vector<int32_t>> pending(S);   // stage rows waiting for the piece holding seq
    const int first_task = (int)P.tasks.size();
    int64_t total_inf = 0;
    auto count_rows = [&]() {
      int64_t total = 0;
      total_inf = 0;
      for (int i = ni - 1; i >= 0; --i) {
        if (!alive[i]) continue;
        int r = inf[i].nact, c = 1;
        for (int a = 0; a < inf[i].nact; ++a)
          for (int j : kids[inf[i].first + a])
            if (alive[j]) {
              r += rows[j];
              c += nis[j];
            }
        rows[i] = r;
        nis[i] = c;
        if (inf[i].parent < 0) {
          total += r;
          total_inf += c;
        }
      }
      return total;
    };
    auto fits = [&](int i) { return rows[i] <= cap && nis[i] <= kTaskInfMax; };
    // emit one piece from a list of infosets (depth-first order)
    auto emit = [&](std::vector<int>& members) {
      std::sort(members.begin(), members.end());
      RmTask t{};
      t.vec_base = b.vec_off[p];
      t.stride = b.stride[p];
      t.n_hands = b.inst.n[p];
      t.inst = (int32_t)ii;
      t.depth = 0;
      std::vector<int32_t> seqs;
      for (int i : members)
        for (int a = 0; a < inf[i].nact; ++a) seqs.push_back(inf[i].first + a);
      std::sort(seqs.begin(), seqs.end());
      auto local = [&](int s) {
        auto it = std::lower_bound(seqs.begin(), seqs.end(), s);
        return (it != seqs.end() && *it == s) ? (int)(it - seqs.begin()) : -1;
      };
      t.rows_off = (int32_t)P.rows.size();
      t.n_rows = (int32_t)seqs.size();
      P.rows.insert(P.rows.end(), seqs.begin(), seqs.end());
      t.row0 = (!seqs.empty() && seqs.back() - seqs.front() + 1 == (int)seqs.size()) ? seqs.front() : -1;
      std::vector<int32_t> ext;
      t.inf_off = (int32_t)P.infs.size();
      const int nm = (int)members.size();
      t.n_inf = (int32_t)nm;
      std::vector<int> par_of(nm), pinf(nm, -1);   // parent code; member index of the parent infoset
      for (int m = 0; m < nm; ++m) {
        const int i = members[m];
        int par;
        if (inf[i].parent < 0) {
          par = -1;
        } else if (local(inf[i].parent) >= 0) {
          par = local(inf[i].parent);
          pinf[m] = (int)(std::lower_bound(members.begin(), members.end(), owner[inf[i].parent]) - members.begin());
        } else {
          auto it = std::find(ext.begin(), ext.end(), inf[i].parent);
          int k = (int)(it - ext.begin());
          if (it == ext.end()) ext.push_back(inf[i].parent);
          par = -2 - k;
        }
        par_of[m] = par;
      }
      // Split the piece for the kRmGroups wavefronts of a block: up to that
      // many groups of whole subtrees (largest first onto the least loaded
      // wavefront)
      // walked concurrently, and the top part above them walked by wavefront
      // 0.  A group root's value goes to its wavefront's accumulator slot j
      // (one per distinct parent target); wavefront 0 adds the slots into
      // their targets in a fixed order before walking the top part.
      std::vector<int> rows_t(nm, 0);
      for (int m = nm - 1; m >= 0; --m) {
        rows_t[m] += inf[members[m]].nact;
        if (pinf[m] >= 0) rows_t[pinf[m]] += rows_t[m];
      }
      int total_rows = 0;
      for (int m = 0; m < nm; ++m)
        if (pinf[m] < 0) total_rows += rows_t[m];
      std::vector<int> group(nm, -1), root_slot(nm, -1);
      std::vector<std::vector<int>> gtargets(kRmGroups);
      int n_groups = 0;
      if (nm >= 8 && total_rows >= 16) {
        const int target = std::max(4, (total_rows + kRmGroups - 1) / kRmGroups);
        std::vector<int> cand;
        for (int m = 0; m < nm; ++m)
          if (rows_t[m] <= target && (pinf[m] < 0 || rows_t[pinf[m]] > target)) cand.push_back(m);
        std::stable_sort(cand.begin(), cand.end(), [&](int a, int c) { return rows_t[a] > rows_t[c]; });
        int load[kRmGroups] = {};
        for (int m : cand) {
          int w = 0;
          for (int q2 = 1; q2 < kRmGroups; ++q2)
            if (load[q2] < load[w]) w = q2;
          auto& tg = gtargets[w];
          auto it = std::find(tg.begin(), tg.end(), par_of[m]);
          if (it == tg.end()) {
            if ((int)tg.size() >= kRmGroupSlots) continue;   // stays in the top part
            tg.push_back(par_of[m]);
            it = tg.end() - 1;
          }
          root_slot[m] = (int)(it - tg.begin());
          load[w] += rows_t[m];
          group[m] = w;
        }
        // members below a group root belong to its group (depth-first order:
        // parents come first)
        for (int m = 0; m < nm; ++m)
          if (group[m] < 0 && pinf[m] >= 0 && group[pinf[m]] >= 0) group[m] = group[pinf[m]];
        for (int w = 0; w < kRmGroups; ++w)
          if (load[w] > 0) ++n_groups;
        if (n_groups < 2) {
          std::fill(group.begin(), group.end(), -1);
          std::fill(root_slot.begin(), root_slot.end(), -1);
          for (auto& tg : gtargets) tg.clear();
          n_groups = 0;
        }
      }
      std::vector<int> order;
      int gb[kRmGroups + 1];
      for (int w = 0; w < kRmGroups; ++w) {
        gb[w] = (int)order.size();
        for (int m = 0; m < nm; ++m)
          if (group[m] == w) order.push_back(m);
      }
      gb[kRmGroups] = (int)order.size();
      for (int m = 0; m < nm; ++m)
        if (group[m] < 0) order.push_back(m);
      // parent code -> LDS row (root sink / root weight, external parent,
      // local row)
      auto lds_row = [](int par) {
        return par == -1 ? kRmRowOne : (par <= -2 ? kRmRowExt + (-2 - par) : kRmRowLocal + par);
      };
      for (int m : order) {
        const int i = members[m];
        const int f = local(inf[i].first);
        const int down = lds_row(par_of[m]);
        const int up = root_slot[m] >= 0 ? kRmRowSlot + kRmGroupSlots * group[m] + root_slot[m] : down;
        P.infs.push_back((int32_t)((uint32_t)f | ((uint32_t)inf[i].nact << 8) | ((uint32_t)up << 16) |
                                   ((uint32_t)down << 24)));
      }
      t.grp_off = -1;
      if (n_groups > 0) {
        t.grp_off = (int32_t)P.grp.size();
        std::vector<int32_t> G(64, 0);
        G[0] = kRmGroups;
        std::vector<std::pair<int, int>> merge;   // (target row, slot row)
        for (int w = 0; w < kRmGroups; ++w) {
          G[kRmGBeg + w] = gb[w];
          G[kRmGEnd + w] = gb[w + 1];
          G[kRmGCnt + w] = (int)gtargets[w].size();
          for (size_t j = 0; j < gtargets[w].size(); ++j)
            merge.emplace_back(lds_row(gtargets[w][j]), kRmRowSlot + kRmGroupSlots * w + (int)j);
        }
        while ((int)merge.size() < kRmMergeMax) merge.emplace_back(kRmRowOne, kRmRowOne);
        std::stable_sort(merge.begin(), merge.end(),
                         [](const std::pair<int, int>& a, const std::pair<int, int>& c) { return a.first < c.first; });
        for (int e = 0; e < kRmMergeMax; ++e)
          G[kRmGMrg + e / 2] |= (merge[e].second | (merge[e].first << 8)) << (16 * (e & 1));
        G[kRmGTop] = gb[kRmGroups];
        G[kRmGTop + 1] = nm;
        P.grp.insert(P.grp.end(), G.begin(), G.end());
      }
      t.ext_off = (int32_t)P.ext_seq.size();
      t.n_ext = (int32_t)ext.size();
      for (int e : ext) {
        P.ext_seq.push_back(e);
        P.ext_slot.push_back(P.n_slot);
        pending[e].push_back(P.n_slot);
        ++P.n_slot;
      }
      // pulls: a header of per-wavefront counts, then each wavefront's pulls
      // (rows r with r % kRmGroups == w, the rows that wavefront loads), in
      // row order, so a row's pulls are consecutive
      t.pull_off = (int32_t)P.pulls.size();
      std::vector<std::vector<int32_t>> by_wave(kRmGroups);
      for (int r = 0; r < (int)seqs.size(); ++r) {
        for (int32_t slot : pending[seqs[r]])
          by_wave[r % kRmGroups].push_back((int32_t)((uint32_t)r | ((uint32_t)slot << 8)));
        pending[seqs[r]].clear();
      }
      size_t n_pulls = 0;
      for (const auto& v : by_wave) n_pulls += v.size();
      if (n_pulls > 0) {
        for (const auto& v : by_wave) P.pulls.push_back((int32_t)v.size());
        for (const auto& v : by_wave) P.pulls.insert(P.pulls.end(), v.begin(), v.end());
      }
      t.n_pull = (int32_t)P.pulls.size() - t.pull_off;
      for (int i : members) alive[i] = 0;
      P.tasks.push_back(t);
    };
    int64_t total = count_rows();
    while (total > cap || total_inf > kTaskInfMax) {
      // maximal subtrees that fit, in depth-first order
      std::vector<int> roots;
      for (int i = 0; i < ni; ++i) {
        if (!alive[i] || !fits(i)) continue;
        const int par = inf[i].parent;
        if (par < 0 || !fits(owner[par])) roots.push_back(i);
      }
      if (roots.empty()) {
        msg = "treeplex cannot be cut into pieces of task_rows";
        return PMX_EINVAL;
      }
      std::vector<int> members, exts;
      int r_sum = 0, n_sum = 0;
      auto collect = [&](int root, std::vector<int>& out) {
        std::vector<int> st{root};
        while (!st.empty()) {
          int i = st.back();
          st.pop_back();
          out.push_back(i);
          for (int a = 0; a < inf[i].nact; ++a)
            for (int j : kids[inf[i].first + a])
              if (alive[j]) st.push_back(j);
        }
      };
      for (int i : roots) {
        const int par = inf[i].parent;
        const bool new_ext = par >= 0 && std::find(exts.begin(), exts.end(), par) == exts.end();
        if (!members.empty() && (r_sum + rows[i] > cap || n_sum + nis[i] > kTaskInfMax ||
                                 (new_ext && (int)exts.size() >= kTaskExtMax))) {
          emit(members);
          members.clear();
          exts.clear();
          r_sum = n_sum = 0;
        }
        collect(i, members);
        r_sum += rows[i];
        n_sum += nis[i];
        if (par >= 0 && std::find(exts.begin(), exts.end(), par) == exts.end()) exts.push_back(par);
      }
      if (!members.empty()) emit(members);
      total = count_rows();
    }
    if (total > 0) {
      std::vector<int> members;
      for (int i = 0; i < ni; ++i)
        if (alive[i]) members.push_back(i);
      emit(members);
    }
    // depth: pieces with no external parent run in the fused launch (0);
    // the others sit one below the deepest piece holding a parent sequence
    std::vector<int> task_of_seq(S, -1);
    for (int t = first_task; t < (int)P.tasks.size(); ++t)
      for (int r = 0; r < P.tasks[t].n_rows; ++r) task_of_seq[P.rows[P.tasks[t].rows_off + r]] = t;
    for (int t = (int)P.tasks.size() - 1; t >= first_task; --t) {
      RmTask& T = P.tasks[t];
      int d = 0;
      for (int k = 0; k < T.n_ext; ++k) d = std::max(d, 1 + P.tasks[task_of_seq[P.ext_seq[T.ext_off + k]]].depth);
      T.depth = d;
    }
    for (int s = 0; s < S; ++s)
      if (!pending[s].empty()) {
        msg = "internal: a stage row has no receiving piece";
        return PMX_EINVAL;
      }
  }
  int max_depth = 0;
  for (const RmTask& t : P.tasks) max_depth = std::max(max_depth, (int)t.depth);
  P.by_depth.assign(max_depth + 1, {});
  for (int t = 0; t < (int)P.tasks.size(); ++t) {
    const RmTask& T = P.tasks[t];
    P.by_depth[T.depth].push_back(t);
    const int k = T.depth == 0 ? 0 : 1;
    P.max_rows[k] = std::max(P.max_rows[k], (int)T.n_rows);
    P.max_ext[k] = std::max(P.max_ext[k], (int)T.n_ext);
  }
  return PMX_OK;
}

namespace {

void build_treeplex_plan(HostGame& hg, int p) {
  TpPlan& T = hg.tp[p];
  T = TpPlan();
  int64_t hand_base = 0;
  for (size_t ii = 0; ii < hg.inst.size(); ++ii) {
    const Built& b = hg.inst[ii];
    const int base = (int)T.inf_parent.size();
    for (const Infoset& I : b.sf.inf[p]) {
      T.inf_parent.push_back(I.parent);
      T.inf_first.push_back(I.first);
      T.inf_nact.push_back(I.nact);
    }
    T.stage_stride = std::max(T.stage_stride, b.stride[p]);
    auto new_task = [&]() {
      TpTask t{};
      t.vec_base = b.vec_off[p];
      t.stride = b.stride[p];
      t.n_hands = b.inst.n[p];
      t.inf_begin = (int)T.order.size();
      t.stage = -1;
      t.pull_begin = t.pull_end = (int)T.pulls.size();
      t.inst = (int)ii;
      t.hand_base = (int32_t)hand_base;
      t.ext_parent = -1;
      t.seq_begin = t.seq_end = -1;
      return t;
    };
    auto seq_range = [&](TpTask& t) {
      int lo = 1 << 30, hi = -1, cnt = 0;
      for (int k = t.inf_begin; k < t.inf_end; ++k) {
        int I = T.order[k] - base;
        lo = std::min(lo, b.sf.inf[p][I].first);
        hi = std::max(hi, b.sf.inf[p][I].first + b.sf.inf[p][I].nact);
        cnt += b.sf.inf[p][I].nact;
      }
      if (hi >= 0 && cnt == hi - lo) {
        t.seq_begin = lo;
        t.seq_end = hi;
      }
    };
    if (b.sf.rivers.empty()) {
      TpTask t = new_task();
      for (int i = 0; i < (int)b.sf.inf[p].size(); ++i) T.order.push_back(base + i);
      t.inf_end = (int)T.order.size();
      seq_range(t);
      T.single.push_back((int)T.tasks.size());
      T.tasks.push_back(t);
    } else {
      // deep tasks: one per (chance node, river card) subtree
      std::vector<TpPull> pulls;
      for (const RiverTask& rt : b.sf.rivers) {
        TpTask t = new_task();
        for (int i = rt.inf_begin[p]; i < rt.inf_end[p]; ++i) T.order.push_back(base + i);
        t.inf_end = (int)T.order.size();
        seq_range(t);
        t.stage = T.n_stage++;
        t.ext_parent = rt.parent_seq[p];
        pulls.push_back(TpPull{rt.parent_seq[p], t.stage});
        T.deep.push_back((int)T.tasks.size());
        T.tasks.push_back(t);
      }
      TpTask top = new_task();
      for (int i = 0; i < (int)b.sf.inf[p].size(); ++i)
        if (b.sf.inf[p][i].board < 0) T.order.push_back(base + i);
      top.inf_end = (int)T.order.size();
      top.pull_begin = (int)T.pulls.size();
      T.pulls.insert(T.pulls.end(), pulls.begin(), pulls.end());
      top.pull_end = (int)T.pulls.size();
      T.top.push_back((int)T.tasks.size());
      T.tasks.push_back(top);
    }
    hand_base += b.inst.n[p];
  }
  T.hands_total = hand_base;
}

}  // namespace

int build_game(const GameDesc* descs, int n, HostGame& hg, std::string& msg) {
  if (!descs || n < 1) {
    msg = "need at least one descriptor";
    return PMX_EINVAL;
  }
  hg = HostGame();
  hg.inst.resize(n);
  int64_t off[2] = {0, 0};
  for (int i = 0; i < n; ++i) {
    Built& b = hg.inst[i];
    std::string m;
    int rc = validate(descs[i], b.inst, m);
    if (rc) {
      msg = "instance " + std::to_string(i) + ": " + m;
      return rc;
    }
    build_seqform(b.inst, b.sf);
    if (b.sf.n_seq[0] < 0) {
      msg = "instance " + std::to_string(i) + ": betting tree too large";
      return PMX_EINVAL;
    }
    for (const Terminal& t : b.sf.terms) {
      if (t.seq[0] < 0 || t.seq[1] < 0) {
        msg = "instance " + std::to_string(i) + ": a terminal is reached before both players act";
        return PMX_EINVAL;
      }
    }
    build_hand_meta(b);
    if (!(b.beta > 0) || !std::isfinite(b.beta)) {
      msg = "instance " + std::to_string(i) + ": ranges give no compatible deal (beta = 0)";
      return PMX_EINVAL;
    }
    for (int p = 0; p < 2; ++p) {
      b.stride[p] = (b.inst.n[p] + 3) & ~3;
      b.vec_off[p] = off[p];
      off[p] += (int64_t)b.sf.n_seq[p] * b.stride[p];
      hg.max_stride = std::max(hg.max_stride, b.stride[p]);
      for (const Infoset& I : b.sf.inf[p]) {
        b.inf_parent[p].push_back(I.parent);
        b.inf_first[p].push_back(I.first);
        b.inf_nact[p].push_back(I.nact);
        b.inf_board[p].push_back(I.board);
      }
    }
    for (const Terminal& t : b.sf.terms) {
      b.t_seq1.push_back(t.seq[0]);
      b.t_seq2.push_back(t.seq[1]);
      b.t_kind.push_back(t.kind);
      b.t_board.push_back(t.board);
      b.t_runout.push_back(t.runout);
      b.t_c1.push_back(t.c1);
      b.t_c2.push_back(t.c2);
    }
  }
  hg.elems[0] = off[0];
  hg.elems[1] = off[1];
  {
    int64_t rows = 0, hands = 0;
    for (auto& b : hg.inst) {
      rows += std::max(b.sf.n_seq[0], b.sf.n_seq[1]);
      hands += std::max(b.inst.n[0], b.inst.n[1]);
    }
    const int mc_kernel = default_mv_kernel(hands / (int64_t)hg.inst.size());
    hg.mv_kernel = 4;
    hg.groups_per_chunk = 1;
    hg.mc_block = mc_kernel == 3 ? 512 : 256;
    hg.rows_per_block = default_rows_per_block(rows, mc_kernel);
  }
  for (int d = 0; d < 2; ++d) {
    build_matvec_plan(hg, d, hg.rows_per_block);
  }
  for (int p = 0; p < 2; ++p) build_treeplex_plan(hg, p);
  // small games: one piece per treeplex when every instance's fits one and
  // the whole update stays a launch of few workgroups
  {
    bool whole = true;
    int64_t blocks = 0;
    for (const Built& b : hg.inst)
      for (int p = 0; p < 2; ++p) {
        if (b.sf.n_seq[p] > kTaskRowsWhole || (int)b.sf.inf[p].size() > kTaskInfMax) whole = false;
        blocks += (b.inst.n[p] + 63) / 64;
      }
    hg.rm_whole = whole && blocks <= hg.rm_quad_max;
  }
  for (int p = 0; p < 2; ++p) {
    int rc = build_rm_plan(hg, p, hg.rm_whole ? kTaskRowsWhole : hg.task_rows, msg);
    if (rc) return rc;
  }
  return PMX_OK;
}

}  // namespace pmx
