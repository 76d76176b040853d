// Host builder under AddressSanitizer and UndefinedBehaviorSanitizer (test
// helper, CPU only, built with g++).  Reads game descriptors from a text file
// (written by the Python test from the seeded instance generators), then runs
// every host-side builder on them: validation, the skeleton and sequence
// form, hand metadata, the matvec row plans, the chunk-aligned layouts for
// 256- and 512-thread workgroups, the grouped layout at two chunk lengths,
// the regret-update pieces at two cuts and, for a single river game,
// Technique B's explicit factors.  Any sanitizer report aborts the run.
//
// File: the number of games, then per game (whitespace separated)
//   deck cph n_board board... n_river rivers... n0 n1
//   cards0[n0*cph] cards1[n1*cph] strength0[nb*n0] strength1[nb*n1]
//   range0[n0] range1[n1] contrib stack0 stack1 n_fracs fracs... max_raises allin
// with nb = max(1, n_river).
#include <cstdio>
#include <fstream>
#include <string>
#include <vector>

#include "pmx_internal.hpp"

using namespace pmx;

namespace {

struct Owned {
  std::vector<uint8_t> board, rivers, cards[2];
  std::vector<int32_t> strength[2];
  std::vector<double> range[2], fracs, menu;
  std::vector<int32_t> menu_len;
  GameDesc d{};
};

template <typename T>
bool read_vec(std::ifstream& in, std::vector<T>& v, size_t n) {
  v.resize(n);
  for (size_t i = 0; i < n; ++i) {
    double x;
    if (!(in >> x)) return false;
    v[i] = (T)x;
  }
  return true;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s descriptors.txt\n", argv[0]);
    return 2;
  }
  std::ifstream in(argv[1]);
  int n = 0;
  if (!(in >> n) || n < 1) return 2;
  std::vector<Owned> own(n);
  std::vector<GameDesc> descs(n);
  for (int k = 0; k < n; ++k) {
    Owned& o = own[k];
    GameDesc& d = o.d;
    int nb = 0, nr = 0;
    in >> d.deck_size >> d.cards_per_hand >> nb;
    if (!read_vec(in, o.board, nb)) return 2;
    in >> nr;
    if (!read_vec(in, o.rivers, nr)) return 2;
    in >> d.n_hands[0] >> d.n_hands[1];
    const size_t rows = nr > 0 ? (size_t)nr : 1;
    for (int p = 0; p < 2; ++p)
      if (!read_vec(in, o.cards[p], (size_t)d.n_hands[p] * d.cards_per_hand)) return 2;
    for (int p = 0; p < 2; ++p)
      if (!read_vec(in, o.strength[p], rows * d.n_hands[p])) return 2;
    for (int p = 0; p < 2; ++p)
      if (!read_vec(in, o.range[p], (size_t)d.n_hands[p])) return 2;
    int nf = 0;
    in >> d.contrib >> d.stack[0] >> d.stack[1] >> nf;
    if (!read_vec(in, o.fracs, nf)) return 2;
    in >> d.max_raises >> d.allow_allin;
    int has_menu = 0;
    in >> has_menu;
    if (!in) return 2;
    if (has_menu) {
      if (!read_vec(in, o.menu_len, 10)) return 2;
      size_t tot = 0;
      for (int32_t l : o.menu_len) tot += (size_t)l;
      if (!read_vec(in, o.menu, tot)) return 2;
      d.bet_menu_len = o.menu_len.data();
      d.bet_menu = o.menu.data();
    }
    d.n_board = nb;
    d.board = o.board.data();
    d.n_river = nr;
    d.river_cards = o.rivers.data();
    for (int p = 0; p < 2; ++p) {
      d.hand_cards[p] = o.cards[p].data();
      d.strength[p] = o.strength[p].data();
      d.range[p] = o.range[p].data();
    }
    d.n_bet_fracs = nf;
    d.bet_fracs = o.fracs.data();
    descs[k] = d;
  }
  HostGame hg;
  std::string msg;
  int rc = build_game(descs.data(), n, hg, msg);
  if (rc) {
    std::fprintf(stderr, "build_game: %s\n", msg.c_str());
    return 1;
  }
  for (int d = 0; d < 2; ++d) {
    for (int block : {256, 512}) {
      std::string m;
      const int r = build_mc_layout(hg, d, block, m);
      if (r && block == 256) {
        std::fprintf(stderr, "build_mc_layout(%d): %s\n", block, m.c_str());
        return 1;
      }
    }
    for (int gpc : {1, 8}) {
      std::string m;
      if (build_grp_layout(hg, d, gpc, m)) {
        std::fprintf(stderr, "build_grp_layout(%d): %s\n", gpc, m.c_str());
        return 1;
      }
    }
  }
  for (int p = 0; p < 2; ++p)
    for (int cap : {13, 64}) {
      std::string m;
      if (build_rm_plan(hg, p, cap, m)) {
        std::fprintf(stderr, "build_rm_plan(%d): %s\n", cap, m.c_str());
        return 1;
      }
    }
  // Technique B's explicit factors of one-instance river games
  long long tb_nnz = -1;
  if (n == 1 && descs[0].n_river == 0) {
    TbHost T;
    std::string m;
    if (build_tb_factors(hg, T, m)) {
      std::fprintf(stderr, "build_tb_factors: %s\n", m.c_str());
      return 1;
    }
    tb_nnz = (long long)(T.nnz_pp[0] + T.nnz_pp[1] + T.nnz_pp[2] + T.nnz_pp[3]);
  }
  std::printf("ok %d games, %lld + %lld elements, %zu + %zu groups, explicit factors %lld\n", n,
              (long long)hg.elems[0], (long long)hg.elems[1], hg.grp[0].groups.size(), hg.grp[1].groups.size(),
              tb_nnz);
  return 0;
}
