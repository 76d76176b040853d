// Host-logic check of the grouped matvec layout (test helper, CPU only).
//
// Builds a game with the library's host builder and the grouped layout of one
// direction, then computes the product the way the grouped workgroup kernel
// does, in FP64 and sequentially: per group, every opponent hand's weighted
// inputs of the group's components go to its staging row, each thread
// gathers its chunk's entries from the staging rows, chunk sums are carried
// across the chunks of a segment (reset at a segment's first chunk), every
// entry's exclusive prefix sum is stored at its slot, the chunk ending a
// segment records the segment totals, and every own hand combines six prefix
// sums, the card totals and the identical hand (the difference of two
// adjacent prefix sums) into the showdown and fold values of each component,
// weighted per output by the group's coefficients and carried over the
// groups of a sequence.  The caller compares the result with the oracle.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "pmx_internal.hpp"

using namespace pmx;

extern "C" int grp_matvec(const GameDesc* d, int n, int gpc, int dir, const double* in, int64_t in_len,
                          double* out, int64_t out_len, char* msg, int msglen) {
  HostGame hg;
  std::string m;
  int rc = build_game(d, n, hg, m);
  if (!rc) rc = build_grp_layout(hg, dir, gpc, m);
  if (rc) {
    snprintf(msg, msglen, "%s", m.c_str());
    return rc;
  }
  if (in_len != hg.elems[1 - dir] || out_len != hg.elems[dir]) {
    snprintf(msg, msglen, "vector sizes do not match the layout");
    return 1;
  }
  const GrpDir& M = hg.grp[dir];
  const int BLK = kGrpBlock, NC = kGrpComps;
  std::vector<const std::vector<double>*> lam_own, lam_opp;
  for (const Built& b : hg.inst)
    for (int c = 0; c < b.n_ctx; ++c) {
      lam_own.push_back(&b.lam[dir]);
      lam_opp.push_back(&b.lam[1 - dir]);
    }
  for (int64_t i = 0; i < out_len; ++i) out[i] = -7.0;   // every element must be written
  auto fail = [&](const char* what) {
    snprintf(msg, msglen, "%s", what);
    return 2;
  };
  for (int cls = 0; cls < kGrpClasses; ++cls) {
    const int KE = kGrpKE[cls], KH = cls + 1;
    for (int kind = 0; kind < GrpDir::kKinds; ++kind) {
    // bytes of the staging rows: the shared staging / prefix region, or (kind
    // 3, prefix slots for two components only) a region of their own
    const int region = kind == 3 ? 16 * (KH * BLK + KH * BLK / 16 + 2) : 16 * BLK * KE;
    const std::vector<int32_t>& L = M.chunks[kind][cls];
    for (size_t c = 0; c + 3 < L.size(); c += 4) {
      const int g0 = L[c], g1 = L[c + 1];
      std::vector<std::vector<double>> acc(NC);
      for (int gi = g0; gi < g1; ++gi) {
        const GGroup& G = M.groups[gi];
        // two-wide chunks: terms on components 0 and 1 only, one group each
        if (kind == 2) {
          if ((G.acc >> 4 & 0x0f) != (G.acc & 0x0f)) return fail("a two-wide chunk carries sums");
          if (G.ctx < 0 || G.in[2] >= 0 || G.in[3] >= 0) return fail("a two-wide group uses components 2 or 3");
          for (int o = 0; o < NC; ++o)
            if (((G.fc >> (2 * o)) & 3) >= 2 || ((G.sc >> (2 * o)) & 3) >= 2)
              return fail("a two-wide output names component 2 or 3");
        } else if (kind == 3) {
          if ((G.acc >> 4 & 0x0f) != (G.acc & 0x0f)) return fail("a split chunk carries sums");
          if (G.ctx < 0) return fail("a split group has no context");
          for (int o = 0; o < NC; ++o)
            if (G.out[o] >= 0 && G.ks[o] != 0.0 && ((G.sc >> (2 * o)) & 3) >= 2)
              return fail("a split group's showdown term names a component without prefix slots");
        } else if (G.sc != 0xe4) {
          return fail("a four-wide group permutes its showdown components");
        }
        if (G.ctx < 0) {
          for (int o = 0; o < NC; ++o)
            if (G.out[o] >= 0)
              for (int h = 0; h < G.stride; ++h) out[G.out[o] + h] = 0.0;
          continue;
        }
        const GCtx& C = M.ctx[G.ctx];
        if (C.n_own > KH * BLK || C.n_opp > KH * BLK) return fail("hands exceed the class");
        if (C.n_chunk > BLK) return fail("chunks exceed the workgroup");
        // staging rows (byte offset / 16 -> 4 values)
        std::vector<double> U((size_t)region / 16 * NC, 0.0);
        std::vector<char> written((size_t)region / 16, 0);
        for (int h = 0; h < C.n_opp; ++h) {
          const int off = M.rk[C.rk_off + h];
          if (off % 16 || off + 16 > region) return fail("staging row out of the region");
          if (off == C.zrow) return fail("a hand is staged on the zero row");
          if (off != C.trash && written[off / 16]) return fail("two hands share a staging row");
          written[off / 16] = 1;
          for (int j = 0; j < NC; ++j)
            U[(size_t)off / 16 * NC + j] = G.in[j] >= 0 ? (*lam_opp[G.ctx])[h] * in[G.in[j] + h] : 0.0;
        }
        if (C.zrow % 16 || C.zrow + 32 > region) return fail("zero row out of the region");
        for (int j = 0; j < NC; ++j) U[(size_t)C.zrow / 16 * NC + j] = 0.0;
        // gather, carry, prefix sums at their slots, segment totals
        std::vector<double> P((size_t)BLK * KE * NC, 0.0);
        std::vector<double> T(kMcSegMax * NC, 0.0);
        std::vector<double> carry(NC, 0.0);
        for (int t = 0; t < BLK; ++t) {
          const uint32_t cm = M.meta[C.meta_off + t];
          if (cm & (1u << 8)) carry.assign(NC, 0.0);
          std::vector<double> run = carry;
          for (int i = 0; i < KE; ++i) {
            const uint32_t pr = M.src[C.src_off + (int64_t)(i / 2) * BLK + t];
            const int off = (int)((i & 1) ? pr >> 16 : pr & 0xffff);
            if (off % 16 || off + 16 > region) return fail("entry source out of the region");
            const size_t sl = (size_t)i * BLK + t;
            for (int j = 0; j < NC; ++j) {
              P[sl * NC + j] = run[j];
              run[j] += U[(size_t)off / 16 * NC + j];
            }
          }
          carry = run;
          const int endseg = (cm >> 16) & 255;
          if (endseg)
            for (int j = 0; j < NC; ++j) T[(endseg - 1) * NC + j] = carry[j];
        }
        // own hands
        for (int o = 0; o < NC; ++o)
          if (G.acc & (1 << o)) acc[o].assign(G.stride, 0.0);
        for (int h = 0; h < C.n_own; ++h) {
          const uint32_t* r = &M.q[(size_t)(C.q_off + h) * 4];
          if (r[0] == 0xffffffffu) continue;
          const int c0 = r[3] & 63, c1 = (r[3] >> 6) & 63;
          const bool has_self = (r[3] >> 12) & 1, wrap = (r[3] >> 13) & 1;
          const uint32_t s0 = r[3] >> 14;
          auto pf = [&](uint32_t s, int j) {
            return P[(size_t)s * NC + j];
          };
          for (uint32_t w : {r[0], r[1], r[2]})
            if ((w & 0xffff) >= (uint32_t)(BLK * KE) || (w >> 16) >= (uint32_t)(BLK * KE))
              return fail("query slot out of range");
          double sd[NC], fo[NC];
          for (int j = 0; j < NC; ++j) {
            double v = pf(r[0] & 0xffff, j) + pf(r[0] >> 16, j) - T[j];
            v -= pf(r[1] & 0xffff, j) + pf(r[1] >> 16, j) - T[(1 + c0) * NC + j];
            double f = T[j] - T[(1 + c0) * NC + j];
            if (C.cph == 2) {
              v -= pf(r[2] & 0xffff, j) + pf(r[2] >> 16, j) - T[(1 + c1) * NC + j];
              f -= T[(1 + c1) * NC + j];
              if (has_self) {
                const uint32_t s1 = wrap ? s0 - (uint32_t)((KE - 1) * BLK) + 1u : s0 + (uint32_t)BLK;
                if (s0 >= (uint32_t)(BLK * KE) || s1 >= (uint32_t)(BLK * KE)) return fail("self slot out of range");
                if (kind == 3) {
                  // the kernel reads the identical hand from the staging row
                  // of global entry i = (s0 % BLK) * KE + s0 / BLK
                  const int i = (int)(s0 % (uint32_t)BLK) * KE + (int)(s0 / (uint32_t)BLK);
                  const int row = i + (i >> 4);
                  if (16 * row + 16 > region) return fail("identical hand's staging row out of the region");
                  const double u = U[(size_t)row * NC + j];
                  if (std::fabs(u - (pf(s1, j) - pf(s0, j))) > 1e-9 * (1.0 + std::fabs(u)))
                    return fail("the identical hand's staging row is not its global entry");
                  f += u;
                } else {
                  f += pf(s1, j) - pf(s0, j);
                }
              }
            }
            sd[j] = v;
            fo[j] = f;
          }
          for (int o = 0; o < NC; ++o) {
            if (G.out[o] < 0) continue;
            const int fj = (G.fc >> (2 * o)) & 3, sj = (G.sc >> (2 * o)) & 3;
            acc[o][h] += G.ks[o] * sd[sj] + G.kf[o] * fo[fj];
          }
        }
        for (int o = 0; o < NC; ++o) {
          if (G.out[o] < 0 || !(G.acc & (1 << (4 + o)))) continue;
          if (kind == 0 && (G.acc & 0xff) != (((G.acc & 0xf) << 4) | (G.acc & 0xf)))
            return fail("a group of a plain chunk carries a sum");
          for (int h = 0; h < G.stride; ++h)
            out[G.out[o] + h] = h < C.n_own ? (*lam_own[G.ctx])[h] * acc[o][h] : 0.0;
        }
      }
    }
    }
  }
  for (int64_t i = 0; i < out_len; ++i)
    if (out[i] == -7.0) return fail("an output element was never written");
  snprintf(msg, msglen, "ok");
  return 0;
}
