// Host-logic check of the chunk-aligned matvec layout (test helper, CPU only).
//
// Builds a game with the library's host builder and its chunk-aligned layout
// for one direction and workgroup size, then computes the product the way the
// workgroup kernel does, in FP64 and sequentially: per item, the weighted
// opponent inputs go to their three slots, each chunk's valid entries are
// summed, sums are carried across the chunks of a segment (reset at a
// segment's first chunk), each chunk's exclusive prefix sums are written back,
// the chunk ending a segment records the segment totals, and every own hand
// combines six prefix sums, the card totals and the identical hand.  The caller
// compares the result with the oracle.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "pmx_internal.hpp"

using namespace pmx;

extern "C" int mc_matvec(const GameDesc* d, int n, int block, int dir, const double* in, int64_t in_len,
                         double* out, int64_t out_len, char* msg, int msglen) {
  HostGame hg;
  std::string m;
  int rc = build_game(d, n, hg, m);
  if (!rc) rc = build_mc_layout(hg, dir, block, m);
  if (rc) {
    snprintf(msg, msglen, "%s", m.c_str());
    return rc;
  }
  if (in_len != hg.elems[1 - dir] || out_len != hg.elems[dir]) {
    snprintf(msg, msglen, "vector sizes do not match the layout");
    return 1;
  }
  const MvDir& D = hg.dir[dir];
  const McDir& M = hg.mc[dir];
  // lambdas per context (the device layer fills these offsets from its arrays)
  std::vector<const std::vector<double>*> lam_own, lam_opp;
  for (const Built& b : hg.inst)
    for (int c = 0; c < b.n_ctx; ++c) {
      lam_own.push_back(&b.lam[dir]);
      lam_opp.push_back(&b.lam[1 - dir]);
    }
  for (int64_t i = 0; i < out_len; ++i) out[i] = 0.0;
  std::vector<double> part((size_t)D.part_elems, 0.0);
  for (int cls = 0; cls < kMcClasses; ++cls) {
    const int ke = mc_ke(block, cls + 1), sk = mc_sk(ke), nslot = block * sk;
    const std::vector<int32_t>& L = M.chunks[cls];
    for (size_t c = 0; c + 3 < L.size(); c += 4) {
      const int it0 = L[c], it1 = L[c + 1];
      std::vector<double> acc;
      for (int it = it0; it < it1; ++it) {
        const MvItem& item = D.items[it];
        if (item.ctx < 0) continue;   // the row's output stays 0
        const McCtx& C = M.ctx[item.ctx];
        if ((int)acc.size() != C.n_own) acc.assign(C.n_own, 0.0);
        std::vector<double> S(nslot, 0.0), F(nslot, 0.0);
        auto at = [&](int off4) { return off4 / 4; };
        for (int h = 0; h < C.n_opp; ++h) {
          const uint32_t px = M.pos[2 * (C.pos_off + h)], py = M.pos[2 * (C.pos_off + h) + 1];
          const int g = (int16_t)(px & 0xffff), c0 = (int16_t)(px >> 16), c1 = (int16_t)(py & 0xffff);
          if (g < 0) continue;
          const double w = (*lam_opp[item.ctx])[h];
          const double vs = item.in_s >= 0 ? item.ks * w * in[item.in_s + h] : 0.0;
          const double vf = item.in_f >= 0 ? item.kf * w * in[item.in_f + h] : 0.0;
          for (int sl : {g, c0, c1}) {
            if (sl < 0) continue;
            S[at(sl)] = vs;
            F[at(sl)] = vf;
          }
        }
        std::vector<double> T(2 * kMcSegMax, 0.0);
        double cs = 0.0, cf = 0.0;
        for (int t = 0; t < block; ++t) {
          const uint32_t cm = M.meta[C.meta_off + t];
          const int nv = cm & 255, endseg = (cm >> 16) & 255;
          if (cm & (1u << 8)) cs = cf = 0.0;
          double run = cs;
          for (int j = 0; j < ke; ++j) {
            const double v = j < nv ? S[t * sk + j] : 0.0;
            S[t * sk + j] = run;   // exclusive prefix
            run += v;
          }
          double fs = 0.0;
          for (int j = 0; j < nv; ++j) fs += F[t * sk + j];
          cs = run;
          cf += fs;
          if (endseg) {
            T[2 * (endseg - 1)] = cs;
            T[2 * (endseg - 1) + 1] = cf;
          }
        }
        for (int h = 0; h < C.n_own; ++h) {
          const QueryRec16& r = M.q[C.q_off + h];
          const int lt = (int16_t)(r.x & 0xffff);
          if (lt < 0) continue;
          const int le = (int16_t)(r.x >> 16), lt0 = (int16_t)(r.y & 0xffff), le0 = (int16_t)(r.y >> 16);
          const int lt1 = (int16_t)(r.z & 0xffff), le1 = (int16_t)(r.z >> 16);
          const int c0 = r.w & 255, c1 = (r.w >> 8) & 255, self = (int16_t)(r.w >> 16);
          double sd = S[at(lt)] + S[at(le)] - T[0];
          sd -= S[at(lt0)] + S[at(le0)] - T[2 * (1 + c0)];
          double fo = T[1] - T[2 * (1 + c0) + 1];
          if (C.cph == 2) {
            sd -= S[at(lt1)] + S[at(le1)] - T[2 * (1 + c1)];
            fo -= T[2 * (1 + c1) + 1];
            if (self >= 0) fo += F[at(self)];
          }
          acc[h] += (item.in_s >= 0 ? sd : 0.0) + (item.in_f >= 0 ? fo : 0.0);
        }
        if (item.last) {
          // last = 2: a partial row of a row cut into parts
          double* dst = item.last == 2 ? part.data() : out;
          for (int h = 0; h < C.n_own; ++h) dst[item.out + h] = (*lam_own[item.ctx])[h] * acc[h];
          acc.assign(C.n_own, 0.0);
        }
      }
    }
  }
  // rows cut into parts: the sum of their partial rows in part order
  for (const MvRed& r : D.red)
    for (int h = 0; h < r.stride; ++h) {
      double v = 0.0;
      for (int j = 0; j < r.n_parts; ++j) v += part[(size_t)(r.part + (int64_t)j * r.stride + h)];
      out[r.out + h] = v;
    }
  snprintf(msg, msglen, "ok parts=%d", (int)D.red.size());
  return 0;
}
