// Host-logic check of the regret-update pieces (test helper, CPU only).
//
// Builds a game with the library's host builder, cuts each player's treeplex
// into pieces of at most `cap` rows, and plays one regret-matching+ update of
// one hand per instance through the pieces exactly as the launch sequence
// does: bottom-up passes of the deep pieces from the deepest depth up, the
// pieces without external parents (pulls, grouped bottom-up walk, top-down
// walk), then the top-down passes of the deep pieces, with the workgroup's
// LDS rows in the numbering the packed infosets and group tables use.  The result is compared
// with a plain walk over the whole treeplex (children before parents for the
// values, parents before children for the plan).  Also checks that every
// sequence belongs to exactly one piece and that pieces respect the cap.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "pmx_internal.hpp"

using namespace pmx;

namespace {

float rm_plus(float r, float inst) {
  const float v = r + inst;
  return v < 0.f ? 0.f : v;
}

// regret update of one infoset (rows f .. f+n of q and R); returns V(I)
float update_infoset(float* q, float* R, int f, int n) {
  float rs = 0.f;
  for (int a = 0; a < n; ++a) rs += std::max(R[f + a], 0.f);
  float V = 0.f;
  for (int a = 0; a < n; ++a) V += (rs > 0.f ? std::max(R[f + a], 0.f) / rs : 1.f / n) * q[f + a];
  for (int a = 0; a < n; ++a) R[f + a] = rm_plus(R[f + a], q[f + a] - V);
  return V;
}

// behaviour from regrets times the parent's weight, into rows f .. f+n of x
void descend_infoset(float* x, const float* R, int f, int n, float xp) {
  float rs = 0.f;
  for (int a = 0; a < n; ++a) rs += std::max(R[f + a], 0.f);
  for (int a = 0; a < n; ++a) x[f + a] = xp * (rs > 0.f ? std::max(R[f + a], 0.f) / rs : 1.f / n);
}

}  // namespace

extern "C" int check_rm_plan(const GameDesc* d, int n, int cap, char* msg, int msglen, int* n_tasks,
                             int* n_grouped, int* max_depth) {
  HostGame hg;
  std::string m;
  int rc = build_game(d, n, hg, m);
  if (rc) {
    snprintf(msg, msglen, "build: %s", m.c_str());
    return rc;
  }
  for (int p = 0; p < 2; ++p)
    if ((rc = build_rm_plan(hg, p, cap, m))) {
      snprintf(msg, msglen, "plan: %s", m.c_str());
      return rc;
    }
  *n_tasks = *n_grouped = *max_depth = 0;
  std::mt19937 rng(1);
  std::uniform_real_distribution<float> U(0.f, 1.f);
  for (int p = 0; p < 2; ++p) {
    const RmPlan& P = hg.rm[p];
    *n_tasks += (int)P.tasks.size();
    *max_depth = std::max(*max_depth, (int)P.by_depth.size() - 1);
    for (const RmTask& t : P.tasks) *n_grouped += t.grp_off >= 0;
    for (size_t ii = 0; ii < hg.inst.size(); ++ii) {
      const Built& b = hg.inst[ii];
      const int S = b.sf.n_seq[p];
      const std::vector<Infoset>& inf = b.sf.inf[p];
      std::vector<int> count(S, 0);
      for (const RmTask& t : P.tasks) {
        if (t.inst != (int)ii) continue;
        if (t.n_rows > cap) {
          snprintf(msg, msglen, "piece with %d rows above the cap %d", t.n_rows, cap);
          return 1;
        }
        for (int r = 0; r < t.n_rows; ++r) {
          count[P.rows[t.rows_off + r]]++;
          if (t.row0 >= 0 && P.rows[t.rows_off + r] != t.row0 + r) {
            snprintf(msg, msglen, "piece marked contiguous from %d has row %d at %d", t.row0,
                     P.rows[t.rows_off + r], r);
            return 1;
          }
        }
      }
      for (int s = 0; s < S; ++s)
        if (count[s] != 1) {
          snprintf(msg, msglen, "instance %zu player %d: sequence %d in %d pieces", ii, p, s, count[s]);
          return 1;
        }
      // one hand's state
      std::vector<float> g(S), R(S), x(S, 0.f);
      for (int s = 0; s < S; ++s) {
        g[s] = U(rng) - 0.5f;
        R[s] = U(rng) < 0.3f ? 0.f : U(rng);
      }
      // reference: the whole treeplex
      std::vector<float> qr = g, Rr = R, xr(S, 0.f);
      for (int i = (int)inf.size() - 1; i >= 0; --i) {
        const float V = update_infoset(qr.data(), Rr.data(), inf[i].first, inf[i].nact);
        if (inf[i].parent >= 0) qr[inf[i].parent] += V;
      }
      for (const Infoset& I : inf)
        descend_infoset(xr.data(), Rr.data(), I.first, I.nact, I.parent >= 0 ? xr[I.parent] : 1.f);
      // the pieces, in launch order; U models a workgroup's LDS rows (sink /
      // root weight, group-root slots, external parents, the piece's rows)
      std::vector<float> stage(std::max(P.n_slot, 1), 0.f);
      auto run = [&](int mode, int depth) {
        for (int id : P.by_depth[depth]) {
          const RmTask& t = P.tasks[id];
          if (t.inst != (int)ii) continue;
          std::vector<float> U(kRmRowLocal + t.n_rows, 0.f), Rl(t.n_rows);
          float* A = &U[kRmRowLocal];
          for (int r = 0; r < t.n_rows; ++r) {
            const int s = P.rows[t.rows_off + r];
            A[r] = mode == 2 ? 0.f : g[s];
            Rl[r] = R[s];
          }
          auto decode = [&](int i, int& f, int& na, int& up, int& dn) {
            const uint32_t v = (uint32_t)P.infs[t.inf_off + i];
            f = v & 255;
            na = (v >> 8) & 255;
            up = (v >> 16) & 255;
            dn = v >> 24;
          };
          const int* G = t.grp_off >= 0 ? &P.grp[t.grp_off] : nullptr;
          const int tb = G ? G[kRmGTop] : 0, te = G ? G[kRmGTop + 1] : t.n_inf;
          if (mode != 2) {
            if (t.n_pull > 0) {
              // header of per-wavefront counts, then each wavefront's pulls
              // (rows r % kRmGroups == w) in row order, summed per row
              int beg = kRmGroups, total = kRmGroups;
              for (int w = 0; w < kRmGroups; ++w) total += P.pulls[t.pull_off + w];
              if (total != t.n_pull) {
                snprintf(msg, msglen, "pull header counts %d entries for %d", total, t.n_pull);
                throw 1;
              }
              for (int w = 0; w < kRmGroups; ++w) {
                const int cnt = P.pulls[t.pull_off + w];
                float acc = 0.f;
                int row = -1;
                for (int j = 0; j < cnt; ++j) {
                  const int v = P.pulls[t.pull_off + beg + j], lr = v & 255;
                  if (lr % kRmGroups != w || lr < row) {
                    snprintf(msg, msglen, "pull into row %d listed for wavefront %d out of row order", lr, w);
                    throw 1;
                  }
                  if (lr != row) {
                    if (row >= 0) A[row] += acc;
                    acc = 0.f;
                    row = lr;
                  }
                  acc += stage[(uint32_t)v >> 8];
                }
                if (row >= 0) A[row] += acc;
                beg += cnt;
              }
            }
            if (G)
              for (int w = 0; w < kRmGroups; ++w)
                for (int i = G[kRmGEnd + w] - 1; i >= G[kRmGBeg + w]; --i) {
                  int f, na, up, dn;
                  decode(i, f, na, up, dn);
                  const bool own_slot = up >= kRmRowSlot + kRmGroupSlots * w && up < kRmRowSlot + kRmGroupSlots * (w + 1);
                  if (!own_slot && up < kRmRowLocal) {
                    snprintf(msg, msglen, "group %d infoset %d sends its value to LDS row %d", w, i, up);
                    throw 1;
                  }
                  U[up] += update_infoset(A, Rl.data(), f, na);
                }
            if (G) {
              // merge entries: every group slot once plus sink fillers,
              // sorted by target; each entry writes the target's value plus
              // the sum of its run so far
              std::vector<int> slots_seen;
              int prev = -1;
              float run = 0.f;
              std::vector<float> before(U);
              for (int e = 0; e < kRmMergeMax; ++e) {
                const int c = (G[kRmGMrg + e / 2] >> (16 * (e & 1))) & 0xffff, sl = c & 255, tg = c >> 8;
                if (tg < prev) {
                  snprintf(msg, msglen, "merge entries not sorted by target");
                  throw 1;
                }
                if (sl != kRmRowOne) slots_seen.push_back(sl);
                else if (tg != kRmRowOne) {
                  snprintf(msg, msglen, "a filler merge entry targets LDS row %d", tg);
                  throw 1;
                }
                run = (tg == prev ? run : 0.f) + before[sl];
                U[tg] = before[tg] + run;
                prev = tg;
              }
              int n_slots = 0;
              for (int w = 0; w < kRmGroups; ++w) n_slots += G[kRmGCnt + w];
              std::sort(slots_seen.begin(), slots_seen.end());
              if ((int)slots_seen.size() != n_slots ||
                  std::unique(slots_seen.begin(), slots_seen.end()) != slots_seen.end()) {
                snprintf(msg, msglen, "merge entries do not cover the %d group slots once each", n_slots);
                throw 1;
              }
            }
            for (int i = te - 1; i >= tb; --i) {
              int f, na, up, dn;
              decode(i, f, na, up, dn);
              U[up] += update_infoset(A, Rl.data(), f, na);
            }
            if (mode == 1)
              for (int k = 0; k < t.n_ext; ++k) stage[P.ext_slot[t.ext_off + k]] = U[kRmRowExt + k];
            for (int r = 0; r < t.n_rows; ++r) R[P.rows[t.rows_off + r]] = Rl[r];
          }
          if (mode != 1) {
            if (mode == 2)
              for (int k = 0; k < t.n_ext; ++k) U[kRmRowExt + k] = x[P.ext_seq[t.ext_off + k]];
            U[kRmRowOne] = 1.f;
            auto down = [&](int i0, int i1) {
              for (int i = i0; i < i1; ++i) {
                int f, na, up, dn;
                decode(i, f, na, up, dn);
                descend_infoset(A, Rl.data(), f, na, U[dn]);
              }
            };
            down(tb, te);
            if (G) down(0, tb);
            for (int r = 0; r < t.n_rows; ++r) x[P.rows[t.rows_off + r]] = A[r];
          }
        }
      };
      const int D = (int)P.by_depth.size();
      try {
        for (int dd = D - 1; dd >= 1; --dd) run(1, dd);
        run(0, 0);
        for (int dd = 1; dd < D; ++dd) run(2, dd);
      } catch (int) {
        return 1;
      }
      for (int s = 0; s < S; ++s) {
        if (std::fabs(R[s] - Rr[s]) > 1e-4f * (1.f + std::fabs(Rr[s])) || std::fabs(x[s] - xr[s]) > 1e-5f) {
          snprintf(msg, msglen, "instance %zu player %d sequence %d: R %g vs %g, x %g vs %g", ii, p, s, R[s],
                   Rr[s], x[s], xr[s]);
          return 1;
        }
      }
    }
  }
  snprintf(msg, msglen, "ok");
  return 0;
}
