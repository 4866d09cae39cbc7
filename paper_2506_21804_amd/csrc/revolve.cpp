// Binomial checkpointing for the reverse sweep (Griewank and Walther,
// "Algorithm 799: revolve", ACM TOMS 26, 2000).  The schedule is built from
// the optimal-cost recursion: to reverse l steps from a stored state with s
// free snapshot slots, advance m steps, store, reverse the last l-m steps with
// s-1 free slots, then the first m with s.  Costs count forward steps.
#include <algorithm>
#include <climits>
#include <vector>

#include "internal.h"

namespace lbmk {

namespace {

struct Table {
  int T, S;
  std::vector<long long> cost;  // [(l) * (S+1) + s]
  std::vector<int> split;
  long long &C(int l, int s) { return cost[(size_t)l * (S + 1) + s]; }
  int &M(int l, int s) { return split[(size_t)l * (S + 1) + s]; }
};

void fill(Table &t) {
  t.cost.assign((size_t)(t.T + 1) * (t.S + 1), 0);
  t.split.assign((size_t)(t.T + 1) * (t.S + 1), 0);
  for (int l = 1; l <= t.T; ++l) {
    t.C(l, 0) = (long long)l * (l - 1) / 2;  // no free slot: recompute each step from the start
    for (int s = 1; s <= t.S; ++s) {
      if (l == 1) {
        t.C(l, s) = 0;
        continue;
      }
      long long best = LLONG_MAX;
      int bm = 1;
      for (int m = 1; m < l; ++m) {
        const long long c = m + t.C(l - m, s - 1) + t.C(m, s);
        if (c < best) {
          best = c;
          bm = m;
        }
      }
      t.C(l, s) = best;
      t.M(l, s) = bm;
    }
  }
}

void emit(Table &t, int a, int b, int s, int slot_a, std::vector<int> &free_slots, std::vector<Action> &out) {
  const int l = b - a;
  if (l == 1) {
    out.push_back({ACT_RESTORE, slot_a, a});
    out.push_back({ACT_REVERSE, a, a});
    return;
  }
  if (s == 0) {
    for (int n = b - 1; n >= a; --n) {
      out.push_back({ACT_RESTORE, slot_a, a});
      if (n > a) out.push_back({ACT_ADVANCE, n - a, a});
      out.push_back({ACT_REVERSE, n, n});
    }
    return;
  }
  const int m = a + t.M(l, s);
  const int slot = free_slots.back();
  free_slots.pop_back();
  out.push_back({ACT_RESTORE, slot_a, a});
  out.push_back({ACT_ADVANCE, m - a, a});
  out.push_back({ACT_STORE, slot, m});
  emit(t, m, b, s - 1, slot, free_slots, out);
  free_slots.push_back(slot);
  emit(t, a, m, s, slot_a, free_slots, out);
}

}  // namespace

// Forward steps of the reverse sweep over T steps with nsnap slots, one of
// which holds the starting state.
long long revolve_cost(int T, int nsnap) {
  if (T < 1 || nsnap < 1) return -1;
  Table t{T, std::min(nsnap - 1, T), {}, {}};
  fill(t);
  return t.C(T, t.S);
}

std::vector<Action> revolve_schedule(int T, int nsnap) {
  std::vector<Action> out;
  if (T < 1 || nsnap < 1) return out;
  Table t{T, std::min(nsnap - 1, T), {}, {}};
  fill(t);
  std::vector<int> free_slots;
  for (int k = nsnap - 1; k >= 1; --k) free_slots.push_back(k);
  emit(t, 0, T, t.S, 0, free_slots, out);
  return out;
}

}  // namespace lbmk
