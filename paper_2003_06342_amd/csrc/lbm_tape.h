// Binomial checkpointing schedule of the adjoint's tape (host code).
//
// Griewank and Walther's schedule, written here in recursive form.  To
// reverse the l steps n0 .. n1-1 when the state X^n0 sits in a slot and c
// further slots are free: advance to a split point j, store X^(n0+j) in the
// next slot, reverse the last l - j steps with c - 1 free slots, then the
// first j steps with c.  With no free slot, each state is recomputed from
// X^n0.  binom_reach(c, r) = C(c + r + 1, r) is the longest span reversible
// when no step is advanced more than r times: the first part's steps are
// advanced once more than the second part's, so reach(c, r) = reach(c, r-1)
// + reach(c-1, r), with reach(0, r) = r + 1 and reach(c, 0) = 1.  The split
// j = max(1, l - reach(c-1, r)), for the least r with reach(c, r) >= l,
// keeps both parts within their reach.  The tape holds binom_slots(N)
// checkpoints (slot 0: X^0) and two work states; no step is advanced more
// than kBinomRepeats times in the reverse sweep.
#pragma once
#include <cstdint>

namespace lbm {

constexpr int64_t kBinomRepeats = 3;

inline int64_t binom_reach(int64_t c, int64_t r) {
  double v = 1.0;   // C(c + r + 1, r), saturated far above any step count
  for (int64_t i = 1; i <= r; ++i) {
    v = v * (double)(c + 1 + i) / (double)i;
    if (v > 4e18) return (int64_t)4e18;
  }
  return (int64_t)(v + 0.5);
}

// split of a span of l >= 2 steps with c >= 1 free slots: j in [1, l - 1]
inline int64_t binom_split(int64_t l, int64_t c) {
  int64_t r = 0;
  while (binom_reach(c, r) < l) ++r;
  const int64_t j = l - binom_reach(c - 1, r);
  return j < 1 ? 1 : j;
}

// checkpoint slots for n steps (slot 0 included)
inline int64_t binom_slots(int64_t n) {
  int64_t s = 1;
  while (binom_reach(s - 1, kBinomRepeats) < n) ++s;
  return s;
}

// The states the forward run stores on the way: the split points of the
// reverse sweep's first descent (its right spine), in slots 1, 2, ...
// visit(step, slot) is called in increasing step order.
template <class Visit>
inline void binom_spine(int64_t n, Visit&& visit) {
  const int64_t slots = binom_slots(n);
  int64_t from = 0, slot = 0;
  for (;;) {
    const int64_t l = n - from, cfree = slots - 1 - slot;
    if (l < 2 || cfree < 1) return;
    from += binom_split(l, cfree);
    ++slot;
    visit(from, slot);
  }
}

// Reverse steps n1-1 .. n0 (in that order).  X^n0 is in `slot`; slots
// slot+1 .. slot+cfree are free; on the right spine (spine == true) the split
// states are already stored.  adj(slot, k): run the adjoint of the step whose
// input is X^n0 advanced by k steps; store(slot, j, to): advance X^n0 by j
// steps into slot `to`.  Both return false on failure, which stops the sweep.
template <class Adj, class Store>
inline bool binom_reverse(int64_t n0, int64_t n1, int64_t cfree, int64_t slot, bool spine, Adj& adj,
                          Store& store) {
  const int64_t l = n1 - n0;
  if (l == 1) return adj(slot, 0);
  if (cfree == 0) {
    for (int64_t k = l - 1; k >= 0; --k)
      if (!adj(slot, k)) return false;
    return true;
  }
  const int64_t j = binom_split(l, cfree);
  if (!spine && !store(slot, j, slot + 1)) return false;
  return binom_reverse(n0 + j, n1, cfree - 1, slot + 1, spine, adj, store) &&
         binom_reverse(n0, n0 + j, cfree, slot, false, adj, store);
}

}  // namespace lbm
