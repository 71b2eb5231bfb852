// Host check of the binomial checkpointing schedule (lbm_tape.h): a
// simulated reverse sweep over integer "states" must run the adjoint steps
// N-1 .. 0 in order, each on the right state, use no slot beyond
// binom_slots(N), advance no step more than kBinomRepeats times, and find
// the right-spine states where the forward run stored them.
#include <cstdio>
#include <map>
#include <vector>

#include "../../paper_2003_06342_amd/csrc/lbm_tape.h"

using namespace lbm;

static int check(int64_t n, int64_t& recompute) {
  const int64_t slots = binom_slots(n);
  std::map<int64_t, int64_t> store_at;   // slot -> step index of its state
  store_at[0] = 0;
  binom_spine(n, [&](int64_t step, int64_t slot) { store_at[slot] = step; });
  std::vector<int64_t> order, advanced(n, 0);
  int bad = 0;
  auto adj = [&](int64_t slot, int64_t k) -> bool {
    if (!store_at.count(slot) || slot >= slots) { ++bad; return false; }
    const int64_t x = store_at[slot];
    for (int64_t q = x; q < x + k; ++q) ++advanced[q];
    order.push_back(x + k);
    return true;
  };
  auto store = [&](int64_t slot, int64_t j, int64_t to) -> bool {
    if (!store_at.count(slot) || to >= slots) { ++bad; return false; }
    const int64_t x = store_at[slot];
    for (int64_t q = x; q < x + j; ++q) ++advanced[q];
    store_at[to] = x + j;
    return true;
  };
  if (!binom_reverse(0, n, slots - 1, 0, true, adj, store)) ++bad;
  if ((int64_t)order.size() != n) ++bad;
  for (int64_t i = 0; i < (int64_t)order.size(); ++i)
    if (order[i] != n - 1 - i) ++bad;
  recompute = 0;
  for (int64_t q = 0; q < n; ++q) {
    if (advanced[q] > kBinomRepeats) ++bad;
    recompute += advanced[q];
  }
  return bad;
}

int main() {
  int failures = 0;
  std::vector<int64_t> ns;
  for (int64_t n = 1; n <= 400; ++n) ns.push_back(n);
  for (int64_t n : {1000, 2000, 5000, 20000}) ns.push_back(n);
  for (int64_t n : ns) {
    int64_t rc = 0;
    const int b = check(n, rc);
    if (b) {
      std::printf("n=%lld: %d violations\n", (long long)n, b);
      ++failures;
    }
    if (n == 200 || n == 2000)
      std::printf("n=%lld: %lld slots + 2 work states, %lld recomputed steps (%.2f n)\n", (long long)n,
                  (long long)binom_slots(n), (long long)rc, (double)rc / (double)n);
  }
  // reach is Pascal's rule with reach(0, r) = r + 1 and reach(c, 0) = 1
  for (int64_t c = 1; c < 30; ++c)
    for (int64_t r = 1; r < 10; ++r)
      if (binom_reach(c, r) != binom_reach(c, r - 1) + binom_reach(c - 1, r)) ++failures;
  for (int64_t r = 0; r < 10; ++r)
    if (binom_reach(0, r) != r + 1) ++failures;
  if (binom_slots(2000) != 21 || binom_slots(200) != 9) ++failures;
  std::printf("%d failures\n", failures);
  return failures != 0;
}
