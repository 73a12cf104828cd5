// Queue order from per-system cost estimates (host code, no GPU needed).
//
// The integrator hands out queue positions in order.  When every system has a
// lane from the start, wave w takes positions 64w .. 64w+63, and the waves of
// one round (one wave per SIMD across the chip) share their SIMDs with the
// waves of the next round.  A SIMD's time is then the sum of its waves' chain
// lengths, so the order below deals 64-position chunks, most expensive first,
// over the rounds in alternating direction: a SIMD's first wave gets one of
// the longest chunks and its second wave one of the shortest.  With more
// systems than lanes, the counter hands out positions as lanes free up, and
// the order is simply the most expensive chunks first (longest processing
// time first).  Only the assignment of systems to lanes changes; each system's
// arithmetic, and so its result, does not.
#include "ode_ensemble.h"

#include <algorithm>
#include <cstdint>
#include <limits>
#include <vector>

namespace {
constexpr int64_t kChunk = 64;  // lanes of one wave
}  // namespace

extern "C" int ode_plan_order(const int64_t *cost, const int64_t *queue, int64_t n,
                              int64_t waves, int64_t round_waves, int64_t *out,
                              int64_t capacity, int64_t *n_out) {
  if (!n_out || n < 0 || waves < 1 || round_waves < 1 || (n > 0 && !cost))
    return ODE_EINVAL;
  const bool resident = waves * kChunk >= n;
  const int64_t total = n == 0 ? 0 : (resident ? waves * kChunk : n);
  *n_out = total;
  if (!out) return ODE_OK;
  if (capacity < total) return ODE_EINVAL;
  const int64_t chunks = (n + kChunk - 1) / kChunk;
  std::vector<int64_t> chunk_cost(chunks, std::numeric_limits<int64_t>::min()), order(chunks);
  for (int64_t q = 0; q < n; ++q)
    chunk_cost[q / kChunk] = std::max(chunk_cost[q / kChunk], cost[q]);
  for (int64_t k = 0; k < chunks; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return chunk_cost[a] > chunk_cost[b]; });
  auto copy_chunk = [&](int64_t k, int64_t dst) {
    const int64_t lo = k * kChunk, hi = std::min(n, lo + kChunk);
    for (int64_t q = lo; q < hi; ++q) out[dst + (q - lo)] = queue ? queue[q] : q;
  };
  if (!resident) {
    // chunks back to back (a partial last chunk may land anywhere)
    int64_t dst = 0;
    for (int64_t r = 0; r < chunks; ++r) {
      const int64_t k = order[r];
      copy_chunk(k, dst);
      dst += std::min(n, k * kChunk + kChunk) - k * kChunk;
    }
    return ODE_OK;
  }
  for (int64_t p = 0; p < total; ++p) out[p] = -1;
  for (int64_t r = 0; r < chunks; ++r) {
    const int64_t round = r / round_waves, off = r % round_waves;
    const int64_t size = std::min(round_waves, waves - round * round_waves);
    const int64_t slot = round * round_waves + ((round & 1) ? size - 1 - off : off);
    copy_chunk(order[r], slot * kChunk);
  }
  return ODE_OK;
}
