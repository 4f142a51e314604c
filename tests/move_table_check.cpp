// Host check of grow's move table (make_moves in kernels.hpp) against the
// brick geometry, for every dimension count: each lane of each quadrant of each
// move must be the lane of a cell whose moved position falls in that quadrant's
// target brick, and the coded shift must carry it to the moved cell's lane
// there.  The moves are decoded from their index independently of the table.
// TEST INFRASTRUCTURE ONLY.
#include <cstdio>
#include <cstdlib>

#include "kernels.hpp"

namespace {

int failures = 0;

template <int N>
void check() {
  using gbees::brick_off;
  using gbees::brick_side;
  constexpr auto t = gbees::make_moves<N>();
  constexpr int kMoves = gbees::MoveTable<N>::kMoves;
  for (int m = 0; m < kMoves; ++m) {
    // The move: offsets d[] of the cell, and the dimensions it changes.
    int d[6] = {0, 0, 0, 0, 0, 0}, ja = -1, jb = -1, pair = -1;
    if (m < 2 * N) {
      ja = m / 2;
      d[ja] = (m % 2) ? 1 : -1;
    } else {
      const int e = m - 2 * N;
      pair = e / 4;
      int p = pair;
      for (int a = 0; a < N; ++a)
        for (int b = a + 1; b < N; ++b)
          if (p-- == 0) ja = a, jb = b;
      d[ja] = (e % 4) / 2 ? 1 : -1;
      d[jb] = (e % 2) ? 1 : -1;
    }
    for (int lane = 0; lane < 64; ++lane) {
      int brick[6] = {0, 0, 0, 0, 0, 0}, dst = 0;
      for (int j = 0; j < N; ++j) {
        const int side = brick_side(N, j);
        const int a = ((lane >> brick_off(N, j)) & (side - 1)) + d[j];
        brick[j] = a < 0 ? -1 : (a >= side ? 1 : 0);
        dst |= ((a + side) % side) << brick_off(N, j);
      }
      const bool leave_a = brick[ja] != 0, leave_b = jb >= 0 && brick[jb] != 0;
      const int qd = (leave_a ? 1 : 0) | (leave_b ? 2 : 0);
      int target = 0;
      if (leave_a && leave_b)
        target = 1 + 2 * N + 4 * pair + 2 * (d[ja] > 0) + (d[jb] > 0);
      else if (leave_a)
        target = 1 + 2 * ja + (d[ja] > 0);
      else if (leave_b)
        target = 1 + 2 * jb + (d[jb] > 0);
      for (int q = 0; q < 4; ++q) {
        const bool in = (t.q[q][m] >> lane) & 1ull;
        if (in != (q == qd)) {
          std::printf("n=%d move %d lane %d: in quadrant %d %d, expected quadrant %d\n", N, m, lane, q, in, qd);
          ++failures;
        }
      }
      const unsigned code = t.sh[qd][m];
      const int moved = lane + static_cast<int>(code & 0xFFu) - static_cast<int>(code >> 8);
      const unsigned tg = (t.tg[m] >> (8 * qd)) & 0xFFu;
      if (moved != dst || tg != static_cast<unsigned>(target)) {
        std::printf("n=%d move %d lane %d: lane %d target %u, expected lane %d target %d\n", N, m, lane, moved, tg, dst,
                    target);
        ++failures;
      }
    }
    const unsigned sa = t.src[m] & 0xFFu, sb = t.src[m] >> 8;
    const unsigned want_a = 2 * ja + (d[ja] > 0), want_b = jb >= 0 ? 2 * jb + (d[jb] > 0) : 0xFFu;
    if (sa != want_a || sb != want_b) {
      std::printf("n=%d move %d: source sets %u %u, expected %u %u\n", N, m, sa, sb, want_a, want_b);
      ++failures;
    }
  }
}

}  // namespace

int main() {
  check<1>();
  check<2>();
  check<3>();
  check<4>();
  check<5>();
  check<6>();
  if (failures) return 1;
  std::printf("move tables ok\n");
  return 0;
}
