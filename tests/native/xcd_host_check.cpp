// Host-side check of the XCD-aware launch shapes (kernels.hpp):
// * xcd_line_tile<LG> is a bijection of [0, gx) for every grid width, and in
//   every whole group of 8 LG workgroups the LG tiles of one line are taken
//   by workgroups whose linear ids are congruent mod 8 (one XCD) and lie
//   within 8 (LG - 1) of each other (dispatched close together);
// * xcd_pencil_blocks never removes blocks, adds at most an eighth, and
//   returns a multiple of 8 wherever that eighth allows one (>= 56 blocks).
#include <cstdio>
#include <vector>

#include "kernels.hpp"

template <int LG>
static int check_tiles(int gx) {
  int bad = 0;
  std::vector<int> block_of(gx, -1);
  for (int x = 0; x < gx; ++x) {
    const int t = bzq::xcd_line_tile<LG>(x, gx);
    if (t < 0 || t >= gx || block_of[t] != -1) {
      ++bad;
      continue;
    }
    block_of[t] = x;
  }
  const int whole = gx / (8 * LG) * (8 * LG);
  for (int t = 0; t < whole; t += LG)
    for (int j = 1; j < LG; ++j) {
      const int d = block_of[t + j] - block_of[t];
      if (d % 8 != 0 || d < 0 || d > 8 * (LG - 1)) ++bad;
    }
  return bad;
}

int main() {
  int bad = 0;
  for (int gx = 1; gx <= 4096; ++gx) bad += check_tiles<1>(gx) + check_tiles<2>(gx) + check_tiles<4>(gx);
  std::printf("line tiles: %d bad\n", bad);
  int badp = 0;
  for (int gx = 1; gx <= 100000; ++gx) {
    const int gp = bzq::xcd_pencil_blocks(gx);
    if (gp < gx || gp - gx > gx / 8 || (gp != gx && gp % 8 != 0) || (gx >= 56 && gp % 8 != 0)) ++badp;
  }
  std::printf("pencil blocks: %d bad; 63 -> %d, 1009 -> %d, 16 -> %d, 35 -> %d\n", badp,
              bzq::xcd_pencil_blocks(63), bzq::xcd_pencil_blocks(1009), bzq::xcd_pencil_blocks(16),
              bzq::xcd_pencil_blocks(35));
  bad += badp;
  if (bzq::xcd_pencil_blocks(63) != 64 || bzq::xcd_pencil_blocks(1009) != 1016) ++bad;
  std::printf("%s\n", bad ? "FAIL" : "OK");
  return bad ? 1 : 0;
}
