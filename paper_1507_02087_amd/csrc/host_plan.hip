// Host-side planning of the square launches; see host_plan.h.
#include "host_plan.h"

#include <algorithm>

namespace sp2 {

// Row stride of an instance's iterate buffers for padded dimension np: np,
// plus 128 elements when np is a multiple of 512 of at least 2048, so that
// the rows of a tile do not all start at one offset modulo the memory
// channel interleave (at N = 8192 this made the BF16x3 square 2 % faster;
// a 16-element pad, which breaks the 128-byte alignment of bf16 rows, was
// 7 % slower).
int64_t row_stride(int64_t np) {
  return (np >= 2048 && np % 512 == 0) ? np + 128 : np;
}

// Upper-triangle tiles (I <= J) of an nt x nt tile grid, ordered by groups of
// G x G neighbouring tiles so that consecutive list entries share row panels.
void append_tile_list(int nt, std::vector<int2>& out) {
  const int G = 4;
  for (int gi = 0; gi < nt; gi += G)
    for (int gj = gi; gj < nt; gj += G)
      for (int i = gi; i < gi + G && i < nt; ++i)
        for (int j = gj; j < gj + G && j < nt; ++j)
          if (i <= j) out.push_back(make_int2(i, j));
}

// Given the group's tiles (global slots, owning instance, K slices of each),
// splits the tiles of an incomplete last round of workgroups into K pieces
// and deals the work to the 8 XCDs: workgroup b runs on XCD b mod 8, so XCD x
// receives a contiguous chunk of the (neighbour-grouped) tile list followed
// by a chunk of the pieces, which keeps the panels its tiles share in its
// own L2. Pieces are numbered from 0 within the group.
Plan make_plan(const std::vector<int>& slots, const std::vector<int>& owner,
               const std::vector<int>& nk, int concurrency, int tail_split) {
  Plan pl;
  const int ntiles = static_cast<int>(slots.size());
  const int rounds = ntiles / concurrency;
  const int rem = ntiles % concurrency;
  int min_nk = 1 << 30;
  for (int k : nk) min_nk = std::min(min_nk, k);
  int split = 1;
  if (tail_split >= 2) {
    split = tail_split;
  } else if (tail_split == 0 && rem > 0 && 2 * rem <= concurrency) {
    split = std::min({concurrency / rem, min_nk / 2, 16});
  }
  split = std::max(1, std::min(split, min_nk));
  const int ntail = (split > 1) ? (rounds > 0 ? rem : ntiles) : 0;
  const int nfull = ntiles - ntail;
  const int npieces = ntail * split;
  pl.split = split;
  for (int t = 0; t < ntail; ++t)
    pl.tails.push_back(TailItem{owner[nfull + t], slots[nfull + t],
                                     t * split, 0});
  const int X = 8;
  std::vector<int> f0(X + 1, 0), q0(X + 1, 0);
  for (int x = 0; x < X; ++x) {
    f0[x + 1] = f0[x] + nfull / X + (x < nfull % X ? 1 : 0);
    q0[x + 1] = q0[x] + npieces / X + (x < npieces % X ? 1 : 0);
  }
  int per = 0;
  for (int x = 0; x < X; ++x)
    per = std::max(per, (f0[x + 1] - f0[x]) + (q0[x + 1] - q0[x]));
  pl.items.assign(static_cast<size_t>(per) * X,
                  WorkItem{0, -1, -1, 0, 0, 0});
  for (int x = 0; x < X; ++x) {
    const int nf = f0[x + 1] - f0[x], nq = q0[x + 1] - q0[x];
    for (int r = 0; r < nf + nq; ++r) {
      WorkItem& w = pl.items[static_cast<size_t>(r) * X + x];
      if (r < nf) {
        const int t = f0[x] + r;
        w = WorkItem{owner[t], slots[t], -1, 0, nk[t], 0};
      } else {
        const int q = q0[x] + (r - nf);
        const int t = nfull + q / split, j = q % split;
        w = WorkItem{
            owner[t], slots[t], q,
            static_cast<int32_t>(static_cast<int64_t>(j) * nk[t] / split),
            static_cast<int32_t>(static_cast<int64_t>(j + 1) * nk[t] / split),
            0};
      }
    }
  }
  return pl;
}

}  // namespace sp2
