// Host checks of the library's pure host code, built with the address and
// undefined-behaviour sanitizers by tests/test_host_sanitize.py (no GPU):
// the launch planning (tile order, K-split tail tiles, per-XCD dealing) on
// random groups, checked for exact coverage of every tile and K slice, and
// the SP2-ACC schedule (Alg. 3) on random, edge and invalid bounds, and the
// storage order of the block-sparse blocks.
// Prints "ok" and returns 0 when every check holds.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <random>
#include <set>
#include <utility>
#include <vector>

#include "../include/sp2.h"
#include "../paper_1507_02087_amd/csrc/host_plan.h"

namespace {

int g_fail = 0;

#define CHECK(cond, ...)                              \
  do {                                                \
    if (!(cond)) {                                    \
      fprintf(stderr, "check failed: %s: ", #cond);   \
      fprintf(stderr, __VA_ARGS__);                   \
      fprintf(stderr, "\n");                          \
      if (++g_fail > 20) exit(1);                     \
    }                                                 \
  } while (0)

void check_row_stride() {
  for (int64_t np = 32; np <= 70000; np += 32) {
    const int64_t ld = sp2::row_stride(np);
    const bool pad = np >= 2048 && np % 512 == 0;
    CHECK(ld == (pad ? np + 128 : np), "np %lld ld %lld", (long long)np, (long long)ld);
  }
}

void check_tile_list() {
  for (int nt = 1; nt <= 80; ++nt) {
    std::vector<int2> t;
    sp2::append_tile_list(nt, t);
    CHECK(static_cast<int>(t.size()) == nt * (nt + 1) / 2, "nt %d size %zu", nt, t.size());
    std::set<std::pair<int, int>> seen;
    for (const int2& p : t) {
      CHECK(0 <= p.x && p.x <= p.y && p.y < nt, "nt %d tile (%d, %d)", nt, p.x, p.y);
      CHECK(seen.insert({p.x, p.y}).second, "nt %d duplicate (%d, %d)", nt, p.x, p.y);
    }
  }
}

// Every full tile once with its whole K range; every tail tile split into
// `split` consecutive non-empty K pieces numbered t * split + j; filler
// items (slot -1) only where an XCD has fewer items than the widest.
void check_plan_once(std::mt19937& rng) {
  std::uniform_int_distribution<int> dtiles(1, 2500), dconc(1, 2048), dnk(1, 600),
      dsplit(0, 64), dinst(0, 40);
  const int ntiles = dtiles(rng);
  const int conc = dconc(rng);
  int tail_split = dsplit(rng);
  if (tail_split > 4 && rng() % 3) tail_split = rng() % 2;   // mostly auto / off
  std::vector<int> slots(ntiles), owner(ntiles), nk(ntiles);
  const bool same_nk = rng() % 2;
  const int nk0 = dnk(rng);
  for (int t = 0; t < ntiles; ++t) {
    slots[t] = t;
    owner[t] = dinst(rng);
    nk[t] = same_nk ? nk0 : dnk(rng);
  }
  std::shuffle(slots.begin(), slots.end(), rng);
  const sp2::Plan pl = sp2::make_plan(slots, owner, nk, conc, tail_split);
  const int min_nk = *std::min_element(nk.begin(), nk.end());
  const int split = pl.split;
  CHECK(split >= 1 && split <= std::max(1, min_nk), "split %d min_nk %d", split, min_nk);
  const int ntail = static_cast<int>(pl.tails.size());
  const int nfull = ntiles - ntail;
  CHECK(ntail >= 0 && ntail <= ntiles, "ntail %d", ntail);
  if (split == 1) CHECK(ntail == 0, "no split but %d tails", ntail);
  CHECK(pl.items.size() % 8 == 0, "items %zu", pl.items.size());
  std::vector<int> full_seen(ntiles, 0), piece_seen(static_cast<size_t>(ntail) * split, 0);
  // slot -> tile index
  std::vector<int> tile_of(ntiles);
  for (int t = 0; t < ntiles; ++t) tile_of[slots[t]] = t;
  for (int t = 0; t < ntail; ++t) {
    const sp2::TailItem& ti = pl.tails[t];
    CHECK(ti.slot == slots[nfull + t] && ti.inst == owner[nfull + t] &&
              ti.piece0 == t * split,
          "tail %d", t);
  }
  for (size_t b = 0; b < pl.items.size(); ++b) {
    const sp2::WorkItem& w = pl.items[b];
    if (w.slot < 0) continue;
    CHECK(w.slot < ntiles, "item %zu slot %d", b, w.slot);
    if (w.slot >= ntiles) continue;
    const int t = tile_of[w.slot];
    CHECK(w.inst == owner[t], "item %zu owner", b);
    if (w.piece < 0) {
      CHECK(t < nfull, "full item %zu on tail tile %d", b, t);
      CHECK(w.k0 == 0 && w.k1 == nk[t], "full item %zu k [%d, %d) nk %d", b, w.k0, w.k1,
            nk[t]);
      ++full_seen[t];
    } else {
      CHECK(w.piece < ntail * split, "piece %d", w.piece);
      if (w.piece >= ntail * split) continue;
      const int tt = nfull + w.piece / split, j = w.piece % split;
      CHECK(tt == t, "piece %d of tile %d on tile %d", w.piece, tt, t);
      const int e0 = static_cast<int>(static_cast<int64_t>(j) * nk[t] / split);
      const int e1 = static_cast<int>(static_cast<int64_t>(j + 1) * nk[t] / split);
      CHECK(w.k0 == e0 && w.k1 == e1 && e1 > e0, "piece %d k [%d, %d)", w.piece, w.k0,
            w.k1);
      ++piece_seen[w.piece];
    }
  }
  for (int t = 0; t < nfull; ++t) CHECK(full_seen[t] == 1, "full tile %d seen %d", t, full_seen[t]);
  for (size_t q = 0; q < piece_seen.size(); ++q)
    CHECK(piece_seen[q] == 1, "piece %zu seen %d", q, piece_seen[q]);
}

// Block storage order of the block-sparse iterates (blk_off): a permutation
// of the 1024 elements in which lane l = m + 32 g reads its MFMA operand
// (row m, columns 16 g .. 16 g + 15) as four 16-byte loads at 256 u + 4 l,
// and in which the four elements (r, 8 a + 4 h + e), e = 0..3, of a row are
// consecutive (the stored transpose read for the old block, and the
// transposed output block written as 16-byte stores).
void check_blk_off() {
  std::vector<int> seen(1024, 0);
  for (int m = 0; m < 32; ++m)
    for (int c = 0; c < 32; ++c) {
      const int o = sp2::blk_off(m, c);
      CHECK(o >= 0 && o < 1024, "blk_off(%d, %d) = %d", m, c, o);
      if (o >= 0 && o < 1024) ++seen[o];
    }
  for (int o = 0; o < 1024; ++o) CHECK(seen[o] == 1, "offset %d used %d times", o, seen[o]);
  for (int l = 0; l < 64; ++l)
    for (int u = 0; u < 4; ++u)
      for (int e = 0; e < 4; ++e) {
        const int m = l & 31, g = l >> 5;
        CHECK(sp2::blk_off(m, 16 * g + 4 * u + e) == 256 * u + 4 * l + e,
              "operand load of lane %d, panel %d", l, u);
      }
  for (int r = 0; r < 32; ++r)
    for (int h = 0; h < 2; ++h)
      for (int a = 0; a < 4; ++a)
        for (int e = 0; e < 4; ++e)
          CHECK(sp2::blk_off(r, 8 * a + 4 * h + e) ==
                    ((2 * a + h) & 3) * 256 + (r + 32 * (a >> 1)) * 4 + e,
                "row segment (%d, %d, %d)", r, h, a);
}

void check_schedule(std::mt19937& rng) {
  std::uniform_real_distribution<double> u(0.0, 1.0);
  std::vector<int8_t> p(SP2_MAX_ITER_LIMIT);
  std::vector<double> alpha(SP2_MAX_ITER_LIMIT);
  int valid = 0;
  for (int it = 0; it < 4000; ++it) {
    // sorted random bounds, sometimes degenerate, sometimes out of order
    double v[6];
    for (double& x : v) x = -3.0 + 6.0 * u(rng);
    std::sort(v, v + 6);
    if (it % 7 == 0) v[2] = v[3];                       // homo_out = homo_in
    if (it % 11 == 0) v[4] = v[5];                      // lumo_in = lumo_out
    if (it % 13 == 0) std::swap(v[3], v[4]);            // overlapping
    if (it % 17 == 0) v[1] = NAN;
    if (it % 19 == 0) v[5] = INFINITY;
    const int cap = (it % 5 == 0) ? 1 + static_cast<int>(rng() % 40) : SP2_MAX_ITER_LIMIT;
    const int acc = static_cast<int>(rng() % 2);
    int32_t n_min = -1, n_max = -1;
    const sp2_status st = sp2_acc_schedule(v[0], v[5], v[1], v[2], v[3], v[4], acc, cap,
                                           &n_min, &n_max, p.data(), alpha.data());
    if (st != SP2_OK) {
      CHECK(st == SP2_INVALID_ARG, "status %d", static_cast<int>(st));
      continue;
    }
    ++valid;
    CHECK(n_min >= 1 && n_min <= n_max && n_max <= cap, "n_min %d n_max %d cap %d", n_min,
          n_max, cap);
    for (int i = 0; i < n_max; ++i) {
      CHECK(p[i] == 0 || p[i] == 1, "p %d", p[i]);
      CHECK(isfinite(alpha[i]) && alpha[i] >= 1.0 && alpha[i] <= 2.0, "alpha %g", alpha[i]);
      if (!acc) CHECK(alpha[i] == 1.0, "alpha %g without acceleration", alpha[i]);
    }
    // NULL arrays: only the lengths
    int32_t m0 = -1, m1 = -1;
    CHECK(sp2_acc_schedule(v[0], v[5], v[1], v[2], v[3], v[4], acc, 0, &m0, &m1, nullptr,
                           nullptr) == SP2_OK &&
              m0 == n_min && m1 == n_max,
          "lengths without arrays");
  }
  CHECK(valid > 500, "only %d valid bound sets", valid);
  int32_t a = 0, b = 0;
  CHECK(sp2_acc_schedule(-1, 1, -0.5, -0.5, 0.5, 0.5, 1, 10, nullptr, &b, nullptr,
                         nullptr) == SP2_INVALID_ARG,
        "NULL n_min");
  CHECK(sp2_acc_schedule(-1, 1, -0.5, -0.5, 0.5, 0.5, 1, 10, &a, nullptr, nullptr,
                         nullptr) == SP2_INVALID_ARG,
        "NULL n_max");
}

}  // namespace

int main() {
  std::mt19937 rng(20150708);
  check_row_stride();
  check_tile_list();
  check_blk_off();
  for (int i = 0; i < 3000; ++i) check_plan_once(rng);
  check_schedule(rng);
  if (g_fail) {
    fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  printf("ok\n");
  return 0;
}
