// Host-code check under AddressSanitizer and UndefinedBehaviorSanitizer: the operator planner and the float64
// tables of the library, built on their own with g++ (no device code) by tests/test_host_sanitized.py.
//
// Every plan of a set of seeded workloads (uniform and centre-heavy coverage, every visibility in one cell,
// coordinates on cell edges and at -pi and just below pi, one-visibility blocks, several problems, small work
// items) is checked against invariants recomputed here from the inputs:
//   * the internal order is a permutation that keeps every block in place, sorted by (tile, cell) with equal
//     keys in user order, and its fixed-point coordinates are the visibility's position on the grid;
//   * the work items tile the internal order, each one (block, tile) run cut into ceil(run / chunk) items, and
//     their patch slots group the items of each tile in item order;
//   * the J = 8 gridder's row spans are the rows each stream holds, and their sum stays within the
//     T + streams - 1 rows its LDS pool is sized for;
//   * the reduction chunks tile each block.
// The tables: I0 against its value at 1, the Daubechies filters' sum, norm, orthogonality to even shifts and
// vanishing moments, the tap polynomials against the window, unit twiddles.
// Exit status 0 and a last line "ok" when everything holds.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "plan.hpp"
#include "tables.hpp"

#define CHECK(c, ...)                                                               \
  do {                                                                              \
    if (!(c)) {                                                                     \
      std::fprintf(stderr, "FAILED %s:%d: %s: ", __FILE__, __LINE__, #c);           \
      std::fprintf(stderr, __VA_ARGS__);                                            \
      std::fprintf(stderr, "\n");                                                   \
      std::exit(1);                                                                 \
    }                                                                               \
  } while (0)

namespace {

int ilog2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

struct Case {
  std::string name;
  int n, T, chunk, streams, P;
  std::vector<int64_t> block_sizes;   // per block, problems get consecutive runs of blocks
  int kind;                           // 0 uniform, 1 centre-heavy, 2 one cell, 3 cell edges and range ends
};

std::vector<double> make_uv(const Case& c, int64_t M, int K, std::mt19937_64& rng) {
  std::vector<double> uv(2 * M);
  std::uniform_real_distribution<double> U(-M_PI, M_PI);
  std::normal_distribution<double> G(0.0, 0.4);
  std::uniform_int_distribution<int> cellpick(-K / 2, K / 2 - 1);
  for (int64_t m = 0; m < 2 * M; ++m) {
    double x = 0;
    switch (c.kind) {
      case 0: x = U(rng); break;
      case 1: x = std::fmod(G(rng), M_PI); break;
      case 2: x = 0.3; break;
      default: {
        const int r = int(rng() % 4);
        if (r == 0) x = -M_PI;
        else if (r == 1) x = std::nextafter(M_PI, 0.0);
        else x = 2.0 * M_PI * double(cellpick(rng)) / K;   // on a cell edge
        if (x >= M_PI) x = -M_PI;
      }
    }
    uv[m] = x;
  }
  return uv;
}

void check_plan(const Case& c, std::mt19937_64& rng) {
  const int K = 2 * c.n, log2K = ilog2(K), F = 32 - log2K, T = c.T, log2T = ilog2(T), nT = K / T;
  const int R = int(c.block_sizes.size());
  std::vector<int64_t> offs(R + 1, 0);
  for (int b = 0; b < R; ++b) offs[b + 1] = offs[b] + c.block_sizes[b];
  const int64_t M = offs[R];
  std::vector<int32_t> block_prob(R);
  for (int b = 0; b < R; ++b) block_prob[b] = int32_t((int64_t)b * c.P / R);
  const std::vector<double> uv = make_uv(c, M, K, rng);
  sh::PlanShape s{M, K, log2K, T, log2T, nT, c.P, R, c.chunk, c.streams};
  sh::HostPlan h;
  sh::plan_host(s, uv.data(), offs.data(), block_prob.data(), h);

  CHECK((int64_t)h.coord.size() == M && (int64_t)h.perm.size() == M, "%s: sizes", c.name.c_str());
  // cells recomputed from the coordinates, and the coordinates against the input
  std::vector<int> cell0(M), cell1(M);
  const double ulp = std::ldexp(1.0, -F);
  for (int64_t i = 0; i < M; ++i) {
    const int64_t m = h.perm[i];
    const uint32_t q[2] = {h.coord[i].x, h.coord[i].y};
    for (int ax = 0; ax < 2; ++ax) {
      const int64_t cl = q[ax] >> F;
      const double pos = double(cl) + double(q[ax] & ((F == 32) ? 0xffffffffu : ((1u << F) - 1u))) * ulp;
      const double kappa = uv[2 * m + ax] * K / (2.0 * M_PI);
      double d = pos - kappa;
      d -= K * std::round(d / K);
      CHECK(cl >= 0 && cl < K, "%s: cell %lld", c.name.c_str(), (long long)cl);
      CHECK(d <= 1e-9 && d > -ulp - 1e-9, "%s: visibility %lld axis %d: grid position %.17g, kappa %.17g",
            c.name.c_str(), (long long)m, ax, pos, kappa);
      (ax == 0 ? cell0 : cell1)[i] = int(cl);
    }
  }
  auto tile_of = [&](int64_t i) { return (cell0[i] >> log2T) * nT + (cell1[i] >> log2T); };
  auto key_of = [&](int64_t i) {
    return (uint64_t(tile_of(i)) << (2 * log2T)) | uint64_t(((cell0[i] & (T - 1)) << log2T) | (cell1[i] & (T - 1)));
  };
  // permutation, blocks kept in place, sorted keys with ties in user order
  std::vector<char> seen(M, 0);
  for (int b = 0; b < R; ++b)
    for (int64_t i = offs[b]; i < offs[b + 1]; ++i) {
      const int64_t m = h.perm[i];
      CHECK(m >= offs[b] && m < offs[b + 1] && !seen[m], "%s: perm[%lld] = %lld", c.name.c_str(), (long long)i,
            (long long)m);
      seen[m] = 1;
      if (i > offs[b]) {
        const uint64_t k0 = key_of(i - 1), k1 = key_of(i);
        CHECK(k0 < k1 || (k0 == k1 && h.perm[i - 1] < h.perm[i]), "%s: order at %lld", c.name.c_str(), (long long)i);
      }
    }
  // work items
  const int64_t NI = (int64_t)h.items.size();
  const int gtiles = c.P * nT * nT;
  CHECK((int64_t)h.item_block.size() == NI, "%s: item_block size", c.name.c_str());
  int64_t pos = 0;
  for (int64_t q = 0; q < NI; ++q) {
    const int4 it = h.items[q];
    const int b = h.item_block[q];
    CHECK(it.y == pos && it.z >= 1 && it.z <= c.chunk, "%s: item %lld (%d, %d)", c.name.c_str(), (long long)q, it.y,
          it.z);
    CHECK(b >= 0 && b < R && it.y >= offs[b] && it.y + it.z <= offs[b + 1], "%s: item %lld block", c.name.c_str(),
          (long long)q);
    for (int64_t i = it.y; i < it.y + it.z; ++i)
      CHECK(it.x == block_prob[b] * nT * nT + tile_of(i), "%s: item %lld tile", c.name.c_str(), (long long)q);
    pos += it.z;
  }
  CHECK(pos == M, "%s: items cover %lld of %lld", c.name.c_str(), (long long)pos, (long long)M);
  for (int64_t q = 0; q < NI;) {   // each (block, tile) run: ceil(run / chunk) items, lengths within one
    int64_t e = q, len = 0, lo = INT64_MAX, hi = 0;
    while (e < NI && h.items[e].x == h.items[q].x && h.item_block[e] == h.item_block[q]) {
      len += h.items[e].z;
      lo = std::min<int64_t>(lo, h.items[e].z);
      hi = std::max<int64_t>(hi, h.items[e].z);
      ++e;
    }
    CHECK(e - q == (len + c.chunk - 1) / c.chunk && hi - lo <= 1, "%s: run at item %lld", c.name.c_str(),
          (long long)q);
    q = e;
  }
  // patch slots
  CHECK((int)h.tile_items.size() == gtiles + 1 && h.tile_items[0] == 0 && h.tile_items[gtiles] == NI,
        "%s: tile_items ends", c.name.c_str());
  std::vector<char> slot_seen(NI, 0);
  std::vector<int64_t> last_item(gtiles, -1);
  int most = 0;
  for (int t = 0; t < gtiles; ++t) most = std::max(most, h.tile_items[t + 1] - h.tile_items[t]);
  CHECK(h.max_items_per_tile == most, "%s: max_items_per_tile %d, %d", c.name.c_str(), h.max_items_per_tile, most);
  for (int64_t q = 0; q < NI; ++q) {
    const int4 it = h.items[q];
    CHECK(it.w >= 0 && it.w < NI && !slot_seen[it.w], "%s: slot of item %lld", c.name.c_str(), (long long)q);
    slot_seen[it.w] = 1;
    CHECK(it.w >= h.tile_items[it.x] && it.w < h.tile_items[it.x + 1], "%s: slot range", c.name.c_str());
    CHECK(last_item[it.x] < 0 || h.items[last_item[it.x]].w < it.w, "%s: slot order", c.name.c_str());
    last_item[it.x] = q;
  }
  // row spans of the J = 8 gridder
  if (c.streams > 0) {
    CHECK((int64_t)h.item_rows.size() == NI, "%s: item_rows size", c.name.c_str());
    for (int64_t q = 0; q < NI; ++q) {
      const int4 it = h.items[q];
      const uint32_t f[2] = {uint32_t(h.item_rows[q].x), uint32_t(h.item_rows[q].y)};
      const uint32_t r[2] = {uint32_t(h.item_rows[q].z), uint32_t(h.item_rows[q].w)};
      int sum = 0;
      for (int k = 0; k < c.streams; ++k) {
        const int64_t lo = it.y + (int64_t)it.z * k / c.streams, hi = it.y + (int64_t)it.z * (k + 1) / c.streams;
        int mn = T, mx = -1;
        for (int64_t i = lo; i < hi; ++i) {
          mn = std::min(mn, cell0[i] & (T - 1));
          mx = std::max(mx, cell0[i] & (T - 1));
        }
        const int first = (f[k / 4] >> (8 * (k % 4))) & 0xff, rows = (r[k / 4] >> (8 * (k % 4))) & 0xff;
        if (hi > lo) CHECK(first == mn && rows == mx - mn + 1, "%s: item %lld stream %d rows", c.name.c_str(),
                           (long long)q, k);
        else CHECK(first == 0 && rows == 1, "%s: empty stream", c.name.c_str());
        CHECK(first + rows <= T, "%s: row span past the tile", c.name.c_str());
        sum += rows;
      }
      CHECK(sum <= T + c.streams - 1, "%s: item %lld: %d rows over the streams, pool holds %d", c.name.c_str(),
            (long long)q, sum, T + c.streams - 1);
    }
  } else {
    CHECK(h.item_rows.empty(), "%s: row spans without streams", c.name.c_str());
  }
  // reduction chunks
  CHECK((int)h.chunk_first.size() == R + 1 && h.chunk_first[R] == (int32_t)h.chunks.size(), "%s: chunk_first",
        c.name.c_str());
  for (int b = 0; b < R; ++b) {
    int64_t at = offs[b];
    for (int k = h.chunk_first[b]; k < h.chunk_first[b + 1]; ++k) {
      const int4 ch = h.chunks[k];
      CHECK(ch.x == b && ch.y == at && ch.z > ch.y && ch.z - ch.y <= sh::BALL_CHUNK, "%s: chunk %d", c.name.c_str(), k);
      at = ch.z;
    }
    CHECK(at == offs[b + 1], "%s: chunks of block %d", c.name.c_str(), b);
  }
  std::printf("plan %-28s M=%-7lld items=%-6lld most/tile=%d\n", c.name.c_str(), (long long)M, (long long)NI,
              h.max_items_per_tile);
}

void check_tables() {
  CHECK(sh::bessel_i0(0.0) == 1.0, "I0(0)");
  CHECK(std::fabs(sh::bessel_i0(1.0) - 1.2660658777520082) < 1e-15, "I0(1) = %.17g", sh::bessel_i0(1.0));
  for (int p = 1; p <= 8; ++p) {
    double h[16];
    CHECK(sh::daubechies(p, h), "db%d", p);
    const int L = 2 * p;
    double s = 0, e = 0;
    for (int k = 0; k < L; ++k) s += h[k], e += h[k] * h[k];
    CHECK(std::fabs(s - std::sqrt(2.0)) < 1e-12 && std::fabs(e - 1.0) < 1e-12, "db%d sum %.17g norm %.17g", p, s, e);
    for (int m = 1; m < p; ++m) {
      double o = 0;
      for (int k = 0; k + 2 * m < L; ++k) o += h[k] * h[k + 2 * m];
      CHECK(std::fabs(o) < 1e-12, "db%d shift %d: %.3g", p, m, o);
    }
    for (int j = 0; j < p; ++j) {   // the high-pass filter g_k = (-1)^k h_(L-1-k) has p vanishing moments
      double mom = 0, scale = 0;
      for (int k = 0; k < L; ++k) {
        const double g = (k % 2 ? -1.0 : 1.0) * h[L - 1 - k];
        mom += g * std::pow(double(k), j);
        scale += std::fabs(g) * std::pow(double(k), j);
      }
      CHECK(std::fabs(mom) < 1e-10 * scale, "db%d moment %d: %.3g", p, j, mom);
    }
  }
  CHECK(!sh::daubechies(0, nullptr) && !sh::daubechies(21, nullptr), "db order range");
  double worst = 0;
  for (int J = 2; J <= 16; J += 2) {
    const double beta = sh::kb_beta(J, 2);
    std::vector<float> coef(J * 8);
    sh::kb_tap_polys(J, beta, 7, coef.data());
    for (int t = 0; t < J; ++t)
      for (int k = 0; k <= 64; ++k) {
        const double f = k / 64.0 * (1.0 - 1e-12), sv = 2 * f - 1;
        double w = 0, pw = 1;
        for (int i = 0; i < 8; ++i) w += coef[t * 8 + i] * pw, pw *= sv;
        const double err = std::fabs(w - sh::kb_window(f + J / 2 - 1 - t, J, beta));
        worst = std::max(worst, err);
        CHECK(err < 5e-6, "J=%d tap %d f=%g: polynomial off the window by %.3g", J, t, f, err);
      }
  }
  std::vector<float2> tw;
  for (int L : {8, 64, 2048}) {
    sh::fft_twiddles(L, tw);
    CHECK((int)tw.size() == L, "twiddle count");
    for (int m = 0; m < L; ++m)
      CHECK(std::fabs(std::hypot(tw[m].x, tw[m].y) - 1.0) < 1e-6, "twiddle %d of %d", m, L);
  }
  std::printf("tables ok (tap polynomials within %.2g of the window)\n", worst);
}

}  // namespace

int main() {
  std::mt19937_64 rng(20150217);
  std::vector<Case> cases = {
      {"uniform n64 T16 J8", 64, 16, 4096, 4, 1, {3000, 2000, 1, 500}, 0},
      {"centre-heavy n128 T16 chunk 97", 128, 16, 97, 4, 1, {20000, 7000, 1}, 1},
      {"one cell, long runs", 64, 16, 1000, 4, 1, {5000, 1, 2500}, 2},
      {"cell edges and range ends", 32, 8, 33, 8, 1, {4000, 3000}, 3},
      {"three problems n32 T8", 32, 8, 64, 4, 3, {700, 1, 900, 50, 2, 3000}, 0},
      {"T32 no row spans", 64, 32, 512, 0, 1, {9000}, 1},
      {"T64 single visibility", 64, 64, 4096, 4, 1, {1}, 0},
      {"n1024 chunk 4096", 1024, 16, 4096, 4, 1, {60000, 40000, 30000}, 1},
  };
  for (const Case& c : cases) check_plan(c, rng);
  check_tables();
  std::printf("ok\n");
  return 0;
}
