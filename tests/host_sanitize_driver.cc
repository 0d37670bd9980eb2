// Host runtime of libtsqbx.so under AddressSanitizer and UBSan (CPU only):
// geometry validation, the host layout (Morton orders, row remap, padding),
// the batch schedule with list lengths whose sums pass 2^31, and the
// server's first-fit arena against a byte-map model.  Exit status 0 and no
// sanitizer report on success; a nonzero status names the failed check.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "tsqbx.h"
#include "tsqbx_arena.h"

static int fails = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++fails;                                                       \
    }                                                                \
  } while (0)

struct Problem {
  std::vector<double> src, w, nrm, ctr, tgt;
  std::vector<int64_t> off;
  std::vector<int32_t> idx, tc;
  tsqbx_geometry_desc desc() const {
    tsqbx_geometry_desc d;
    std::memset(&d, 0, sizeof d);
    d.n_sources = (int64_t)w.size();
    d.sources = src.data();
    d.weights = w.data();
    d.normals = nrm.data();
    d.n_centers = (int64_t)ctr.size() / 3;
    d.centers = ctr.data();
    d.list_offsets = off.data();
    d.list_sources = idx.data();
    d.n_targets = (int64_t)tgt.size() / 3;
    d.targets = tgt.data();
    d.target_center = tc.empty() ? nullptr : tc.data();
    return d;
  }
};

// Ragged lists with empty rows and duplicates, several targets per center.
static Problem make(std::mt19937_64 &rng, int n, int m, int max_list, int tpc) {
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  Problem P;
  for (int i = 0; i < 3 * n; ++i) P.src.push_back(u(rng));
  for (int i = 0; i < n; ++i) P.w.push_back(0.5 + 0.25 * u(rng));
  P.nrm = P.src;
  for (int i = 0; i < 3 * m; ++i) P.ctr.push_back(0.3 * u(rng));
  P.off.push_back(0);
  for (int c = 0; c < m; ++c) {
    const int len = (int)(rng() % (uint64_t)(max_list + 1));
    for (int j = 0; j < len; ++j) P.idx.push_back((int32_t)(rng() % (uint64_t)n));
    P.off.push_back((int64_t)P.idx.size());
  }
  for (int c = 0; c < m; ++c)
    for (int k = 0; k < tpc; ++k) {
      P.tc.push_back(c);
      for (int a = 0; a < 3; ++a) P.tgt.push_back(P.ctr[3 * c + a] + 0.05 * u(rng));
    }
  return P;
}

static void layout_case(const Problem &P, unsigned flags) {
  const tsqbx_geometry_desc d = P.desc();
  CHECK(tsqbx_validate_geometry(&d) == TSQBX_OK);
  tsqbx_layout_info info;
  CHECK(tsqbx_geometry_layout(&d, flags, nullptr, nullptr, nullptr, nullptr, 0, nullptr, 0,
                              &info) == TSQBX_OK);
  const int64_t N = d.n_sources, T = d.n_targets;
  std::vector<int64_t> so(N), to(T), tr(T), ro(info.n_rows + 1);
  std::vector<int32_t> rows(info.nnz);
  // too small a row buffer is refused with the counts filled in
  if (info.nnz > 0)
    CHECK(tsqbx_geometry_layout(&d, flags, so.data(), to.data(), tr.data(), ro.data(),
                                info.n_rows + 1, rows.data(), info.nnz - 1, &info) ==
          TSQBX_E_RANGE);
  CHECK(tsqbx_geometry_layout(&d, flags, so.data(), to.data(), tr.data(), ro.data(),
                              info.n_rows + 1, rows.data(), info.nnz, &info) == TSQBX_OK);
  std::vector<int64_t> rank(N, -1);
  for (int64_t i = 0; i < N; ++i) {
    CHECK(so[i] >= 0 && so[i] < N && rank[so[i]] < 0);
    if (so[i] >= 0 && so[i] < N) rank[so[i]] = i;
  }
  for (int64_t k = 0; k < T; ++k) {
    CHECK(tr[k] >= 0 && tr[k] < info.n_rows);
    const int64_t t = to[k];
    const int64_t c = P.tc[t];
    const int64_t r = tr[k];
    const int64_t len = P.off[c + 1] - P.off[c];
    CHECK(ro[r + 1] - ro[r] == (len + 15) / 16 * 16);
    std::vector<int64_t> want;
    for (int64_t j = P.off[c]; j < P.off[c + 1]; ++j) want.push_back(rank[P.idx[j]]);
    std::sort(want.begin(), want.end());
    for (int64_t j = 0; j < ro[r + 1] - ro[r]; ++j)
      CHECK(rows[ro[r] + j] == (j < len ? want[j] : N));
  }
}

static void schedule_case(int64_t n_items, int64_t per_item, int64_t len, int group_lanes,
                          int max_waves) {
  std::vector<int64_t> nt(n_items, per_item), rl(n_items * per_item, len);
  std::vector<int32_t> p(n_items);
  std::vector<uint32_t> lay(n_items);
  for (int64_t i = 0; i < n_items; ++i) {
    p[i] = (int32_t)(4 * (i % 7));
    lay[i] = 1u + (uint32_t)(i % 7);
  }
  int64_t n_units = 0;
  int32_t n_waves = 0;
  std::vector<int32_t> wb(max_waves + 1);
  // first ask with no room: TSQBX_E_RANGE and the unit count
  int rc = tsqbx_schedule_preview(n_items, nt.data(), rl.data(), p.data(), lay.data(), group_lanes,
                                  max_waves, nullptr, 0, &n_units, wb.data(), &n_waves);
  CHECK(rc == TSQBX_E_RANGE || (rc == TSQBX_OK && n_units == 0));
  std::vector<int32_t> units(3 * std::max<int64_t>(n_units, 1));
  rc = tsqbx_schedule_preview(n_items, nt.data(), rl.data(), p.data(), lay.data(), group_lanes,
                              max_waves, units.data(), n_units, &n_units, wb.data(), &n_waves);
  CHECK(rc == TSQBX_OK);
  // every target of every item exactly once, in contiguous runs
  std::vector<int64_t> seen(n_items, 0);
  for (int64_t u = 0; u < n_units; ++u) {
    const int32_t it = units[3 * u], first = units[3 * u + 1], cnt = units[3 * u + 2];
    CHECK(it >= 0 && it < n_items && cnt > 0);
    if (it >= 0 && it < n_items) {
      CHECK(first == seen[it]);
      seen[it] += cnt;
    }
  }
  for (int64_t i = 0; i < n_items; ++i) CHECK(seen[i] == per_item);
  CHECK(wb[0] == 0 && wb[n_waves] == n_units && n_waves <= max_waves);
}

static void arena_case(std::mt19937_64 &rng, size_t size) {
  tsqbx::Arena a;
  a.init(size);
  std::vector<unsigned char> used(size, 0);
  struct Block { size_t off, n; };
  std::vector<Block> live;
  for (int step = 0; step < 20000; ++step) {
    if (!live.empty() && (rng() % 3 == 0 || live.size() > 64)) {
      const size_t k = (size_t)(rng() % live.size());
      a.release(live[k].off, live[k].n);
      for (size_t b = 0; b < live[k].n; ++b) used[live[k].off + b] = 0;
      live[k] = live.back();
      live.pop_back();
    } else {
      const size_t n = 1 + (size_t)(rng() % (size / 8));
      size_t off = 0;
      // the model: is there a free run of n bytes, and where is the first?
      size_t run = 0, first = size;
      for (size_t b = 0; b < size && first == size; ++b) {
        run = used[b] ? 0 : run + 1;
        if (run >= n) first = b + 1 - n;
      }
      const bool ok = a.alloc(n, &off);
      CHECK(ok == (first < size));
      if (ok) {
        CHECK(off == first);  // first fit over coalesced free ranges
        for (size_t b = 0; b < n; ++b) {
          CHECK(!used[off + b]);
          used[off + b] = 1;
        }
        live.push_back({off, n});
      }
    }
    size_t free_model = 0;
    for (unsigned char x : used) free_model += x ? 0 : 1;
    CHECK(a.free_bytes() == free_model);
  }
  for (auto &b : live) a.release(b.off, b.n);
  CHECK(a.free_bytes() == size && a.free_ranges() == 1);
}

int main() {
  std::mt19937_64 rng(20181101);
  for (int rep = 0; rep < 6; ++rep) {
    Problem P = make(rng, 300 + 50 * rep, 40 + 7 * rep, 90, 1 + rep % 3);
    layout_case(P, 0);
    layout_case(P, TSQBX_NO_REORDER);
  }
  {  // no targets, no sources
    Problem P;
    P.off.push_back(0);
    layout_case(P, 0);
  }
  {  // invalid descriptions are refused before any array is read past its end
    Problem P = make(rng, 50, 5, 10, 1);
    tsqbx_geometry_desc d = P.desc();
    CHECK(tsqbx_validate_geometry(&d) == TSQBX_OK);
    if (!P.idx.empty()) {
      P.idx[0] = 50;  // out of range
      d = P.desc();
      CHECK(tsqbx_validate_geometry(&d) == TSQBX_E_RANGE);
      P.idx[0] = 0;
    }
    P.off[2] = P.off[1] - 1;  // decreasing offsets
    d = P.desc();
    CHECK(tsqbx_validate_geometry(&d) != TSQBX_OK);
    tsqbx_layout_info info;
    CHECK(tsqbx_geometry_layout(&d, 0, nullptr, nullptr, nullptr, nullptr, 0, nullptr, 0,
                                &info) != TSQBX_OK);
  }
  // schedules whose summed list lengths pass 2^31 (int64 arithmetic)
  schedule_case(3, 2000, int64_t(1) << 30, 64, 4096);
  schedule_case(5, 4097, 3000000, 16, 1000);
  schedule_case(64, 37, 200, 32, 49152);
  schedule_case(1, 1, 0, 16, 1);
  for (size_t size : {64u, 1000u, 4096u}) arena_case(rng, size);
  if (fails) {
    std::fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  std::printf("host sanitize ok\n");
  return 0;
}
