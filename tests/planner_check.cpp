// Host-only checks of the encode planner (paper_2505_00690_amd/csrc/plan.cpp),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_planner_host.py.  Seeded random batches of images and token
// sequences, for several model shapes, one- and two-part and bucketed plans;
// every plan is checked against what the kernels assume of it:
//   - parts cover the images in order; token starts are contiguous and
//     relative to the part; token counts and pixel offsets follow the sizes;
//   - every query block of every image is covered exactly once, by a
//     streamed attention item or by the K/V-resident list (129..640 tokens);
//   - capacities hold the live counts (and, for tokens, keep floor(log2));
//     the count records hold the live counts and, once bound, the pointers;
//   - descriptor and workspace regions are aligned, inside their sizes and
//     pairwise disjoint across parts; the pooled rows fit the QKV region;
//   - two batches with equal per-part capacities get the same layout;
//   - invalid batches are refused with a reason.
// Prints "ok <counts>" and exits 0, or prints the first failure and exits 1.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <random>
#include <string>
#include <utility>
#include <vector>

#include "plan.hpp"

using namespace vl;

namespace {

int g_fail = 0;
#define CHECK(cond, ...)                                        \
  do {                                                          \
    if (!(cond)) {                                              \
      fprintf(stderr, "FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond); \
      fprintf(stderr, __VA_ARGS__);                             \
      fprintf(stderr, "\n");                                    \
      g_fail = 1;                                               \
      return false;                                             \
    }                                                           \
  } while (0)

struct Interval { size_t a, b; const char* what; };

bool disjoint(std::vector<Interval> v, const char* where) {
  std::sort(v.begin(), v.end(), [](const Interval& x, const Interval& y) {
    return x.a != y.a ? x.a < y.a : x.b < y.b;   // empty intervals before others at one offset
  });
  for (size_t i = 1; i < v.size(); ++i)
    CHECK(v[i - 1].b <= v[i].a, "%s: %s [%zu,%zu) overlaps %s [%zu,%zu)", where, v[i - 1].what,
          v[i - 1].a, v[i - 1].b, v[i].what, v[i].a, v[i].b);
  return true;
}

int floor_log2(int x) { return 31 - __builtin_clz((unsigned)x); }

template <typename T>
T read_at(const Plan& p, size_t off, size_t i) {
  T v;
  memcpy(&v, p.desc.data() + off + i * sizeof(T), sizeof(T));
  return v;
}

// Checks one valid plan of the batch (ntok[i] tokens, pixel floats px[i]).
bool check_plan(const PlanModel& m, const Plan& p, const std::vector<int>& ntok,
                const std::vector<int64_t>& px, bool one_part, bool bucketed) {
  const int n = (int)ntok.size();
  int64_t T = 0;
  for (int t : ntok) T += t;
  CHECK(p.n == n && p.T == T, "n %d/%d T %d/%lld", p.n, n, p.T, (long long)T);
  CHECK(p.bucketed == bucketed, "bucketed flag");
  CHECK(p.desc.size() == p.desc_bytes, "descriptor image size");
  const bool two = !one_part && m.split && n >= 2 && T >= kSplitMinTokens;
  CHECK((int)p.parts.size() == (two ? 2 : 1), "parts %zu", p.parts.size());
  std::vector<Interval> dreg, wreg;
  const size_t es = m.es;
  const size_t qh_cols = std::max<size_t>({(size_t)3 * m.D, (size_t)m.F, (size_t)m.Kpad});
  int next_img = 0;
  int64_t sumT = 0;
  for (size_t k = 0; k < p.parts.size(); ++k) {
    const Part& q = p.parts[k];
    CHECK(q.i0 == next_img && q.n >= 1, "part %zu starts at %d, n %d", k, q.i0, q.n);
    next_img += q.n;
    sumT += q.T;
    // descriptors
    int ts = 0, maxn = 0;
    for (int i = 0; i < q.n; ++i) {
      const ImgDesc d = read_at<ImgDesc>(p, q.off_imgs, i);
      CHECK(d.tok_start == ts && d.ntok == ntok[q.i0 + i], "image %d tokens", q.i0 + i);
      CHECK(d.pix_off == px[q.i0 + i], "image %d pixel offset", q.i0 + i);
      if (!m.text) CHECK(d.ntok == 1 + d.gh * d.gw && d.gh == d.H / m.P && d.gw == d.W / m.P,
                         "image %d grid", q.i0 + i);
      ts += d.ntok;
      maxn = std::max(maxn, d.ntok);
    }
    CHECK(ts == q.T && maxn == q.max_ntok, "part %zu token count", k);
    // attention coverage
    std::vector<std::vector<int>> seen(q.n);
    std::vector<int> res_seen(q.n, 0);
    for (int j = 0; j < q.n_items; ++j) {
      const AttnItem it = read_at<AttnItem>(p, q.off_items, j);
      CHECK(it.img >= 0 && it.img < q.n, "item %d image %d", j, it.img);
      CHECK(it.q0 >= 0 && it.q0 < ntok[q.i0 + it.img] && it.q0 % kAttnQ == 0, "item %d q0", j);
      seen[it.img].push_back(it.q0);
    }
    int max_tiles = 0;
    for (int j = 0; j < q.n_res; ++j) {
      const int32_t r = read_at<int32_t>(p, q.off_res, j);
      CHECK(r >= 0 && r < q.n, "resident entry %d", j);
      res_seen[r] += 1;
      max_tiles = std::max(max_tiles, (ntok[q.i0 + r] + 63) / 64);
    }
    CHECK(max_tiles == q.res_tiles, "resident tile count");
    const bool res_ok = m.resident && !m.text;
    for (int i = 0; i < q.n; ++i) {
      const int nt = ntok[q.i0 + i];
      const bool want_res = res_ok && nt > kResMinTokens && nt <= 64 * kResMaxTiles;
      CHECK(res_seen[i] == (want_res ? 1 : 0), "image %d resident %d times", q.i0 + i, res_seen[i]);
      std::vector<int> s = seen[i];
      std::sort(s.begin(), s.end());
      std::vector<int> want;
      if (!want_res)
        for (int q0 = 0; q0 < nt; q0 += kAttnQ) want.push_back(q0);
      CHECK(s == want, "image %d query blocks", q.i0 + i);
    }
    // capacities and count records
    if (!bucketed) {
      CHECK(!q.bucketed && q.T_cap == q.T && q.n_cap == q.n && q.items_cap == q.n_items &&
                q.res_cap == q.n_res && q.ntok_cap == q.max_ntok && q.res_class == q.res_tiles,
            "part %zu capacities of an exact plan", k);
    } else {
      CHECK(q.bucketed && q.T_cap >= q.T && q.n_cap >= q.n && q.items_cap >= q.n_items &&
                q.res_cap >= q.n_res && q.ntok_cap >= q.max_ntok && q.res_class >= q.res_tiles,
            "part %zu capacities below counts", k);
      CHECK(floor_log2(q.T_cap) == floor_log2(q.T), "token capacity %d of %d crosses a power of two",
            q.T_cap, q.T);
      CHECK(q.T <= 16 ? q.T_cap == q.T : 4 * (int64_t)(q.T_cap - q.T) < (int64_t)q.T_cap,
            "token capacity %d of %d", q.T_cap, q.T);
      CHECK(q.n_cap == kMaxItems || (q.n_cap & (q.n_cap - 1)) == 0, "image capacity %d", q.n_cap);
      CHECK(q.n_cap < 2 * q.n || q.n == 1, "image capacity %d of %d", q.n_cap, q.n);
      CHECK(q.ntok_cap == kMaxTokens && q.res_class == kResMaxTiles, "fixed capacities");
      CHECK(q.off_bc % 16 == 0, "count record alignment");
      const BatchCounts bc = read_at<BatchCounts>(p, q.off_bc, 0);
      CHECK(bc.T == q.T && bc.n == q.n && bc.n_items == q.n_items && bc.n_res == q.n_res,
            "count record of part %zu", k);
      dreg.push_back({q.off_bc, q.off_bc + sizeof(BatchCounts), "counts"});
    }
    // descriptor regions
    CHECK(q.off_imgs % 16 == 0 && q.off_items % 16 == 0 && q.off_res % 16 == 0, "desc alignment");
    dreg.push_back({q.off_imgs, q.off_imgs + sizeof(ImgDesc) * q.n_cap, "imgs"});
    dreg.push_back({q.off_items, q.off_items + sizeof(AttnItem) * q.items_cap, "items"});
    dreg.push_back({q.off_res, q.off_res + sizeof(int32_t) * q.res_cap, "res"});
    // workspace regions
    const size_t Tc = q.T_cap, nc = q.n_cap;
    wreg.push_back({q.off_tok, q.off_tok + 8 * Tc, "tok"});
    wreg.push_back({q.off_X, q.off_X + 4 * Tc * m.D, "X"});
    wreg.push_back({q.off_Y, q.off_Y + es * Tc * m.D, "Y"});
    wreg.push_back({q.off_QH, q.off_QH + es * Tc * qh_cols, "QH"});
    wreg.push_back({q.off_E, q.off_E + 4 * nc * m.Pd, "E"});
    if (!m.text && m.map_pool)
      wreg.push_back({q.off_map, q.off_map + 4 * nc * (3 * (size_t)m.D + m.F), "map"});
    if (m.fold_buffers) {
      wreg.push_back({q.off_U, q.off_U + 2 * Tc * m.D, "U"});
      wreg.push_back({q.off_PS, q.off_PS + 4 * Tc * (m.D / 32) * 2, "PS"});
      wreg.push_back({q.off_RS, q.off_RS + 8 * Tc, "RS"});
    }
    // the pooled rows (n x D FP32) reuse the QKV region after the last block
    CHECK(es * Tc * qh_cols >= 4 * nc * (size_t)m.D, "pooled rows do not fit the QKV region");
  }
  CHECK(next_img == n && sumT == T, "parts cover %d images, %lld tokens", next_img, (long long)sumT);
  for (const Interval& r : dreg) CHECK(r.b <= p.desc_bytes, "%s past the descriptor region", r.what);
  for (const Interval& r : wreg) {
    CHECK(r.a % kAlign == 0, "%s not aligned", r.what);
    CHECK(r.a >= align_up(p.desc_bytes) && r.b <= p.total, "%s [%zu,%zu) outside [%zu,%zu)",
          r.what, r.a, r.b, align_up(p.desc_bytes), p.total);
  }
  if (!disjoint(dreg, "descriptors")) return false;
  if (!disjoint(wreg, "workspace")) return false;
  return true;
}

bool check_bind(const PlanModel& m, Plan p) {
  float pix_dummy[4], emb_dummy[4];
  float* emb = emb_dummy;
  bind_batch(p, pix_dummy, emb, m.Pd);
  if (!p.bucketed) return true;
  for (const Part& q : p.parts) {
    const BatchCounts bc = read_at<BatchCounts>(p, q.off_bc, 0);
    CHECK(bc.pix == pix_dummy, "bound pixel pointer");
    CHECK(bc.emb == emb + (size_t)q.i0 * m.Pd, "bound output pointer of part at %d", q.i0);
  }
  return true;
}

std::vector<std::pair<int, int>> caps_of(const Plan& p) {
  std::vector<std::pair<int, int>> c;
  for (const Part& q : p.parts) c.push_back({q.T_cap, q.n_cap});
  return c;
}

bool same_layout(const Plan& a, const Plan& b) {
  CHECK(a.total == b.total && a.desc_bytes == b.desc_bytes && a.parts.size() == b.parts.size(),
        "layout of one bucket differs (total %zu vs %zu)", a.total, b.total);
  for (size_t k = 0; k < a.parts.size(); ++k) {
    const Part &x = a.parts[k], &y = b.parts[k];
    const size_t ox[] = {x.off_bc, x.off_imgs, x.off_items, x.off_res, x.off_tok, x.off_X,
                         x.off_Y, x.off_QH, x.off_E, x.off_map, x.off_U, x.off_PS, x.off_RS};
    const size_t oy[] = {y.off_bc, y.off_imgs, y.off_items, y.off_res, y.off_tok, y.off_X,
                         y.off_Y, y.off_QH, y.off_E, y.off_map, y.off_U, y.off_PS, y.off_RS};
    CHECK(memcmp(ox, oy, sizeof ox) == 0, "offsets of part %zu differ within one bucket", k);
    CHECK(x.items_cap == y.items_cap && x.res_cap == y.res_cap, "capacities differ");
  }
  return true;
}

struct Shape { const char* name; PlanModel m; };

}  // namespace

int main() {
  std::vector<Shape> shapes;
  {
    PlanModel l14;   // ViT-L/14, BF16 activations, every option on
    l14.split = true; l14.resident = true; l14.fold_buffers = true; l14.es = 2;
    l14.D = 1024; l14.F = 4096; l14.Kpad = 640; l14.Pd = 768; l14.P = 14; l14.channels = 3;
    shapes.push_back({"l14_bf16", l14});
    PlanModel f32 = l14;   // FP32 model: no split, no resident attention
    f32.split = false; f32.resident = false; f32.fold_buffers = false; f32.es = 4;
    shapes.push_back({"l14_fp32", f32});
    PlanModel map;   // small model with the attention-pooling head, 4 planes
    map.split = true; map.resident = false; map.map_pool = true; map.es = 2;
    map.D = 128; map.F = 512; map.Kpad = 1024; map.Pd = 128; map.P = 16; map.channels = 4;
    shapes.push_back({"tiny_map", map});
    PlanModel text;   // text tower
    text.text = true; text.split = true; text.es = 2; text.D = 768; text.F = 3072;
    text.Kpad = 0; text.Pd = 768; text.ctx = 77;
    shapes.push_back({"text", text});
  }
  std::mt19937_64 rng(20250501);
  auto uni = [&](int lo, int hi) { return (int)std::uniform_int_distribution<int>(lo, hi)(rng); };
  int plans = 0, two_part = 0, bucket_pairs = 0, refused = 0;
  for (int it = 0; it < 1500 && !g_fail; ++it) {
    const Shape& sh = shapes[it % shapes.size()];
    const PlanModel& m = sh.m;
    const bool big = uni(0, 9) == 0;
    const int n = big ? uni(60, 400) : uni(1, 40);
    const bool one_part = uni(0, 3) == 0;
    const bool bucketed = !m.text && uni(0, 1) == 1;
    std::vector<int32_t> hs(n), ws(n);
    std::vector<int> ntok(n);
    std::vector<int64_t> px(n);
    int64_t pix = 0;
    for (int i = 0; i < n; ++i) {
      if (m.text) {
        hs[i] = uni(1, m.ctx);
        ntok[i] = hs[i];
        px[i] = pix;
        pix += hs[i];
      } else {
        hs[i] = uni(m.P, 32 * m.P + m.P - 1);
        ws[i] = uni(m.P, std::max(m.P, (1024 / std::max(1, hs[i] / m.P)) * m.P + m.P - 1));
        ntok[i] = 1 + (hs[i] / m.P) * (ws[i] / m.P);
        px[i] = pix;
        pix += (int64_t)m.channels * hs[i] * ws[i];
      }
    }
    Plan p;
    std::string why;
    const bool ok = m.text ? make_text_plan(m, n, hs.data(), &p, &why)
                           : make_plan(m, n, hs.data(), ws.data(), &p, &why, one_part, bucketed);
    if (!ok) { fprintf(stderr, "FAIL valid batch refused (%s): %s\n", sh.name, why.c_str()); return 1; }
    ++plans;
    two_part += p.parts.size() == 2;
    if (!check_plan(m, p, ntok, px, one_part && !m.text, bucketed && !m.text)) {
      fprintf(stderr, "  model %s, n %d, one_part %d, bucketed %d\n", sh.name, n, one_part, bucketed);
      return 1;
    }
    if (!check_bind(m, p)) return 1;
    // a neighbour batch: one image a patch row shorter or longer; when its
    // parts land in the same buckets the layout must be identical
    if (bucketed && !m.text) {
      std::vector<int32_t> hs2 = hs;
      const int j = uni(0, n - 1);
      const int dh = uni(0, 1) ? m.P : -m.P;
      if (hs2[j] + dh >= m.P && (1 + ((hs2[j] + dh) / m.P) * (ws[j] / m.P)) <= kMaxTokens) {
        hs2[j] += dh;
        Plan p2;
        if (!make_plan(m, n, hs2.data(), ws.data(), &p2, &why, one_part, true)) {
          fprintf(stderr, "FAIL neighbour batch refused: %s\n", why.c_str());
          return 1;
        }
        if (caps_of(p2) == caps_of(p)) {
          ++bucket_pairs;
          if (!same_layout(p, p2)) return 1;
        }
      }
    }
  }
  if (g_fail) return 1;
  // invalid batches are refused with a reason
  {
    const PlanModel& m = shapes[0].m;
    Plan p;
    std::string why;
    int32_t h1[1] = {13}, w1[1] = {224};
    auto refuse = [&](bool ok, const char* what) {
      if (ok || why.empty()) { fprintf(stderr, "FAIL accepted: %s\n", what); return false; }
      why.clear();
      ++refused;
      return true;
    };
    if (!refuse(make_plan(m, 1, h1, w1, &p, &why), "image smaller than one patch")) return 1;
    int32_t h2[1] = {14 * 33}, w2[1] = {14 * 32};
    if (!refuse(make_plan(m, 1, h2, w2, &p, &why), "more than 1024 patches")) return 1;
    if (!refuse(make_plan(m, 0, h2, w2, &p, &why), "no images")) return 1;
    if (!refuse(make_plan(m, 1, nullptr, w2, &p, &why), "NULL sizes")) return 1;
    std::vector<int32_t> big(65536, 224);
    if (!refuse(make_plan(m, 65536, big.data(), big.data(), &p, &why), "65536 images")) return 1;
    std::vector<int32_t> full(20000, 14 * 32);   // 20000 x 1025 tokens > 2^24
    if (!refuse(make_plan(m, 20000, full.data(), full.data(), &p, &why), "over 2^24 tokens")) return 1;
    const PlanModel& t = shapes[3].m;
    int32_t l1[2] = {5, 78};
    if (!refuse(make_text_plan(t, 2, l1, &p, &why), "text longer than ctx")) return 1;
    int32_t l0[1] = {0};
    if (!refuse(make_text_plan(t, 1, l0, &p, &why), "empty text")) return 1;
    if (!refuse(make_plan(t, 1, h1, w1, &p, &why), "images for a text model")) return 1;
  }
  // capacity function landmarks
  const int tc[][2] = {{1, 1}, {16, 16}, {17, 20}, {31, 31}, {32, 32}, {33, 40}, {541, 640},
                       {2364, 2560}, {18464, 20480}, {32767, 32767}, {32769, 40960}};
  for (const auto& c : tc)
    if (cap_tokens(c[0]) != c[1]) {
      fprintf(stderr, "FAIL cap_tokens(%d) = %d, want %d\n", c[0], cap_tokens(c[0]), c[1]);
      return 1;
    }
  const int ic[][2] = {{1, 1}, {2, 2}, {3, 4}, {12, 16}, {32, 32}, {33, 64}, {65535, 65535}};
  for (const auto& c : ic)
    if (cap_images(c[0]) != c[1]) {
      fprintf(stderr, "FAIL cap_images(%d) = %d, want %d\n", c[0], cap_images(c[0]), c[1]);
      return 1;
    }
  printf("ok plans=%d two_part=%d same_bucket_pairs=%d refused=%d\n", plans, two_part,
         bucket_pairs, refused);
  return 0;
}
