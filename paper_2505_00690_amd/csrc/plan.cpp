// Host-side planning of an encode call (see plan.hpp).
#include "plan.hpp"

#include <string.h>

#include <algorithm>

namespace vl {

int cap_tokens(int T) {
  if (T <= 16) return T;
  const int k = 31 - __builtin_clz((unsigned)T);
  const int step = 1 << (k - 2);
  return std::min((T + step - 1) / step * step, (2 << k) - 1);
}

int cap_images(int n) {
  int c = 1;
  while (c < n) c <<= 1;
  return std::min(c, kMaxItems);
}

namespace {

// The common tail of planning: part boundaries, attention work items, the
// descriptor blob and the workspace regions.  imgs[] hold absolute token
// starts on entry.
bool finish_plan(const PlanModel& m, std::vector<ImgDesc>& imgs, int64_t T, Plan* p,
                 bool one_part, bool bucketed) {
  const int n = (int)imgs.size();
  p->T = (int)T;
  p->bucketed = bucketed;
  // Part boundaries: one part, or two holding about half the tokens each.
  std::vector<int> cut = {0};
  if (!one_part && m.split && n >= 2 && T >= kSplitMinTokens) {
    int n1 = 1;
    while (n1 < n - 1 && imgs[n1].tok_start < T / 2) ++n1;
    cut.push_back(n1);
  }
  cut.push_back(n);
  // Descriptor region: per part, its count record (bucketed), image
  // descriptors, streamed attention items and resident images (each
  // 16-byte aligned).
  auto a16 = [](size_t x) { return (x + 15) / 16 * 16; };
  p->parts.clear();
  std::vector<std::vector<AttnItem>> items(cut.size() - 1);
  std::vector<std::vector<int32_t>> res(cut.size() - 1);
  const bool res_ok = m.resident && !m.text;
  size_t doff = 0;
  for (size_t k = 0; k + 1 < cut.size(); ++k) {
    Part q;
    q.i0 = cut[k];
    q.n = cut[k + 1] - cut[k];
    const int t0 = imgs[q.i0].tok_start;
    for (int i = q.i0; i < cut[k + 1]; ++i) {
      imgs[i].tok_start -= t0;
      q.T += imgs[i].ntok;
      q.max_ntok = std::max<int>(q.max_ntok, imgs[i].ntok);
      const int nt = imgs[i].ntok;
      if (res_ok && nt > kResMinTokens && nt <= 64 * kResMaxTiles) {
        res[k].push_back(i - q.i0);
        q.res_tiles = std::max(q.res_tiles, (nt + 63) / 64);
      } else {
        for (int q0 = 0; q0 < nt; q0 += kAttnQ) items[k].push_back(AttnItem{i - q.i0, q0});
      }
    }
    q.n_items = (int)items[k].size();
    q.n_res = (int)res[k].size();
    q.T_cap = q.T; q.n_cap = q.n; q.items_cap = q.n_items; q.res_cap = q.n_res;
    q.ntok_cap = q.max_ntok; q.res_class = q.res_tiles;
    if (bucketed) {
      // Every batch of the bucket fits: a part's streamed items number at
      // most sum ceil(ntok / 128) <= T / 128 + n, its resident images at
      // most n, each of at most kResMaxTiles key tiles, its images at most
      // kMaxTokens tokens.  Both attention kernels are launched (their live
      // counts may be 0).
      q.T_cap = cap_tokens(q.T);
      q.n_cap = cap_images(q.n);
      q.items_cap = (q.T_cap + kAttnQ - 1) / kAttnQ + q.n_cap;
      q.res_cap = res_ok ? q.n_cap : 0;
      q.ntok_cap = kMaxTokens;
      q.res_class = kResMaxTiles;
      q.bucketed = true;
      q.off_bc = doff;
      doff = a16(doff + sizeof(BatchCounts));
    }
    q.off_imgs = doff;
    doff = a16(doff + sizeof(ImgDesc) * q.n_cap);
    q.off_items = doff;
    doff = a16(doff + sizeof(AttnItem) * q.items_cap);
    q.off_res = doff;
    doff = a16(doff + sizeof(int32_t) * q.res_cap);
    p->parts.push_back(q);
  }
  p->desc_bytes = doff;
  p->desc.assign(doff, 0);
  for (size_t k = 0; k < p->parts.size(); ++k) {
    const Part& q = p->parts[k];
    memcpy(p->desc.data() + q.off_imgs, imgs.data() + q.i0, sizeof(ImgDesc) * q.n);
    if (q.n_items)
      memcpy(p->desc.data() + q.off_items, items[k].data(), sizeof(AttnItem) * q.n_items);
    if (q.n_res) memcpy(p->desc.data() + q.off_res, res[k].data(), sizeof(int32_t) * q.n_res);
    if (bucketed) {
      BatchCounts bc{q.T, q.n, q.n_items, q.n_res, nullptr, nullptr};   // pointers: bind_batch
      memcpy(p->desc.data() + q.off_bc, &bc, sizeof bc);
    }
  }
  // Workspace: the descriptor region, then each part's activation regions
  // (token info, residual X, LayerNorm / attention output Y, QKV / MLP
  // hidden QH (which also holds the pooled rows at the end), projected
  // embeddings E, and the optional MAP and LayerNorm-folding buffers).
  const size_t es = m.es;
  const size_t qh_cols = std::max<size_t>({(size_t)3 * m.D, (size_t)m.F, (size_t)m.Kpad});
  size_t off = align_up(p->desc_bytes);
  for (Part& q : p->parts) {
    const size_t Tc = q.T_cap, nc = q.n_cap;
    q.off_tok = off;
    off += align_up(8 * Tc);
    q.off_X = off;
    off += align_up(4ull * Tc * m.D);
    q.off_Y = off;
    off += align_up(es * Tc * m.D);
    q.off_QH = off;
    off += align_up(es * Tc * qh_cols);
    q.off_E = off;
    off += align_up(4ull * nc * m.Pd);
    if (!m.text && m.map_pool) {
      q.off_map = off;
      off += align_up(4ull * nc * (3 * (size_t)m.D + m.F));
    }
    if (m.fold_buffers) {
      q.off_U = off;
      off += align_up(2ull * Tc * m.D);
      q.off_PS = off;
      off += align_up(4ull * Tc * (m.D / 32) * 2);
      q.off_RS = off;
      off += align_up(8ull * Tc);
    }
  }
  p->total = off;
  return true;
}

}  // namespace

bool make_plan(const PlanModel& m, int32_t n, const int32_t* hs, const int32_t* ws, Plan* p,
               std::string* why, bool one_part, bool bucketed) {
  if (m.text) { *why = "this model encodes texts (vl_encode_texts)"; return false; }
  if (n <= 0) { *why = "n_images must be > 0"; return false; }
  if (n > kMaxItems) { *why = "n_images must be <= 65535 (split larger batches)"; return false; }
  if (!hs || !ws) { *why = "heights/widths are NULL"; return false; }
  p->n = n;
  p->hw.resize(2 * (size_t)n);
  std::vector<ImgDesc> imgs(n);
  int64_t pix = 0, T = 0;
  for (int i = 0; i < n; ++i) {
    const int H = hs[i], W = ws[i];
    if (H < m.P || W < m.P) { *why = "image " + std::to_string(i) + " smaller than one patch"; return false; }
    const int gh = H / m.P, gw = W / m.P;
    const int64_t ntok = 1 + (int64_t)gh * gw;
    if (ntok > kMaxTokens) { *why = "image " + std::to_string(i) + " has more than 1024 patches"; return false; }
    ImgDesc& d = imgs[i];
    d.pix_off = pix;
    d.H = H; d.W = W; d.gh = gh; d.gw = gw;
    d.tok_start = (int32_t)T;   // absolute for now
    d.ntok = (int32_t)ntok;
    pix += (int64_t)m.channels * H * W;
    T += ntok;
    p->hw[2 * i] = H;
    p->hw[2 * i + 1] = W;
  }
  if (T > kMaxBatchTokens) { *why = "batch exceeds 2^24 tokens"; return false; }
  return finish_plan(m, imgs, T, p, one_part, bucketed);
}

bool make_text_plan(const PlanModel& m, int32_t n, const int32_t* lens, Plan* p,
                    std::string* why) {
  if (!m.text) { *why = "this model encodes images (vl_encode_images)"; return false; }
  if (n <= 0) { *why = "n_texts must be > 0"; return false; }
  if (n > kMaxItems) { *why = "n_texts must be <= 65535 (split larger batches)"; return false; }
  if (!lens) { *why = "lengths is NULL"; return false; }
  p->n = n;
  p->hw.assign(2 * (size_t)n, 0);
  std::vector<ImgDesc> seqs(n);
  int64_t T = 0;
  for (int i = 0; i < n; ++i) {
    if (lens[i] < 1 || lens[i] > m.ctx) {
      *why = "text " + std::to_string(i) + " has length " + std::to_string(lens[i]) +
             ", not in 1.." + std::to_string(m.ctx);
      return false;
    }
    ImgDesc& d = seqs[i];
    d.pix_off = T;   // offset of the sequence's ids in the packed id stream
    d.H = d.W = d.gh = d.gw = 0;
    d.tok_start = (int32_t)T;
    d.ntok = lens[i];
    T += lens[i];
    p->hw[2 * i] = lens[i];
  }
  if (T > kMaxBatchTokens) { *why = "batch exceeds 2^24 tokens"; return false; }
  return finish_plan(m, seqs, T, p, false, false);
}

void bind_batch(Plan& p, const void* pix, float* emb, int Pd) {
  if (!p.bucketed) return;
  for (const Part& q : p.parts) {
    BatchCounts bc;
    memcpy(&bc, p.desc.data() + q.off_bc, sizeof bc);
    bc.pix = static_cast<const float*>(pix);
    bc.emb = emb + (size_t)q.i0 * Pd;
    memcpy(p.desc.data() + q.off_bc, &bc, sizeof bc);
  }
}

}  // namespace vl
