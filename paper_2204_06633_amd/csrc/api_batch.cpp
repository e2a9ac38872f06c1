// C-ABI host layer of the batched calls: validation, work lists, workspace
// layout and launches.  See include/lisaresp.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/lisaresp.h"
#include "batch_types.hpp"
#include "gb_types.hpp"
#include "internal.hpp"
#include "trace.hpp"

namespace {

using lr::set_error;

constexpr int kYTileDefault = 512;    // link samples per fused tile (2 per lane)
constexpr int kMaxSegment = 64;       // tiles per fused work item (segment)
constexpr int64_t kAdjTile = 256;     // samples per adjoint work item (atomic kernels, sky)
constexpr int64_t kCarryTile = 512;   // samples per work item of the carry adjoint kernels
constexpr int64_t kLikeChunk = 8192;  // elements per likelihood work item

enum Region {
  R_TPL, R_ITEMS, R_COUNTER, R_ADJ_TPL, R_TDI_ITEMS, R_PROJ_ITEMS, R_SKY_PART, R_SKY_SPAN,
  R_LIKE_ITEMS, R_LIKE_PART, R_LIKE_SPAN, R_PAIRS, R_TDI_CITEMS, R_PADJ_CITEMS, R_GB_PART,
  R_PADJ_SPAN, R_GY, R_TRIG, R_COUNT
};

static_assert(R_COUNT <= (int)(sizeof(((lr_batch*)nullptr)->off) / sizeof(size_t)),
              "lr_batch.off has a slot per workspace region");

struct Plan {
  int F = 0, B = 0, T_out = 0, Y = 0, K = 1;
  std::vector<lr::BatchTemplate> tpl;
  std::vector<int> items;
  std::vector<lr::BatchAdjTemplate> adj;
  std::vector<int64_t> tdi_items, proj_items, sky_span, like_items, like_span, pairs;
  std::vector<int64_t> tdi_citems, padj_citems, padj_span;
  int64_t gy_doubles = 0, h_extent = 0, out_extent = 0, max_n_out = 0;
  size_t bytes[R_COUNT] = {};
  size_t off[R_COUNT] = {};
  size_t total = 0;
};

bool valid_order(int order) { return order >= 1 && order <= 31 && (order % 2) == 1; }

// Compiled fused-kernel variants: (templates per item, link samples per item),
// array or waveform mode.
bool fused_variant_exists(int group, int tile, bool wave) {
  if (wave) return (group == 1 && tile == 512) || (group == 2 && (tile == 512 || tile == 1024));
  if (tile != 256 && tile != 512 && tile != 1024) return false;
  if (group == 1 || group == 2) return true;
  return group == 4 && tile <= 512;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int make_plan(const lr_template* t, int64_t n, const lr_orbits* tdi, double dt, int order,
              int generation, int channels, int group, int tile, int segment, int adjoint,
              Plan& P) {
  if (n < 0 || (n > 0 && !t)) return set_error(LR_E_ARG, "bad template list");
  if (group != 1 && group != 2 && group != 4)
    return set_error(LR_E_UNSUPPORTED, "group %d (1, 2 or 4 templates per work item)", group);
  if (tile == 0) tile = kYTileDefault;
  if (!fused_variant_exists(group, tile, false))
    return set_error(LR_E_UNSUPPORTED, "tile %d with group %d (tiles of 256, 512 or 1024 link "
                                       "samples; 1024 not with groups of 4)", tile, group);
  P.Y = tile;
  if (segment < 0 || segment > kMaxSegment)
    return set_error(LR_E_ARG, "segment %d (0 = automatic, or 1..%d tiles)", segment, kMaxSegment);
  if (channels != LR_XYZ && channels != LR_AET && channels != LR_XYZ_AET)
    return set_error(LR_E_UNSUPPORTED, "channels %d", channels);
  if (!valid_order(order)) return set_error(LR_E_UNSUPPORTED, "order %d (odd 1..31)", order);
  int64_t F, B;
  if (int st = lr_tdi_padding(tdi, order, generation, dt, &F, &B)) return st;
  P.F = (int)F;
  P.B = (int)B;
  P.T_out = (tile - P.F - P.B) & ~1;
  if (P.T_out < 2)
    return set_error(LR_E_UNSUPPORTED, "dt = %g s is too small for the fused kernel (the TDI "
                                       "stencil needs %lld + %lld of %d link samples)",
                     dt, (long long)F, (long long)B, tile);
  const int64_t rows = channels == LR_XYZ_AET ? 6 : 3;

  // grouped forward work list: longest templates first
  std::vector<int64_t> order_idx(n);
  std::iota(order_idx.begin(), order_idx.end(), 0);
  std::stable_sort(order_idx.begin(), order_idx.end(),
                   [&](int64_t a, int64_t b) { return t[a].n_out > t[b].n_out; });
  const int64_t n_groups = (n + group - 1) / group;
  P.tpl.assign(n_groups * group, lr::BatchTemplate{0, 0, 0, 0, 0, -1});
  std::vector<int64_t> gmax(n_groups, 0);
  int64_t tiles1 = 0;                       // work items at one tile per segment
  for (int64_t g = 0; g < n_groups; ++g) {
    for (int k = 0; k < group; ++k) {
      const int64_t s = g * group + k;
      if (s >= n) break;
      const lr_template& T = t[order_idx[s]];
      P.tpl[s] = lr::BatchTemplate{T.h_offset, T.n_h, T.out_start, T.n_out, T.out_offset,
                                   order_idx[s]};
      gmax[g] = std::max(gmax[g], T.n_out);
    }
    tiles1 += (gmax[g] + P.T_out - 1) / P.T_out;
  }
  // Segments of K tiles carry the TDI halo from tile to tile (every tile
  // after the first has `tile` outputs) when the halo fits the kernel's
  // rows; automatic K: up to 8 while the batch keeps >= 2048 work items.
  if (tile - P.T_out > lr::fused_halo_cap(group, tile / 2)) P.K = 1;   // workgroup: tile / 2
  else if (segment > 0) P.K = segment;
  else P.K = (int)std::max<int64_t>(1, std::min<int64_t>(8, tiles1 / 2048));
  // Every segment starts before its group's longest template ends: the
  // fused kernel relies on it (an item without a tile would skip the barrier
  // that orders the reads of the item index before the next fetch).
  const int64_t seg_out = P.T_out + (int64_t)(P.K - 1) * tile;
  for (int64_t g = 0; g < n_groups; ++g) {
    const int64_t segs = (gmax[g] + seg_out - 1) / seg_out;
    for (int64_t sg = 0; sg < segs; ++sg) {
      P.items.push_back((int)g);
      P.items.push_back((int)sg);
    }
  }
  if ((int64_t)P.items.size() / 2 > (int64_t)0x7fffffff)
    return set_error(LR_E_ARG, "too many work items");

  // adjoint and likelihood lists, caller's order
  P.adj.resize(n);
  for (int64_t b = 0; b < n; ++b) {
    const lr_template& T = t[b];
    lr::BatchAdjTemplate A;
    A.h_off = T.h_offset;
    A.n_h = T.n_h;
    A.y_start = T.out_start - P.F;
    A.n_y = T.n_out > 0 ? T.n_out + P.F + P.B : 0;
    A.gy_off = P.gy_doubles;
    A.out_off = T.out_offset;
    A.n_out = T.n_out;
    A.index = b;
    A.t_off_h = 0.0;                      // set by prepare (needs the orbit and t0)
    P.adj[b] = A;
    P.gy_doubles += 6 * A.n_y;
    const int64_t first = (int64_t)P.proj_items.size() / 2;
    for (int64_t tl = 0; tl < (A.n_y + kAdjTile - 1) / kAdjTile; ++tl) {
      P.proj_items.push_back(b);
      P.proj_items.push_back(tl);
    }
    P.sky_span.push_back(first);
    P.sky_span.push_back((int64_t)P.proj_items.size() / 2 - first);
    P.sky_span.push_back(b);
    const int64_t cfirst = (int64_t)P.padj_citems.size() / 2;
    for (int64_t tl = 0; tl < (A.n_y + kCarryTile - 1) / kCarryTile; ++tl) {
      P.padj_citems.push_back(b);
      P.padj_citems.push_back(tl);
    }
    P.padj_span.push_back(cfirst);
    P.padj_span.push_back((int64_t)P.padj_citems.size() / 2 - cfirst);
    P.padj_span.push_back(b);
    const int64_t lfirst = (int64_t)P.like_items.size() / 2;
    const int64_t len = rows * T.n_out;
    for (int64_t c = 0; c < len; c += kLikeChunk) {
      P.like_items.push_back(T.out_offset + c);
      P.like_items.push_back(T.out_offset + std::min(len, c + kLikeChunk));
    }
    P.like_span.push_back(lfirst);
    P.like_span.push_back((int64_t)P.like_items.size() / 2 - lfirst);
    P.like_span.push_back(b);
    P.h_extent = std::max(P.h_extent, T.h_offset + T.n_h);
    P.out_extent = std::max(P.out_extent, T.out_offset + len);
    P.max_n_out = std::max(P.max_n_out, T.n_out);
  }

  // TDI adjoint: templates paired by duration (longer first), one work item
  // per (pair, tile) of the longer one
  for (int64_t q = 0; q < n; q += 2) {
    const int64_t b0 = order_idx[q], b1 = q + 1 < n ? order_idx[q + 1] : -1;
    const int64_t pr = (int64_t)P.pairs.size() / 2;
    P.pairs.push_back(b0);
    P.pairs.push_back(b1);
    for (int64_t tl = 0; tl < (t[b0].n_out + kAdjTile - 1) / kAdjTile; ++tl) {
      P.tdi_items.push_back(pr);
      P.tdi_items.push_back(tl);
    }
    for (int64_t tl = 0; tl < (t[b0].n_out + kCarryTile - 1) / kCarryTile; ++tl) {
      P.tdi_citems.push_back(pr);
      P.tdi_citems.push_back(tl);
    }
  }

  P.bytes[R_TPL] = P.tpl.size() * sizeof(lr::BatchTemplate);
  P.bytes[R_ITEMS] = P.items.size() * sizeof(int);
  P.bytes[R_COUNTER] = sizeof(int);
  P.bytes[R_ADJ_TPL] = P.adj.size() * sizeof(lr::BatchAdjTemplate);
  P.bytes[R_TDI_ITEMS] = adjoint ? P.tdi_items.size() * sizeof(int64_t) : 0;
  P.bytes[R_PROJ_ITEMS] = adjoint ? P.proj_items.size() * sizeof(int64_t) : 0;
  P.bytes[R_SKY_PART] = adjoint ? P.proj_items.size() * sizeof(double) : 0;   // 2 per item
  P.bytes[R_SKY_SPAN] = adjoint ? P.sky_span.size() * sizeof(int64_t) : 0;
  P.bytes[R_LIKE_ITEMS] = P.like_items.size() * sizeof(int64_t);
  P.bytes[R_LIKE_PART] = P.like_items.size() / 2 * sizeof(double);
  P.bytes[R_LIKE_SPAN] = P.like_span.size() * sizeof(int64_t);
  P.bytes[R_PAIRS] = adjoint ? P.pairs.size() * sizeof(int64_t) : 0;
  P.bytes[R_TDI_CITEMS] = adjoint ? P.tdi_citems.size() * sizeof(int64_t) : 0;
  P.bytes[R_PADJ_CITEMS] = adjoint ? P.padj_citems.size() * sizeof(int64_t) : 0;
  P.bytes[R_GB_PART] = adjoint ? P.padj_citems.size() / 2 * 7 * sizeof(double) : 0;
  P.bytes[R_PADJ_SPAN] = adjoint ? P.padj_span.size() * sizeof(int64_t) : 0;
  P.bytes[R_GY] = adjoint ? (size_t)P.gy_doubles * sizeof(double) : 0;
  P.bytes[R_TRIG] = (size_t)n * 4 * sizeof(double);
  size_t o = 0;
  for (int r = 0; r < R_COUNT; ++r) {
    P.off[r] = o;
    o = align256(o + P.bytes[r]);
  }
  P.total = std::max<size_t>(o, 256);
  return LR_OK;
}

bool disjoint(std::vector<std::pair<int64_t, int64_t>> iv) {
  std::sort(iv.begin(), iv.end());
  for (size_t i = 1; i < iv.size(); ++i)
    if (iv[i].first < iv[i - 1].second) return false;
  return true;
}

template <typename T>
T* at(const lr_batch* b, Region r) {
  return reinterpret_cast<T*>(static_cast<char*>(b->ws) + b->off[r]);
}

lr::OrbitView view(const lr_orbits& o) {
  lr::OrbitView v;
  v.coef = static_cast<const double*>(o.coef);
  v.dt = o.dt;
  v.inv_dt = 1.0 / o.dt;
  v.nseg = o.n - 1;
  return v;
}

int check_batch(const lr_batch* b) {
  if (!b || !b->ws || !b->proj.coef || !b->tdi.coef) return set_error(LR_E_ARG, "batch not prepared");
  return LR_OK;
}

int launch_forward(const lr_batch* b, const double* hp, const double* hc, const double* sky,
                   int sky_stride, const double* params, double* out, void* stream) {
  lr::BatchFwdArgs a;
  a.orb_p = view(b->proj);
  a.orb_t = view(b->tdi);
  a.tpl = at<const lr::BatchTemplate>(b, R_TPL);
  a.items = at<const int>(b, R_ITEMS);
  a.n_items = (int)b->n_items;
  a.counter = at<int>(b, R_COUNTER);
  a.t_off_p = b->t0 - b->proj.t0;
  a.t_off_t = b->t0 - b->tdi.t0;
  a.dt = b->dt;
  a.inv_dt = 1.0 / b->dt;
  a.F = b->front;
  a.T_out = b->tile_out;
  a.HP = b->segment > 1 ? b->tile - b->tile_out : 0;
  a.seg_tiles = b->segment;
  a.hp = hp;
  a.hc = hc;
  a.sky = sky;
  a.sky_stride = sky_stride;
  a.trig = at<double>(b, R_TRIG);
  a.params = params;
  a.channels = b->channels;
  a.out = out;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = lr::run_forward_prep(a.counter, sky, sky_stride, b->n_templates,
                                      at<double>(b, R_TRIG), s);
  if (e == hipSuccess)
    e = lr::run_fused_forward(b->order, b->generation, b->group, b->tile, params != nullptr, a,
                              b->blocks, s);
  if (e != hipSuccess) return set_error(LR_E_HIP, "lr_response launch: %s", hipGetErrorString(e));
  return LR_OK;
}

}  // namespace

extern "C" {

size_t lr_batch_workspace(const lr_template* t, int64_t n, const lr_orbits* tdi, double dt,
                          int order, int generation, int channels, int group, int tile,
                          int segment, int adjoint) {
  Plan P;
  if (make_plan(t, n, tdi, dt, order, generation, channels, group, tile, segment, adjoint, P))
    return 0;
  return P.total;
}

int lr_batch_prepare(const lr_template* t, int64_t n, const lr_orbits* proj,
                     const lr_orbits* tdi, double t0, double dt, int order, int generation,
                     int channels, int group, int tile, int segment, int adjoint, void* ws,
                     size_t ws_bytes, lr_batch* out, void* stream) {
  LR_CALL_RANGE();
  if (!out || !proj || !tdi) return set_error(LR_E_ARG, "null pointer");
  if (!std::isfinite(t0) || !(dt > 0.0) || !std::isfinite(dt)) return set_error(LR_E_ARG, "bad t0 or dt");
  Plan P;
  if (int st = make_plan(t, n, tdi, dt, order, generation, channels, group, tile, segment,
                         adjoint, P))
    return st;
  if (!ws || ws_bytes < P.total)
    return set_error(LR_E_WORKSPACE, "workspace %zu bytes < %zu", ws_bytes, P.total);
  int64_t fp, bp;
  if (int st = lr_projection_padding(proj, order, dt, &fp, &bp)) return st;
  const int64_t rows = channels == LR_XYZ_AET ? 6 : 3;
  std::vector<std::pair<int64_t, int64_t>> hiv, oiv;
  for (int64_t b = 0; b < n; ++b) {
    const lr_template& T = t[b];
    if (T.n_out < 0 || T.n_h < 0 || T.h_offset < 0 || T.out_offset < 0)
      return set_error(LR_E_ARG, "template %lld: negative size or offset", (long long)b);
    if (T.n_out == 0) continue;
    const int64_t y0 = T.out_start - P.F, y1 = T.out_start + T.n_out + P.B - 1;
    if (y0 - fp < 0 || y1 + bp > T.n_h - 1)
      return set_error(LR_E_RANGE, "template %lld: h covers [0, %lld) but its link samples "
                                   "[%lld, %lld] need %lld before and %lld after",
                       (long long)b, (long long)T.n_h, (long long)y0, (long long)y1,
                       (long long)fp, (long long)bp);
    hiv.push_back({T.h_offset, T.h_offset + T.n_h});
    oiv.push_back({T.out_offset, T.out_offset + rows * T.n_out});
  }
  if (!disjoint(oiv)) return set_error(LR_E_ARG, "output blocks overlap");
  if (adjoint && !disjoint(hiv)) return set_error(LR_E_ARG, "h ranges overlap (adjoint batch)");
  const double t_off_p = t0 - proj->t0, t_off_t = t0 - tdi->t0;
  const double span_p = (double)(proj->n - 1) * proj->dt, span_t = (double)(tdi->n - 1) * tdi->dt;
  if (n > 0 && P.max_n_out > 0) {
    const double a0 = t_off_p - P.F * dt, a1 = t_off_p + (double)(P.max_n_out + P.B) * dt;
    const double b0 = t_off_t, b1 = t_off_t + (double)P.max_n_out * dt;
    if (!(a0 >= 0.0) || !(a1 <= span_p) || !(b0 >= 0.0) || !(b1 <= span_t))
      return set_error(LR_E_RANGE, "the orbit grids do not cover the batch's sample times");
  }
  for (auto& A : P.adj) A.t_off_h = t_off_p - (double)t[A.index].out_start * dt;

  // host image of the workspace, one copy
  std::vector<char> img(P.total, 0);
  auto put = [&](Region r, const void* src) {
    if (P.bytes[r]) std::memcpy(img.data() + P.off[r], src, P.bytes[r]);
  };
  put(R_TPL, P.tpl.data());
  put(R_ITEMS, P.items.data());
  put(R_ADJ_TPL, P.adj.data());
  put(R_TDI_ITEMS, P.tdi_items.data());
  put(R_PROJ_ITEMS, P.proj_items.data());
  put(R_SKY_SPAN, P.sky_span.data());
  put(R_LIKE_ITEMS, P.like_items.data());
  put(R_LIKE_SPAN, P.like_span.data());
  put(R_PAIRS, P.pairs.data());
  put(R_TDI_CITEMS, P.tdi_citems.data());
  put(R_PADJ_CITEMS, P.padj_citems.data());
  put(R_PADJ_SPAN, P.padj_span.data());
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(ws, img.data(), P.off[R_GY], hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(LR_E_HIP, "lr_batch_prepare copy: %s", hipGetErrorString(e));

  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  const int64_t n_items = (int64_t)P.items.size() / 2;
  const int64_t per_cu = lr::fused_blocks_per_cu(order, generation, group, P.Y, false);

  out->proj = *proj;
  out->tdi = *tdi;
  out->t0 = t0;
  out->dt = dt;
  out->order = order;
  out->generation = generation;
  out->channels = channels;
  out->group = group;
  out->front = P.F;
  out->tile_out = P.T_out;
  out->tile = P.Y;
  out->segment = P.K;
  out->blocks = (int)std::max<int64_t>(1, std::min<int64_t>(n_items, (int64_t)cus * per_cu));
  out->adjoint = adjoint ? 1 : 0;
  out->n_templates = n;
  out->n_items = n_items;
  out->n_tdi_items = (int64_t)P.tdi_items.size() / 2;
  out->n_proj_items = (int64_t)P.proj_items.size() / 2;
  out->n_like_items = (int64_t)P.like_items.size() / 2;
  out->n_tdi_citems = (int64_t)P.tdi_citems.size() / 2;
  out->n_padj_citems = (int64_t)P.padj_citems.size() / 2;
  out->gy_doubles = adjoint ? P.gy_doubles : 0;
  out->h_extent = P.h_extent;
  out->out_extent = P.out_extent;
  out->ws = ws;
  for (int r = 0; r < R_COUNT; ++r) out->off[r] = P.off[r];
  return LR_OK;
}

int lr_response(const lr_batch* b, const double* hp, const double* hc, const double* sky,
                double* out, void* stream) {
  LR_CALL_RANGE();
  if (int st = check_batch(b)) return st;
  if (b->n_items == 0) return LR_OK;
  if (!hp || !hc || !sky || !out) return set_error(LR_E_ARG, "null pointer");
  return launch_forward(b, hp, hc, sky, 2, nullptr, out, stream);
}

int lr_response_gb(const lr_batch* b, const double* params, double* out, void* stream) {
  LR_CALL_RANGE();
  if (int st = check_batch(b)) return st;
  if (b->n_items == 0) return LR_OK;
  if (!params || !out) return set_error(LR_E_ARG, "null pointer");
  if (!fused_variant_exists(b->group, b->tile, true))
    return set_error(LR_E_UNSUPPORTED, "waveform mode with group %d, tile %d (compiled: group 1 "
                                       "or 2 at tile 512, group 2 at tile 1024)", b->group, b->tile);
  return launch_forward(b, nullptr, nullptr, params + 6, 8, params, out, stream);
}

int lr_response_adjoint(const lr_batch* b, const double* hp, const double* hc,
                        const double* sky, const double* g_out, double* g_hp, double* g_hc,
                        double* g_sky, void* stream) {
  LR_CALL_RANGE();
  if (int st = check_batch(b)) return st;
  if (!b->adjoint) return set_error(LR_E_WORKSPACE, "batch prepared without adjoint workspace");
  if (!g_hp || !g_hc || !sky || (b->n_tdi_items > 0 && !g_out))
    return set_error(LR_E_ARG, "null pointer");
  if (g_sky && (!hp || !hc)) return set_error(LR_E_ARG, "the sky gradient needs h+ and hx");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = lr::run_fill_zero(g_hp, b->h_extent, s);
  if (e == hipSuccess) e = lr::run_fill_zero(g_hc, b->h_extent, s);
  if (e == hipSuccess) e = lr::run_fill_zero(at<double>(b, R_GY), b->gy_doubles, s);
  if (e == hipSuccess && g_sky) e = lr::run_fill_zero(g_sky, 2 * b->n_templates, s);
  lr::BatchAdjArgs a;
  a.orb_p = view(b->proj);
  a.orb_t = view(b->tdi);
  a.tpl = at<const lr::BatchAdjTemplate>(b, R_ADJ_TPL);
  a.t_off_y = (b->t0 - b->tdi.t0) - b->front * b->dt;
  a.dt = b->dt;
  a.inv_dt = 1.0 / b->dt;
  a.F = b->front;
  a.channels = b->channels;
  a.hp = hp;
  a.hc = hc;
  a.sky = sky;
  a.g_out = g_out;
  a.g_y = at<double>(b, R_GY);
  a.g_hp = g_hp;
  a.g_hc = g_hc;
  a.sky_part = g_sky ? at<double>(b, R_SKY_PART) : nullptr;
  a.pairs = at<const int64_t>(b, R_PAIRS);
  a.sky_items = at<const int64_t>(b, R_PROJ_ITEMS);
  a.sky_stride = 2;
  a.params = nullptr;
  a.gb_part = nullptr;
  // carry kernels (deterministic) where their rows fit LDS, else atomic ones
  const int cap_t = lr::carry_row_capacity(b->order, (b->generation == 1 ? 3 : 7) * b->tdi.L_max,
                                           b->dt, 12, 4, 0);
  const int cap_p = lr::carry_row_capacity(b->order, 2.01 * b->proj.L_max, b->dt, 2, 2, 21 * 64);
  if (e == hipSuccess && b->n_tdi_items > 0) {
    a.rl_cap = cap_t;
    a.items = at<const int64_t>(b, cap_t > 0 ? R_TDI_CITEMS : R_TDI_ITEMS);
    e = lr::run_batch_tdi_adjoint(b->order, b->generation, a,
                                  cap_t > 0 ? b->n_tdi_citems : b->n_tdi_items, s);
  }
  if (e == hipSuccess && b->n_proj_items > 0) {
    a.rl_cap = cap_p;
    a.items = at<const int64_t>(b, cap_p > 0 ? R_PADJ_CITEMS : R_PROJ_ITEMS);
    e = lr::run_batch_project_adjoint(b->order, a, cap_p > 0 ? b->n_padj_citems : b->n_proj_items,
                                      b->n_proj_items, s);
  }
  if (e == hipSuccess && g_sky && b->n_proj_items > 0)
    e = lr::run_batch_sky_finalize(a.sky_part, at<const int64_t>(b, R_SKY_SPAN), b->n_templates,
                                   g_sky, s);
  if (e != hipSuccess)
    return set_error(LR_E_HIP, "lr_response_adjoint launch: %s", hipGetErrorString(e));
  return LR_OK;
}

int lr_response_adjoint_gb(const lr_batch* b, const double* params, const double* g_out,
                           double* g_params, void* stream) {
  LR_CALL_RANGE();
  if (int st = check_batch(b)) return st;
  if (!b->adjoint) return set_error(LR_E_WORKSPACE, "batch prepared without adjoint workspace");
  if (!params || !g_params || (b->n_tdi_items > 0 && !g_out))
    return set_error(LR_E_ARG, "null pointer");
  const size_t pb = (size_t)b->n_templates * 8 * sizeof(double);
  if (pb && (reinterpret_cast<uintptr_t>(g_params) < reinterpret_cast<uintptr_t>(params) + pb &&
             reinterpret_cast<uintptr_t>(params) < reinterpret_cast<uintptr_t>(g_params) + pb))
    return set_error(LR_E_ARG, "g_params overlaps params");
  const int cap_t = lr::carry_row_capacity(b->order, (b->generation == 1 ? 3 : 7) * b->tdi.L_max,
                                           b->dt, 12, 4, 0);
  const int cap_p = lr::carry_row_capacity(b->order, 2.01 * b->proj.L_max, b->dt, 2, 2, 21 * 64);
  if (cap_p == 0)
    return set_error(LR_E_UNSUPPORTED, "dt = %g s is too small for the parameter adjoint (the "
                                       "projection footprints do not fit LDS)", b->dt);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = lr::run_fill_zero(at<double>(b, R_GY), b->gy_doubles, s);
  lr::BatchAdjArgs a;
  a.orb_p = view(b->proj);
  a.orb_t = view(b->tdi);
  a.tpl = at<const lr::BatchAdjTemplate>(b, R_ADJ_TPL);
  a.t_off_y = (b->t0 - b->tdi.t0) - b->front * b->dt;
  a.dt = b->dt;
  a.inv_dt = 1.0 / b->dt;
  a.F = b->front;
  a.channels = b->channels;
  a.hp = nullptr;
  a.hc = nullptr;
  a.sky = params + 6;
  a.sky_stride = 8;
  a.params = params;
  a.g_out = g_out;
  a.g_y = at<double>(b, R_GY);
  a.g_hp = nullptr;
  a.g_hc = nullptr;
  a.sky_part = at<double>(b, R_SKY_PART);
  a.gb_part = at<double>(b, R_GB_PART);
  a.pairs = at<const int64_t>(b, R_PAIRS);
  a.sky_items = at<const int64_t>(b, R_PROJ_ITEMS);
  if (e == hipSuccess && b->n_tdi_items > 0) {
    a.rl_cap = cap_t;
    a.items = at<const int64_t>(b, cap_t > 0 ? R_TDI_CITEMS : R_TDI_ITEMS);
    e = lr::run_batch_tdi_adjoint(b->order, b->generation, a,
                                  cap_t > 0 ? b->n_tdi_citems : b->n_tdi_items, s);
  }
  if (e == hipSuccess && b->n_proj_items > 0) {
    a.rl_cap = cap_p;
    a.items = at<const int64_t>(b, R_PADJ_CITEMS);
    e = lr::run_batch_project_adjoint(b->order, a, b->n_padj_citems, b->n_proj_items, s);
  }
  if (e == hipSuccess)
    e = lr::run_gb_batch_finalize(a.gb_part, at<const int64_t>(b, R_PADJ_SPAN), a.sky_part,
                                  at<const int64_t>(b, R_SKY_SPAN), params, b->n_templates,
                                  g_params, s);
  if (e != hipSuccess)
    return set_error(LR_E_HIP, "lr_response_adjoint_gb launch: %s", hipGetErrorString(e));
  return LR_OK;
}

int lr_batch_loglike(const lr_batch* b, const double* out, const double* data, double sigma,
                     double* loglike, double* g_out, void* stream) {
  LR_CALL_RANGE();
  if (int st = check_batch(b)) return st;
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return set_error(LR_E_ARG, "sigma must be positive");
  if (!loglike || (b->n_like_items > 0 && (!out || !data))) return set_error(LR_E_ARG, "null pointer");
  if (b->n_templates == 0) return LR_OK;
  hipError_t e = lr::run_batch_loglike(out, data, at<const int64_t>(b, R_LIKE_ITEMS),
                                       b->n_like_items, 1.0 / (sigma * sigma), g_out,
                                       at<double>(b, R_LIKE_PART),
                                       at<const int64_t>(b, R_LIKE_SPAN), b->n_templates,
                                       loglike, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return set_error(LR_E_HIP, "lr_batch_loglike launch: %s", hipGetErrorString(e));
  return LR_OK;
}

int lr_batch_set_grid(lr_batch* b, int blocks) {
  if (int st = check_batch(b)) return st;
  if (blocks < 1) return set_error(LR_E_ARG, "grid of %d work-groups", blocks);
  b->blocks = blocks;
  return LR_OK;
}

}  // extern "C"
