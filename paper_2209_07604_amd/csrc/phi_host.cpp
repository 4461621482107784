// Host side of libphi: argument checks, the plan (visibility sort, work
// items, merge lists, workspace layout), G packing/quantisation, and the C ABI
// entry points declared in include/phi.h.
//
// The plan is built for Phi_{l,b} = Theta_{l,b} G_{l,b} F Z (Section 2.1,
// eq. 1) with data blocks (l, b), and for the per-block l2-ball dual step
// (Section 2.2, eq. 2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "phi.h"
#include "phi_internal.h"
#include "phi_plan.h"

using namespace phi;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

inline uint32_t spread_bits(uint32_t v) {  // 13 bits -> even positions
  v &= 0x1FFF;
  v = (v | (v << 8)) & 0x00FF00FF;
  v = (v | (v << 4)) & 0x0F0F0F0F;
  v = (v | (v << 2)) & 0x33333333;
  v = (v | (v << 1)) & 0x55555555;
  return v;
}
// Z-order key of a window origin: any aligned power-of-two tile of the grid
// is one contiguous run of keys, so one sort serves every tile size.
// (26 bits; the plan's sort key keeps bits 25..8 above the window size.)
inline uint32_t morton(uint32_t by, uint32_t bx) { return (spread_bits(by) << 1) | spread_bits(bx); }

inline int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}
// Round a double to the nearest bfloat16 (ties to even) in one step.
inline uint16_t f64_to_bf16_rne(double d) {
  if (!std::isfinite(d)) return f32_to_bf16_rne((float)d);
  if (d == 0.0) return std::signbit(d) ? 0x8000 : 0;
  int e;
  std::frexp(d, &e);              // |d| in [2^(e-1), 2^e)
  int q = e - 8;                  // spacing of 8 significant bits
  if (q < -133) q = -133;         // bfloat16 subnormal spacing
  const double sc = std::ldexp(1.0, q);
  const double r = std::nearbyint(d / sc) * sc;  // exact; default mode is RNE
  return f32_to_bf16_rne((float)r);              // r is representable: exact
}

const char* kStageNames[] = {"rowfft_fwd", "colfft_fwd", "gather",      "finalize",   "scatter", "merge",
                             "colfft_inv", "rowfft_inv", "pdfb_primal", "eps_update", "dual_gs", "vscale"};
constexpr int kNumStages = 12;

}  // namespace

// ------------------------------------------------------------------ checks
static phi_status validate(const phi_desc* d) {
  if (!d) return PHI_ERR_ARG;
  if (d->n_channels < 1) return PHI_ERR_SHAPE;
  if (d->ny < 8 || d->nx < 8 || (d->ny & 1) || (d->nx & 1)) return PHI_ERR_SHAPE;
  if (d->ny > 4096 || d->nx > 4096) return PHI_ERR_UNSUPPORTED;
  if (!fft_length_supported(2 * d->ny) || !fft_length_supported(2 * d->nx)) return PHI_ERR_UNSUPPORTED;
  if (d->g_prec < PHI_G_C64 || d->g_prec > PHI_G_KB) return PHI_ERR_ARG;
  if (d->flags & ~(PHI_PER_CHANNEL | PHI_GRAPH | PHI_PERSISTENT | PHI_FUSED_GH | PHI_DR)) return PHI_ERR_ARG;
  if ((d->flags & PHI_DR) && d->g_prec == PHI_G_KB) return PHI_ERR_ARG;
  if (d->persist_blocks < 0) return PHI_ERR_ARG;
  const int T = d->tile ? d->tile : 32;
  if (T != 16 && T != 32 && T != 64) return PHI_ERR_ARG;
  if ((2 * d->ny) % T || (2 * d->nx) % T) return PHI_ERR_SHAPE;
  if (!d->h_n_blocks || !d->h_n_vis || !d->h_scale_y || !d->h_scale_x) return PHI_ERR_ARG;
  int64_t nblk = 0;
  for (int l = 0; l < d->n_channels; ++l) {
    if (d->h_n_blocks[l] < 1) return PHI_ERR_SHAPE;
    nblk += d->h_n_blocks[l];
  }
  if (nblk > (int64_t)1 << 24) return PHI_ERR_UNSUPPORTED;
  int64_t M = 0;
  for (int64_t b = 0; b < nblk; ++b) {
    if (d->h_n_vis[b] < 0) return PHI_ERR_SHAPE;
    M += d->h_n_vis[b];
  }
  if (M > INT32_MAX - 64) return PHI_ERR_UNSUPPORTED;
  if (M > 0 && (!d->h_base || !d->h_stencil)) return PHI_ERR_ARG;
  const int Ky = 2 * d->ny, Kx = 2 * d->nx;
  for (int64_t m = 0; m < M; ++m) {
    const int S = d->h_stencil[m];
    if (S < 1 || S > kMaxS || !(S & 1) || S > Ky || S > Kx) return PHI_ERR_RANGE;
    const int by = d->h_base[2 * m], bx = d->h_base[2 * m + 1];
    if (by < 0 || by >= Ky || bx < 0 || bx >= Kx) return PHI_ERR_RANGE;
  }
  if (d->g_prec == PHI_G_KB && M > 0) {
    // one Kaiser-Bessel width J for every visibility
    const int J = d->h_stencil[0];
    if (J != 3 && J != 5 && J != 7 && J != 9 && J != 11) return PHI_ERR_UNSUPPORTED;
    for (int64_t m = 1; m < M; ++m)
      if (d->h_stencil[m] != J) return PHI_ERR_RANGE;
  }
  if (d->h_theta)
    for (int64_t b = 0; b < nblk; ++b)
      if (!(d->h_theta[b] > 0.0) || !std::isfinite(d->h_theta[b])) return PHI_ERR_RANGE;
  for (int p = 0; p < d->ny; ++p)
    if (!std::isfinite(d->h_scale_y[p])) return PHI_ERR_RANGE;
  for (int q = 0; q < d->nx; ++q)
    if (!std::isfinite(d->h_scale_x[q])) return PHI_ERR_RANGE;
  return PHI_OK;
}

template <typename F>
static void parallel_for(int64_t n, F&& f, int max_threads = 16) {
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(max_threads,
                                                                               std::thread::hardware_concurrency()),
                                                            n / 4096 + 1));
  if (nt <= 1) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([=, &f] { f(a, b); });
  }
  for (auto& x : th) x.join();
}

// Work items for tile edge T: split each block's plan-order run at tile
// changes and at a tap budget; then the per-tile merge lists.
static void build_worklist(const phi_plan_s* p, int T, WorkList& w) {
  w.T = T;
  const int lt = ilog2(T);
  w.items.clear();
  w.binfo.assign(p->nblk, BlockInfo{});
  w.chan_item0.assign(p->L + 1, 0);
  const int64_t cap_taps = std::max<int64_t>(4096, std::min<int64_t>(65536, p->ntaps / 16384 + 1));
  int64_t poff = 0;
  int max_pitch = 0;
  int64_t v = 0;
  for (int b = 0; b < p->nblk; ++b) {
    BlockInfo bi{};
    bi.chan = p->blk_chan[b];
    bi.item0 = (int32_t)w.items.size();
    bi.v0 = v;
    const int64_t vend = v + p->blk_n[b];
    while (v < vend) {
      const uint32_t m0 = p->meta[v];
      const int ty = (int)(m0 & 8191) >> lt, tx = (int)((m0 >> 13) & 8191) >> lt;
      Item it{};
      it.tap0 = p->tap_off[v];
      it.v0 = (int32_t)v;
      it.blk = b;
      it.chan = bi.chan;
      it.ty0 = ty * T;
      it.tx0 = tx * T;
      int smax = 1;
      int64_t taps = 0;
      while (v < vend) {
        const uint32_t m = p->meta[v];
        if (((int)(m & 8191) >> lt) != ty || ((int)((m >> 13) & 8191) >> lt) != tx) break;
        const int S = p->S_plan[v];
        if (taps > 0 && taps + (int64_t)S * S > cap_taps) break;
        taps += (int64_t)S * S;
        smax = std::max(smax, S);
        ++v;
      }
      it.v1 = (int32_t)v;
      it.ntap = (int32_t)taps;
      {
        // the gather's waves share the item: give each an equal share of the
        // work, counted as S^2 taps plus 64 per window (the per-window cost of
        // the lane reduction and the G fetch, in tap-equivalents)
        const int64_t total = taps + 64 * (int64_t)(it.v1 - it.v0);
        int64_t acc = 0;
        int64_t m = it.v0;
        for (int w = 1; w < kGatherWaves; ++w) {
          const int64_t target = total * w / kGatherWaves;
          while (m < it.v1 && acc + (int64_t)p->S_plan[m] * p->S_plan[m] + 64 <= target) {
            acc += (int64_t)p->S_plan[m] * p->S_plan[m] + 64;
            ++m;
          }
          it.wv[w - 1] = (int32_t)m;
          it.sub[w - 1] = (int32_t)(p->tap_off[m] - it.tap0);
        }
        for (int w = kGatherWaves; w < 4; ++w) {
          it.wv[w - 1] = it.v1;
          it.sub[w - 1] = (int32_t)taps;
        }
      }
      it.pitch = T + smax - 1;
      it.poff = poff;
      poff += (int64_t)it.pitch * it.pitch;
      max_pitch = std::max(max_pitch, it.pitch);
      it.slot = (int32_t)w.items.size();
      w.items.push_back(it);
    }
    bi.item1 = (int32_t)w.items.size();
    bi.v1 = v;
    w.binfo[b] = bi;
  }
  w.partial_elems = poff;
  w.max_pitch = std::max(max_pitch, T);
  // Pitch classes for the one-pass dual step, each launched with the LDS of
  // its largest pitch.  Pitches are grouped from the smallest up until a
  // class holds a few rounds of work-groups over the whole chip (a smaller
  // launch would be mostly tail); an undersized top class joins the one
  // below.  Inside a class the items run largest first, so the short ones
  // fill the launch's tail.
  {
    constexpr int kMaxP = 256;
    int64_t kMinClassItems = 8 * 256 * 4;  // ~4 rounds of 8 groups on 256 CUs
    if (const char* env = std::getenv("PHI_PITCH_CLASS_ITEMS")) {
      const long v = std::strtol(env, nullptr, 10);
      if (v >= 1) kMinClassItems = v;
    }
    std::vector<int64_t> count(kMaxP, 0);
    for (const Item& it : w.items) ++count[std::min(it.pitch, kMaxP - 1)];
    std::vector<int> class_of(kMaxP, -1);
    std::vector<std::pair<int, int64_t>> classes;  // (pitch of the launch, items)
    std::vector<int> members;
    for (int P = 0; P < kMaxP; ++P) {
      if (!count[P]) continue;
      if (classes.empty() || classes.back().second >= kMinClassItems) classes.push_back({P, 0});
      classes.back().first = P;
      classes.back().second += count[P];
      class_of[P] = (int)classes.size() - 1;
    }
    if (classes.size() > 1 && classes.back().second < kMinClassItems) {
      const int top = (int)classes.size() - 1;
      classes[top - 1].first = classes[top].first;
      for (int P = 0; P < kMaxP; ++P)
        if (class_of[P] == top) class_of[P] = top - 1;
      classes.pop_back();
    }
    auto cls = [&](const Item& it) { return class_of[std::min(it.pitch, kMaxP - 1)]; };
    w.items_by_pitch = w.items;
    std::stable_sort(w.items_by_pitch.begin(), w.items_by_pitch.end(), [&](const Item& x, const Item& y) {
      return cls(x) != cls(y) ? cls(x) > cls(y) : x.ntap > y.ntap;
    });
    for (int32_t i = 0; i < (int32_t)w.items_by_pitch.size();) {
      const int c = cls(w.items_by_pitch[i]);
      int32_t j = i;
      while (j < (int32_t)w.items_by_pitch.size() && cls(w.items_by_pitch[j]) == c) ++j;
      w.pitch_runs.push_back({classes[c].first, i, j});
      i = j;
    }
  }
  // channel item ranges (blocks are channel-major)
  for (int b = 0; b < p->nblk; ++b) w.chan_item0[p->blk_chan[b] + 1] = w.binfo[b].item1;
  for (int l = 0; l < p->L; ++l) w.chan_item0[l + 1] = std::max(w.chan_item0[l + 1], w.chan_item0[l]);
  // merge lists: items by (channel, tile)
  const int nty = p->Ky / T, ntx = p->Kx / T;
  const int64_t ntiles = (int64_t)p->L * nty * ntx;
  w.tile_ptr.assign(ntiles + 1, 0);
  for (const Item& it : w.items) {
    const int64_t t = ((int64_t)it.chan * nty + it.ty0 / T) * ntx + it.tx0 / T;
    w.tile_ptr[t + 1]++;
  }
  for (int64_t t = 0; t < ntiles; ++t) w.tile_ptr[t + 1] += w.tile_ptr[t];
  w.entries.assign(w.items.size(), TileEntry{});
  std::vector<int32_t> fill(w.tile_ptr.begin(), w.tile_ptr.end() - 1);
  for (const Item& it : w.items) {
    const int64_t t = ((int64_t)it.chan * nty + it.ty0 / T) * ntx + it.tx0 / T;
    TileEntry e{};
    e.poff = it.poff;
    e.pitch = it.pitch;
    e.blk = it.blk;
    w.entries[fill[t]++] = e;
  }
  w.halo = (p->smax - 1 + T - 1) / T;
  if (w.halo < 1) w.halo = 1;
  // merge regions of rk x rk tiles at 16-cell tiles, where the tile grid
  // allows: 64 cells wide where that still gives 64K regions or more (each
  // work-group takes four times the cells, so fewer regions leave a longer
  // tail: 16 x 4096^2 workload, 262K regions: 2.39 -> 2.28 ms against
  // 32-cell regions; 16 x 1024^2 workload, 16K: 0.28 -> 0.33 ms), else 32
  // (4.51 -> 3.53 ms against one tile); live regions: those whose merge list
  // (the partials of their own tiles and of the tiles up to `halo` above /
  // left, with wrap) is not empty
  const bool many64 = (int64_t)p->L * (nty / 4) * (ntx / 4) >= 65536;
  const int rk =
      (T == 16 && many64 && nty % 4 == 0 && ntx % 4 == 0 && (4 + w.halo) * (4 + w.halo) <= 25) ? 4
      : (T == 16 && nty % 2 == 0 && ntx % 2 == 0 && (2 + w.halo) * (2 + w.halo) <= 25)         ? 2
                                                                                               : 1;
  w.merge_rk = rk;
  const int nry = nty / rk, nrx = ntx / rk;
  w.live.clear();
  w.chan_live0.assign(p->L + 1, 0);
  for (int l = 0; l < p->L; ++l) {
    for (int ry = 0; ry < nry; ++ry)
      for (int rx = 0; rx < nrx; ++rx) {
        bool any = false;
        for (int dy = -w.halo; dy < rk && !any; ++dy)
          for (int dx = -w.halo; dx < rk && !any; ++dx) {
            const int sty = ((ry * rk + dy) % nty + nty) % nty, stx = ((rx * rk + dx) % ntx + ntx) % ntx;
            const int64_t t = ((int64_t)l * nty + sty) * ntx + stx;
            any = w.tile_ptr[t + 1] > w.tile_ptr[t];
          }
        if (any) w.live.push_back((int32_t)(((int64_t)l * nry + ry) * nrx + rx));
      }
    w.chan_live0[l + 1] = (int32_t)w.live.size();
  }
  // the same regions as bits, one row of words per region row of a channel
  w.live_wpr = (nrx + 31) / 32;
  w.live_bits.assign((size_t)p->L * nry * w.live_wpr, 0u);
  for (int32_t t : w.live) {
    const int64_t row = t / nrx;
    const int rx = (int)(t % nrx);
    w.live_bits[(size_t)row * w.live_wpr + rx / 32] |= 1u << (rx % 32);
  }
}

bool phi_plan_s::fused() const {
  if (!(flags & PHI_FUSED_GH)) return false;
  return gprec == PHI_G_KB ? kb_fused_lds_bytes(W().max_pitch) > 0 : fused_lds_bytes(W().max_pitch) > 0;
}

// Workspace regions of a plan from byte offset `base`; with `share`, the
// grid, half grid, twiddles and Z scales are that plan's (a reduced plan).
static void layout(phi_plan_s* p, size_t base = 0, const phi_plan_s* share = nullptr) {
  size_t o = align_up(base);
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return r;
  };
  // G, then kGPadTaps zero taps: a window's fetch reads 64 * NK taps from its
  // first one, so the last windows read into this pad
  p->off_G = take((size_t)(p->ntaps + kGPadTaps) * p->g_elem_bytes());
  p->off_frac = take(p->gprec == PHI_G_KB ? (size_t)p->M * 8 : 0);  // (kappa - b) per visibility, FP32
  p->off_meta = take((size_t)p->M * 4);
  p->off_perm = take((size_t)p->M * 4);
  size_t n_items = 0, n_tptr = 0, n_part = 0, n_live = 0, n_bits = 0;
  for (const WorkList& w : p->cands) {
    n_items = std::max(n_items, w.items.size());
    n_tptr = std::max(n_tptr, w.tile_ptr.size());
    n_part = std::max(n_part, (size_t)w.partial_elems);
    n_live = std::max(n_live, w.live.size());
    n_bits = std::max(n_bits, w.live_bits.size());
  }
  p->off_live = take(n_live * 4);
  p->off_live_bits = take(n_bits * 4);
  p->off_items = take(n_items * sizeof(Item));
  p->off_items_p = take(n_items * sizeof(Item));
  p->off_binfo = take((size_t)p->nblk * sizeof(BlockInfo));
  p->off_tptr = take(n_tptr * 4);
  p->off_ent = take(n_items * sizeof(TileEntry));
  p->off_theta = take((size_t)p->nblk * 4);
  p->off_part = take(n_part * 8);
  p->off_norms = take(n_items * 16);
  p->off_vscr = take((size_t)p->M * 8);   // scratch visibilities (autotuner, analysis calls)
  p->off_anal = take((size_t)p->L * (2 * kNormChunks + 2) * 8);  // per-channel norm partials, norms
  p->off_scale = take((size_t)p->nblk * 8);
  p->off_bpart = take((size_t)p->nblk * kFinChunks * 16);  // per-block chunk sums of the item norms
  p->off_flag = take(16);
  if (share) {
    // a reduced plan's adjoint runs through the shared grid, every tile written
    p->off_grid = share->off_grid;
    p->off_grid_a = share->off_grid;
    p->sparse_merge = false;
    p->off_half = share->off_half;
    p->off_twx = share->off_twx;
    p->off_twy = share->off_twy;
    p->off_sy = share->off_sy;
    p->off_sx = share->off_sx;
  } else {
    p->off_grid = take((size_t)p->L * p->Ky * p->Kx * 8);
    // an adjoint grid of its own where the inverse transform only reads it
    p->sparse_merge = fft_inverse_reads_grid_only(p->Ky, p->Nx);
    p->off_grid_a = p->sparse_merge ? take((size_t)p->L * p->Ky * p->Kx * 8) : p->off_grid;
    p->off_half = take((size_t)p->L * p->Ny * p->Kx * 8);
    p->off_twx = take((size_t)p->Kx * 8);
    p->off_twy = take((size_t)p->Ky * 8);
    p->off_sy = take((size_t)p->Ny * 4);
    p->off_sx = take((size_t)p->Nx * 4);
  }
  p->ws_bytes = o;
  p->ws_total = o;
}

static hipError_t upload_worklist(phi_plan_s* p, hipStream_t s) {
  const WorkList& w = p->W();
  hipError_t e = hipSuccess;
  auto up = [&](size_t off, const void* src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(p->ws + off, src, n, hipMemcpyHostToDevice, s);
  };
  up(p->off_items, w.items.data(), w.items.size() * sizeof(Item));
  up(p->off_items_p, w.items_by_pitch.data(), w.items_by_pitch.size() * sizeof(Item));
  up(p->off_binfo, w.binfo.data(), w.binfo.size() * sizeof(BlockInfo));
  up(p->off_tptr, w.tile_ptr.data(), w.tile_ptr.size() * 4);
  up(p->off_ent, w.entries.data(), w.entries.size() * sizeof(TileEntry));
  up(p->off_live, w.live.data(), w.live.size() * 4);
  up(p->off_live_bits, w.live_bits.data(), w.live_bits.size() * 4);
  // the adjoint grid starts at zero: the merge of this tiling writes only
  // its live tiles, and no window reaches the others' cells
  if (e == hipSuccess && p->sparse_merge)
    e = hipMemsetAsync(p->ws + p->off_grid_a, 0, (size_t)p->L * p->Ky * p->Kx * 8, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

static void destroy_impl(phi_plan_s* p) {
  if (p->dr) destroy_impl(p->dr);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (hipEvent_t e : p->timer.pool) (void)hipEventDestroy(e);
  delete p;
}

// ------------------------------------------------------------------ ABI
extern "C" {

const char* phi_status_string(phi_status s) {
  switch (s) {
    case PHI_OK: return "ok";
    case PHI_ERR_ARG: return "invalid argument";
    case PHI_ERR_SHAPE: return "inconsistent shape";
    case PHI_ERR_RANGE: return "value out of range";
    case PHI_ERR_WORKSPACE: return "workspace missing or too small";
    case PHI_ERR_NONFINITE: return "non-finite norm";
    case PHI_ERR_HIP: return "HIP runtime error";
    case PHI_ERR_UNSUPPORTED: return "unsupported size";
    case PHI_ERR_STATE: return "plan not ready for this call";
  }
  return "unknown status";
}

phi_status phi_plan_create(const phi_desc* d, phi_plan* out) {
  if (!out) return PHI_ERR_ARG;
  *out = nullptr;
  const phi_status st = validate(d);
  if (st != PHI_OK) return st;
  phi_plan_s* p = new (std::nothrow) phi_plan_s();
  if (!p) return PHI_ERR_ARG;
  p->L = d->n_channels;
  p->Ny = d->ny;
  p->Nx = d->nx;
  p->Ky = 2 * d->ny;
  p->Kx = 2 * d->nx;
  // a plan that also reduces keeps its own G in complex64 whatever g_prec
  // asks for the reduced rows: Lam = H_pp^(-1/2) rescales each gridded row
  // by its window taps at p, and at the support's edge those are the
  // windows' smallest taps, whose relative precision FP16 / BF16 storage
  // would not keep
  p->gprec = (d->flags & PHI_DR) ? (int)PHI_G_C64 : d->g_prec;

  p->flags = d->flags;
  p->persist = d->persist_blocks;
  p->n_blocks.assign(d->h_n_blocks, d->h_n_blocks + p->L);
  for (int l = 0; l < p->L; ++l) {
    p->chan_blk0.push_back(p->nblk);
    for (int b = 0; b < p->n_blocks[l]; ++b) p->blk_chan.push_back(l);
    p->nblk += p->n_blocks[l];
  }
  p->chan_blk0.push_back(p->nblk);
  p->blk_n.assign(d->h_n_vis, d->h_n_vis + p->nblk);
  p->blk_u0.resize(p->nblk);
  int64_t M = 0;
  for (int b = 0; b < p->nblk; ++b) {
    p->blk_u0[b] = M;
    M += p->blk_n[b];
  }
  p->M = M;
  if (p->gprec == PHI_G_KB) {
    // Beatty et al. (2005) shape parameter for width J at 2x oversampling,
    // and 1 / I0(beta) from the power series sum_k ((beta/2)^k / k!)^2 (FP64)
    p->kb_J = M > 0 ? d->h_stencil[0] : 7;
    const double J = p->kb_J;
    p->kb_beta = M_PI * std::sqrt((J / 2.0) * (J / 2.0) * 1.5 * 1.5 - 0.8);
    const double h = p->kb_beta / 2.0;
    double sum = 0.0, term = 1.0;
    for (int k = 0; k < 400; ++k) {
      if (k > 0) term *= (h / k) * (h / k);
      sum += term;
      if (k > 0 && term < 1e-18 * sum) break;
    }
    p->kb_inv_i0b = 1.0 / sum;
  }
  p->theta.assign(p->nblk, 1.0);
  if (d->h_theta) p->theta.assign(d->h_theta, d->h_theta + p->nblk);
  p->sy.assign(d->h_scale_y, d->h_scale_y + p->Ny);
  p->sx.assign(d->h_scale_x, d->h_scale_x + p->Nx);

  // sort every block by the Z-order key of its window origins
  p->perm.resize(M);
  p->meta.resize(M);
  p->S_plan.resize(M);
  std::atomic<int> next{0};
  auto sort_blocks = [&](int64_t, int64_t) {
    std::vector<uint64_t> keys;
    for (int b; (b = next.fetch_add(1)) < p->nblk;) {
      const int64_t u0 = p->blk_u0[b], n = p->blk_n[b];
      keys.resize(n);
      for (int64_t i = 0; i < n; ++i) {
        const int64_t m = u0 + i;
        // Z-order of the 16 x 16 sub-tile, then window size, then the Z-order
        // inside the sub-tile: aligned tiles of 16, 32, 64 stay contiguous and
        // each sub-tile holds runs of equal S
        const uint32_t mo = morton((uint32_t)d->h_base[2 * m], (uint32_t)d->h_base[2 * m + 1]);
        const uint32_t key = ((mo >> 8) << 13) | ((uint32_t)d->h_stencil[m] << 8) | (mo & 0xFFu);
        keys[i] = ((uint64_t)key << 32) | (uint64_t)i;
      }
      std::sort(keys.begin(), keys.end());
      for (int64_t i = 0; i < n; ++i) {
        const int64_t m = u0 + (int64_t)(keys[i] & 0xFFFFFFFFu);
        p->perm[u0 + i] = (int32_t)m;
        const int S = d->h_stencil[m];
        p->S_plan[u0 + i] = (uint8_t)S;
        p->meta[u0 + i] = pack_meta(d->h_base[2 * m], d->h_base[2 * m + 1], S);
      }
    }
  };
  {
    const int nt = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < std::min(nt, std::max(1, p->nblk)); ++t) th.emplace_back(sort_blocks, 0, 0);
    for (auto& x : th) x.join();
  }
  p->tap_off.resize(M + 1);
  p->tap_off[0] = 0;
  for (int64_t i = 0; i < M; ++i) {
    const int S = p->S_plan[i];
    p->tap_off[i + 1] = p->tap_off[i] + (int64_t)S * S;
    p->smax = std::max(p->smax, S);
  }
  p->ntaps = p->tap_off[M];
  for (int T : {16, 32, 64}) {
    if (d->tile && d->tile != T) continue;
    if (p->Ky % T || p->Kx % T) continue;
    p->cands.emplace_back();
    build_worklist(p, T, p->cands.back());
    if (T == (d->tile ? d->tile : 32)) p->cur = (int)p->cands.size() - 1;
  }
  layout(p);
  p->g_loaded.assign(p->nblk, 0);
  for (int b = 0; b < p->nblk; ++b)
    if (p->blk_n[b] == 0) p->g_loaded[b] = 1;
  if (d->flags & PHI_DR) {
    const phi_status sd = dr_build(p, d);
    if (sd != PHI_OK) {
      destroy_impl(p);
      return sd;
    }
    // the reduced plan after this plan's regions, then the set-up tables
    layout(p->dr, p->ws_bytes, p);
    size_t o = align_up(p->dr->ws_bytes);
    p->off_drrow = o;
    o = align_up(o + std::max<size_t>(1, p->drt.rows.size() * sizeof(DrRow)));
    p->off_drgrp = o;
    o = align_up(o + std::max<size_t>(1, p->drt.groups.size() * sizeof(DrGroup)));
    p->off_drcand = o;
    o = align_up(o + std::max<size_t>(1, p->drt.cands.size() * sizeof(DrCand)));
    p->ws_total = o;
  }
  *out = p;
  return PHI_OK;
}

phi_status phi_plan_destroy(phi_plan p) {
  if (!p) return PHI_ERR_ARG;
  if (p->dr_parent) return PHI_ERR_STATE;  // a reduced plan goes with its plan
  destroy_impl(p);
  return PHI_OK;
}

phi_status phi_plan_workspace_size(phi_plan p, size_t* bytes) {
  if (!p || !bytes) return PHI_ERR_ARG;
  if (p->dr_parent) return PHI_ERR_STATE;
  *bytes = p->ws_total;
  return PHI_OK;
}

phi_status phi_plan_get_info(phi_plan p, phi_info* info) {
  if (!p || !info) return PHI_ERR_ARG;
  info->n_vis_total = p->M;
  info->n_taps = p->ntaps;
  info->n_items = (int64_t)p->W().items.size();
  info->n_blocks_total = p->nblk;
  info->g_bytes = (int64_t)(p->ntaps * p->g_elem_bytes());
  info->partial_bytes = p->W().partial_elems * 8;
  info->workspace_bytes = (int64_t)p->ws_bytes;
  const double bG = (double)p->g_elem_bytes();
  const double K = (double)p->Ky * p->Kx, N = (double)p->Ny * p->Nx;
  // G read once per pass, 4 B of metadata per pass, v and y read, c written
  // (gather); c read, v+ written (scatter); grids 48 K + 8 N bytes per channel.
  // the Kaiser-Bessel mode reads 8 B of fractional coordinates per
  // visibility and pass instead of the taps
  const double bV = p->gprec == PHI_G_KB ? 8.0 : 0.0;
  info->alg_bytes_gather = p->ntaps * bG + p->M * (4.0 + bV + 24.0) + p->L * 8.0 * K;
  info->alg_bytes_scatter = p->ntaps * bG + p->M * (4.0 + bV + 16.0);
  info->alg_bytes_dual_step = 2.0 * p->ntaps * bG + p->M * (48.0 + 2.0 * bV) + p->L * (48.0 * K + 8.0 * N);
  // fused dual step: G (or the coordinates) read once; the fused pass moves
  // the gather's bytes, then c is read and v+ written (16 B per visibility)
  if (p->fused())
    info->alg_bytes_dual_step = p->ntaps * bG + p->M * (44.0 + bV) + p->L * (48.0 * K + 8.0 * N);
  info->ky = p->Ky;
  info->kx = p->Kx;
  info->tile = p->W().T;
  info->n_stages = kNumStages;
  info->persist_blocks = (p->flags & PHI_PERSISTENT) ? p->persist : 0;
  info->fused = p->fused() ? 1 : 0;
  info->pitch_classes = (int32_t)p->W().pitch_runs.size();
  info->dr_rows = p->dr ? p->dr->M : 0;
  info->dr_taps = p->dr ? p->dr->ntaps : 0;
  info->dr_bytes = p->dr ? (int64_t)(p->dr->ntaps * p->dr->g_elem_bytes()) : 0;
  info->dr_max_window = p->dr ? p->dr->smax : 0;
  info->reduced = p->dr_parent ? 1 : 0;
  info->fft_image_first = fft_image_first(p->Ky, p->Nx) ? 1 : 0;
  return PHI_OK;
}

#define HIP_TRY(x)                         \
  do {                                     \
    if ((x) != hipSuccess) return PHI_ERR_HIP; \
  } while (0)

static phi_status bind_impl(phi_plan_s* p, void* d_ws, hipStream_t s);

phi_status phi_plan_bind(phi_plan p, void* d_ws, size_t bytes, void* stream) {
  if (!p || !d_ws) return PHI_ERR_ARG;
  if (p->dr_parent) return PHI_ERR_STATE;  // bound with its plan
  if (bytes < p->ws_total || ((uintptr_t)d_ws % kAlign)) return PHI_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  phi_status st;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    st = bind_impl(p, d_ws, s);
  }
  if (st != PHI_OK || !p->dr) return st;
  {
    std::lock_guard<std::mutex> lk(p->dr->mu);
    st = bind_impl(p->dr, d_ws, s);
  }
  if (st != PHI_OK) return st;
  std::lock_guard<std::mutex> lk(p->mu);
  const DrTables& t = p->drt;
  if (!t.rows.empty())
    HIP_TRY(hipMemcpyAsync(p->ws + p->off_drrow, t.rows.data(), t.rows.size() * sizeof(DrRow),
                           hipMemcpyHostToDevice, s));
  if (!t.groups.empty())
    HIP_TRY(hipMemcpyAsync(p->ws + p->off_drgrp, t.groups.data(), t.groups.size() * sizeof(DrGroup),
                           hipMemcpyHostToDevice, s));
  if (!t.cands.empty())
    HIP_TRY(hipMemcpyAsync(p->ws + p->off_drcand, t.cands.data(), t.cands.size() * sizeof(DrCand),
                           hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return PHI_OK;
}

static phi_status bind_impl(phi_plan_s* p, void* d_ws, hipStream_t s) {
  p->ws = (char*)d_ws;
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  std::vector<float> th(p->nblk);
  for (int b = 0; b < p->nblk; ++b) th[b] = (float)p->theta[b];
  std::vector<float> fy(p->Ny), fx(p->Nx);
  for (int i = 0; i < p->Ny; ++i) fy[i] = (float)p->sy[i];
  for (int i = 0; i < p->Nx; ++i) fx[i] = (float)p->sx[i];
  auto tw = [](int n) {
    std::vector<float2> t(n);
    for (int m = 0; m < n; ++m) {
      const double a = -2.0 * M_PI * (double)m / (double)n;
      t[m] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    return t;
  };
  const std::vector<float2> twx = tw(p->Kx), twy = tw(p->Ky);
  auto up = [&](size_t off, const void* src, size_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(p->ws + off, src, n, hipMemcpyHostToDevice, s);
  };
  HIP_TRY(up(p->off_meta, p->meta.data(), p->meta.size() * 4));
  HIP_TRY(up(p->off_perm, p->perm.data(), p->perm.size() * 4));
  HIP_TRY(upload_worklist(p, s));
  HIP_TRY(up(p->off_theta, th.data(), th.size() * 4));
  HIP_TRY(up(p->off_twx, twx.data(), twx.size() * 8));
  HIP_TRY(up(p->off_twy, twy.data(), twy.size() * 8));
  HIP_TRY(up(p->off_sy, fy.data(), fy.size() * 4));
  HIP_TRY(up(p->off_sx, fx.data(), fx.size() * 4));
  const int zero[4] = {0, 0, 0, 0};
  HIP_TRY(up(p->off_flag, zero, sizeof(zero)));
  if (p->g_elem_bytes())
    HIP_TRY(hipMemsetAsync(p->ws + p->off_G + p->ntaps * p->g_elem_bytes(), 0, kGPadTaps * p->g_elem_bytes(), s));
  HIP_TRY(hipStreamSynchronize(s));  // host vectors above are temporaries
  if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  p->bound = true;
  return PHI_OK;
}

phi_status phi_plan_set_theta(phi_plan p, const double* h_theta, void* stream) {
  if (!p || !h_theta) return PHI_ERR_ARG;
  for (int b = 0; b < p->nblk; ++b)
    if (!(h_theta[b] > 0.0) || !std::isfinite(h_theta[b])) return PHI_ERR_RANGE;
  if (p->dr) {  // the reduced plan whitens its blocks with the same theta
    const phi_status st = phi_plan_set_theta(p->dr, h_theta, stream);
    if (st != PHI_OK) return st;
  }
  p->theta.assign(h_theta, h_theta + p->nblk);
  if (!p->bound) return PHI_OK;
  std::vector<float> th(p->nblk);
  for (int b = 0; b < p->nblk; ++b) th[b] = (float)p->theta[b];
  HIP_TRY(hipMemcpyAsync(p->ws + p->off_theta, th.data(), th.size() * 4, hipMemcpyHostToDevice,
                         (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return PHI_OK;
}

phi_status phi_plan_load_kb(phi_plan p, int64_t block, const double* h_kappa, void* stream) {
  if (!p) return PHI_ERR_ARG;
  if (block < 0 || block >= p->nblk) return PHI_ERR_RANGE;
  if (p->gprec != PHI_G_KB || !p->bound || p->dr_parent) return PHI_ERR_STATE;
  const int64_t u0 = p->blk_u0[block], n = p->blk_n[block];
  if (n == 0) {
    p->g_loaded[block] = 1;
    return PHI_OK;
  }
  if (!h_kappa) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  hipStream_t s = (hipStream_t)stream;
  float2* stage = nullptr;
  HIP_TRY(hipHostMalloc((void**)&stage, (size_t)n * sizeof(float2), hipHostMallocDefault));
  const double half = p->kb_J / 2.0;
  std::atomic<int> bad{0};
  parallel_for(n, [&](int64_t a, int64_t b) {
    for (int64_t k = a; k < b; ++k) {
      const int64_t ui = p->perm[u0 + k] - u0;  // user index inside the block
      const double ky = h_kappa[2 * ui], kx = h_kappa[2 * ui + 1];
      if (!std::isfinite(ky) || !std::isfinite(kx) || std::fabs(ky) > 1e7 || std::fabs(kx) > 1e7) {
        bad = 1;
        continue;
      }
      // window origin b = floor(kappa - J/2) + 1 must be the one given at
      // plan creation (mod K); the kernels see only kappa - b
      const double by = std::floor(ky - half) + 1.0, bx = std::floor(kx - half) + 1.0;
      const int64_t my = (((int64_t)by % p->Ky) + p->Ky) % p->Ky, mx = (((int64_t)bx % p->Kx) + p->Kx) % p->Kx;
      const uint32_t m = p->meta[u0 + k];
      if (my != (int64_t)(m & 8191) || mx != (int64_t)((m >> 13) & 8191)) {
        bad = 1;
        continue;
      }
      stage[k] = make_float2((float)(ky - by), (float)(kx - bx));
    }
  });
  phi_status rc = PHI_OK;
  if (bad) {
    rc = PHI_ERR_RANGE;
  } else if (hipMemcpyAsync(p->ws + p->off_frac + (size_t)u0 * sizeof(float2), stage, (size_t)n * sizeof(float2),
                            hipMemcpyHostToDevice, s) != hipSuccess ||
             hipStreamSynchronize(s) != hipSuccess) {
    rc = PHI_ERR_HIP;
  }
  (void)hipHostFree(stage);
  if (rc == PHI_OK) p->g_loaded[block] = 1;
  return rc;
}

phi_status phi_plan_load_g(phi_plan p, int64_t block, const void* h_windows, int32_t host_type, void* stream) {
  if (!p) return PHI_ERR_ARG;
  if (block < 0 || block >= p->nblk) return PHI_ERR_RANGE;
  if (p->gprec == PHI_G_KB || p->dr_parent) return PHI_ERR_STATE;  // reduced rows come from phi_dr_setup
  if (!h_windows && p->blk_n[block] > 0) return PHI_ERR_ARG;
  if (host_type != PHI_HOST_C128 && host_type != PHI_HOST_C64) return PHI_ERR_ARG;
  if (!p->bound) return PHI_ERR_STATE;
  std::lock_guard<std::mutex> lk(p->mu);
  hipStream_t s = (hipStream_t)stream;
  const int64_t u0 = p->blk_u0[block], n = p->blk_n[block];
  if (n == 0) {
    p->g_loaded[block] = 1;
    return PHI_OK;
  }
  // user-order window offsets inside the block
  std::vector<int64_t> uoff(n + 1, 0);
  std::vector<int32_t> uS(n);
  {
    // S in user order: invert the block's permutation
    for (int64_t k = 0; k < n; ++k) uS[p->perm[u0 + k] - u0] = p->S_plan[u0 + k];
    for (int64_t i = 0; i < n; ++i) uoff[i + 1] = uoff[i] + (int64_t)uS[i] * uS[i];
  }
  const size_t eb = p->g_elem_bytes();
  const int64_t tap_begin = p->tap_off[u0];
  const int64_t tap_total = p->tap_off[u0 + n] - tap_begin;
  const int64_t stage_taps = std::min<int64_t>(tap_total, (int64_t)(64 << 20) / (int64_t)eb);
  void* stage = nullptr;
  HIP_TRY(hipHostMalloc(&stage, (size_t)stage_taps * eb, hipHostMallocDefault));
  phi_status rc = PHI_OK;
  int64_t k = 0;
  while (k < n && rc == PHI_OK) {
    // plan positions [k, k2) whose taps fit in the staging buffer
    int64_t k2 = k;
    while (k2 < n && p->tap_off[u0 + k2 + 1] - p->tap_off[u0 + k] <= stage_taps) ++k2;
    if (k2 == k) {
      rc = PHI_ERR_ARG;
      break;
    }
    const int64_t t0 = p->tap_off[u0 + k];
    parallel_for(k2 - k, [&](int64_t a, int64_t b) {
      for (int64_t i = k + a; i < k + b; ++i) {
        const int64_t ui = p->perm[u0 + i] - u0;
        const int64_t cnt = uoff[ui + 1] - uoff[ui];
        const int64_t dst0 = p->tap_off[u0 + i] - t0;
        for (int64_t e = 0; e < cnt; ++e) {
          double re, im;
          if (host_type == PHI_HOST_C128) {
            const double* src = static_cast<const double*>(h_windows) + 2 * (uoff[ui] + e);
            re = src[0];
            im = src[1];
          } else {
            const float* src = static_cast<const float*>(h_windows) + 2 * (uoff[ui] + e);
            re = src[0];
            im = src[1];
          }
          const int64_t di = dst0 + e;
          if (p->gprec == PHI_G_C64) {
            float* o = static_cast<float*>(stage) + 2 * di;
            o[0] = (float)re;
            o[1] = (float)im;
          } else if (p->gprec == PHI_G_F16) {
            _Float16* o = static_cast<_Float16*>(stage) + 2 * di;
            o[0] = (_Float16)re;
            o[1] = (_Float16)im;
          } else {
            uint16_t* o = static_cast<uint16_t*>(stage) + 2 * di;
            o[0] = f64_to_bf16_rne(re);
            o[1] = f64_to_bf16_rne(im);
          }
        }
      }
    });
    const int64_t t1 = p->tap_off[u0 + k2];
    if (hipMemcpyAsync(p->ws + p->off_G + (size_t)t0 * eb, stage, (size_t)(t1 - t0) * eb, hipMemcpyHostToDevice,
                       s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = PHI_ERR_HIP;
    k = k2;
  }
  (void)tap_begin;
  (void)hipHostFree(stage);
  if (rc == PHI_OK) p->g_loaded[block] = 1;
  return rc;
}

phi_status phi_to_plan_order(phi_plan p, const void* d_user, void* d_plan, void* stream) {
  if (!p || (p->M > 0 && (!d_user || !d_plan))) return PHI_ERR_ARG;
  if (!p->bound) return PHI_ERR_STATE;
  HIP_TRY(launch_permute((const float2*)d_user, (float2*)d_plan, p->at<int32_t>(p->off_perm), p->M, 1,
                         (hipStream_t)stream));
  return PHI_OK;
}

phi_status phi_from_plan_order(phi_plan p, const void* d_plan, void* d_user, void* stream) {
  if (!p || (p->M > 0 && (!d_user || !d_plan))) return PHI_ERR_ARG;
  if (!p->bound) return PHI_ERR_STATE;
  HIP_TRY(launch_permute((const float2*)d_plan, (float2*)d_user, p->at<int32_t>(p->off_perm), p->M, 0,
                         (hipStream_t)stream));
  return PHI_OK;
}

}  // extern "C"

// ------------------------------------------------------------- execution
namespace {

struct Runner {
  phi_plan_s* p;
  hipStream_t s;
  bool timed;
  hipError_t err = hipSuccess;

  GArgs gargs() const {
    GArgs a;
    a.items = p->at<Item>(p->off_items);
    a.meta = p->at<uint32_t>(p->off_meta);
    a.G = p->ws + p->off_G;
    a.theta = p->at<float>(p->off_theta);
    a.sigma = nullptr;
    a.scale = p->at<double>(p->off_scale);
    a.grid = p->at<float2>(p->off_grid);
    a.Ky = p->Ky;
    a.Kx = p->Kx;
    a.T = p->W().T;
    a.frac = p->gprec == PHI_G_KB ? p->at<float2>(p->off_frac) : nullptr;
    a.kb_J = p->kb_J;
    a.kb_beta = (float)p->kb_beta;
    a.kb_inv_i0b = (float)p->kb_inv_i0b;
    a.partials = p->at<float2>(p->off_part);
    return a;
  }
  int persist_blocks() const {
    if (!(p->flags & PHI_PERSISTENT)) return 0;
    if (p->persist > 0) return p->persist;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return 4 * cus;
  }
  template <typename F>
  void stage(int id, F&& f) {
    if (err != hipSuccess) return;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
      e0 = p->timer.get();
      e1 = p->timer.get();
      if (e0) (void)hipEventRecord(e0, s);
    }
    err = f();
    if (timed && e1) {
      (void)hipEventRecord(e1, s);
      p->timer.pending.push_back({id, {e0, e1}});
    }
  }
  // The merge regions some partial reaches, as bits, where the sparse merge
  // runs (the adjoint grid is zero elsewhere); else none (every cell).
  LiveRegions live_regions() const {
    const WorkList& w = p->W();
    return LiveRegions{p->sparse_merge ? p->at<uint32_t>(p->off_live_bits) : nullptr, w.merge_rk * w.T, w.live_wpr};
  }
  // channel range [l0, l1), matching block and item ranges
  void fwd_fft(const float* x, int l0, int l1) {
    const int nl = l1 - l0;
    if (fft_image_first(p->Ky, p->Nx)) {
      // columns of the image first (packed columns in the grid buffer, T in
      // the half grid), then the Ky rows of T into the grid
      stage(1, [&] {
        return launch_colr_fwd(p->Ky, x, p->at<float2>(p->off_grid), p->at<float2>(p->off_half),
                               p->at<float>(p->off_sy), p->at<float>(p->off_sx), p->at<float2>(p->off_twy), p->Ny,
                               p->Nx, l0, nl, s);
      });
      stage(0, [&] {
        return launch_rowc_fwd(p->Kx, p->at<float2>(p->off_half), p->at<float2>(p->off_grid),
                               p->at<float2>(p->off_twx), p->Ky, l0, nl, s);
      });
      return;
    }
    stage(0, [&] {
      return launch_rowfft_fwd(p->Kx, x, p->at<float2>(p->off_half), p->at<float>(p->off_sy),
                               p->at<float>(p->off_sx), p->at<float2>(p->off_twx), p->Ny, p->Nx, l0, nl, s);
    });
    stage(1, [&] {
      return launch_colfft_fwd(p->Ky, p->at<float2>(p->off_half), p->at<float2>(p->off_grid),
                               p->at<float2>(p->off_twy), p->Ny, p->Kx, l0, nl, s);
    });
  }
  // The merge of channels [l0, l1) into the adjoint grid: the live tiles
  // only (sparse merge), else every tile.
  hipError_t merge(int l0, int l1, const double* msig, const double* mscale) const {
    const WorkList& w = p->W();
    const int32_t* live = p->sparse_merge ? p->at<int32_t>(p->off_live) : nullptr;
    const int lb = live ? w.chan_live0[l0] : 0, ln = live ? w.chan_live0[l1] - w.chan_live0[l0] : 0;
    return launch_merge(p->at<float2>(p->off_grid_a), p->at<float2>(p->off_part), p->at<int32_t>(p->off_tptr),
                        p->at<TileEntry>(p->off_ent), live, lb, ln, p->Ky, p->Kx, w.T, w.halo, w.merge_rk, l0,
                        l1 - l0, msig, mscale, p->at<float>(p->off_theta), s);
  }
  // msig / mscale: per-block merge factors after the fused dual step (null: 1)
  void adj_fft(float* x, int l0, int l1, const double* msig = nullptr, const double* mscale = nullptr) {
    const int nl = l1 - l0;
    stage(5, [&] { return merge(l0, l1, msig, mscale); });
    if (fft_image_first(p->Ky, p->Nx)) {
      // rows first (the Nx kept columns into the half grid), then the image's
      // columns (packed columns in the grid buffer), real part, Z^T
      // with the sparse merge, the row pass reads only the live regions'
      // cells (the others are zero)
      stage(7, [&] {
        return launch_rowc_inv(p->Kx, p->at<float2>(p->off_grid_a), p->at<float2>(p->off_half),
                               p->at<float2>(p->off_twx), p->Ky, l0, nl, live_regions(), s);
      });
      stage(6, [&] {
        return launch_colr_inv(p->Ky, p->at<float2>(p->off_half), p->at<float2>(p->off_grid), x,
                               p->at<float>(p->off_sy), p->at<float>(p->off_sx), p->at<float2>(p->off_twy), p->Ny,
                               p->Nx, l0, nl, s);
      });
      return;
    }
    stage(6, [&] {
      return launch_colfft_inv(p->Ky, p->at<float2>(p->off_grid_a), p->at<float2>(p->off_half),
                               p->at<float2>(p->off_twy), p->Ny, p->Kx, l0, nl, s);
    });
    stage(7, [&] {
      return launch_rowfft_inv(p->Kx, p->at<float2>(p->off_half), x, p->at<float>(p->off_sy),
                               p->at<float>(p->off_sx), p->at<float2>(p->off_twx), p->Ny, p->Nx, l0, nl, s);
    });
  }
  // A G stage over channels [l0, l1).  The one-pass dual step (by_pitch)
  // over all channels runs once per pitch class, on the items grouped by
  // pitch with the largest first, each launch with the LDS of its class: its
  // occupancy is set by LDS, so items with smaller windows fit more
  // work-groups per compute unit, and short items fill each launch's tail.
  // Everything else runs its items in plan order in one launch (the two-pass
  // kernels measured slower by pitch class: they gain no occupancy and lose
  // the locality of neighbouring items).  launch(args, pitch, first, end).
  template <typename F>
  hipError_t g_stage(const GArgs& a, int l0, int l1, bool by_pitch, F&& launch) {
    if (by_pitch && l0 == 0 && l1 == p->L && p->gprec != PHI_G_KB) {
      GArgs b = a;
      b.items = p->at<Item>(p->off_items_p);
      for (const auto& r : p->W().pitch_runs) {
        const hipError_t e = launch(b, r[0], r[1], r[2]);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    }
    return launch(a, p->W().max_pitch, p->W().chan_item0[l0], p->W().chan_item0[l1]);
  }
  hipError_t gather(int mode, const GArgs& a, float2* v, const float2* y, int l0, int l1) {
    double* norms = mode ? p->at<double>(p->off_norms) : nullptr;
    return g_stage(a, l0, l1, mode == 2, [&](const GArgs& b, int P, int i0, int i1) {
      return launch_gather(p->gprec, mode, b, v, y, norms, P, i0, i1, persist_blocks(), s);
    });
  }
  hipError_t scatter(int mode, const GArgs& a, float2* v, int l0, int l1) {
    return g_stage(a, l0, l1, false, [&](const GArgs& b, int P, int i0, int i1) {
      return launch_scatter(p->gprec, mode, b, v, p->at<float2>(p->off_part), P, i0, i1, persist_blocks(), s);
    });
  }
  void forward(const float* x, float2* y, int l0, int l1) {
    fwd_fft(x, l0, l1);
    const GArgs a = gargs();
    stage(2, [&] { return gather(0, a, y, nullptr, l0, l1); });
  }
  void adjoint(const float2* v, float* x, int l0, int l1) {
    const GArgs a = gargs();
    stage(4, [&] { return scatter(0, a, const_cast<float2*>(v), l0, l1); });
    adj_fft(x, l0, l1);
  }
  void dual(const float* xt, float2* v, const float2* y, const double* eps, const double* sigma, float* grad,
            double* rho, double* res, int l0, int l1) {
    fwd_fft(xt, l0, l1);
    GArgs a = gargs();
    a.sigma = sigma;
    const int b0 = p->chan_blk0[l0], b1 = p->chan_blk0[l1];
    if (p->fused()) {
      // c and G^H c in one pass over G; once the norms are known the
      // per-block factor sigma * scale goes into v+, and times theta into
      // the merge
      stage(10, [&] { return gather(2, a, v, y, l0, l1); });
      stage(3, [&] {
        return launch_finalize(p->at<double>(p->off_norms), p->at<BlockInfo>(p->off_binfo),
                               p->at<double>(p->off_bpart), eps, rho, res, p->at<double>(p->off_scale),
                               p->at<int>(p->off_flag), b0, b1 - b0, s);
      });
      stage(11, [&] {
        return launch_vscale(p->at<BlockInfo>(p->off_binfo), v, sigma, p->at<double>(p->off_scale), b0, b1 - b0, s);
      });
      adj_fft(grad, l0, l1, sigma, p->at<double>(p->off_scale));
      return;
    }
    stage(2, [&] { return gather(1, a, v, y, l0, l1); });
    stage(3, [&] {
      return launch_finalize(p->at<double>(p->off_norms), p->at<BlockInfo>(p->off_binfo),
                             p->at<double>(p->off_bpart), eps, rho, res,
                             p->at<double>(p->off_scale), p->at<int>(p->off_flag), b0, b1 - b0, s);
    });
    stage(4, [&] { return scatter(1, a, v, l0, l1); });
    adj_fft(grad, l0, l1);
  }
};

phi_status ready(phi_plan p) {
  if (!p) return PHI_ERR_ARG;
  if (!p->bound) return PHI_ERR_STATE;
  for (char c : p->g_loaded)
    if (!c) return PHI_ERR_STATE;
  return PHI_OK;
}

template <typename F>
phi_status run_channels(phi_plan p, hipStream_t s, F&& body) {
  Runner r{p, s, p->timing};
  if (p->flags & PHI_PER_CHANNEL) {
    for (int l = 0; l < p->L && r.err == hipSuccess; ++l) body(r, l, l + 1);
  } else {
    body(r, 0, p->L);
  }
  if (p->timing) p->timer.calls++;
  return r.err == hipSuccess ? PHI_OK : PHI_ERR_HIP;
}

}  // namespace

extern "C" {

phi_status phi_forward(phi_plan p, const float* d_x, void* d_y, void* stream) {
  const phi_status st = ready(p);
  if (st != PHI_OK) return st;
  if (!d_x || (p->M > 0 && !d_y)) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  return run_channels(p, (hipStream_t)stream,
                      [&](Runner& r, int l0, int l1) { r.forward(d_x, (float2*)d_y, l0, l1); });
}

phi_status phi_adjoint(phi_plan p, const void* d_v, float* d_x, void* stream) {
  const phi_status st = ready(p);
  if (st != PHI_OK) return st;
  if (!d_x || (p->M > 0 && !d_v)) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  return run_channels(p, (hipStream_t)stream,
                      [&](Runner& r, int l0, int l1) { r.adjoint((const float2*)d_v, d_x, l0, l1); });
}

phi_status l2ball_dual_step(phi_plan p, const float* d_xt, void* d_v, const void* d_y, const double* d_eps,
                            const double* d_sigma, float* d_grad, double* d_rho, double* d_res, void* stream) {
  const phi_status st = ready(p);
  if (st != PHI_OK) return st;
  if (!d_xt || !d_grad || !d_eps || (p->M > 0 && (!d_v || !d_y))) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  hipStream_t s = (hipStream_t)stream;
  auto body = [&](Runner& r, int l0, int l1) {
    r.dual(d_xt, (float2*)d_v, (const float2*)d_y, d_eps, d_sigma, d_grad, d_rho, d_res, l0, l1);
  };
  if ((p->flags & PHI_GRAPH) && !p->timing) {
    const void* key[9] = {d_xt, d_v, d_y, d_eps, d_sigma, d_grad, d_rho, d_res, stream};
    if (!p->gexec || std::memcmp(key, p->gkey, sizeof(key)) != 0) {
      if (p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
      }
      // capture on the plan's own stream, ordered after the caller's stream
      hipEvent_t ev;
      HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      (void)hipEventRecord(ev, s);
      (void)hipStreamWaitEvent(p->cap_stream, ev, 0);
      (void)hipEventDestroy(ev);
      HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
      Runner r{p, p->cap_stream, false};
      if (p->flags & PHI_PER_CHANNEL) {
        for (int l = 0; l < p->L && r.err == hipSuccess; ++l) body(r, l, l + 1);
      } else {
        body(r, 0, p->L);
      }
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(p->cap_stream, &g);
      if (r.err != hipSuccess || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return PHI_ERR_HIP;
      }
      const hipError_t ei = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        p->gexec = nullptr;
        return PHI_ERR_HIP;
      }
      std::memcpy(p->gkey, key, sizeof(key));
    }
    HIP_TRY(hipGraphLaunch(p->gexec, s));
    return PHI_OK;
  }
  return run_channels(p, s, body);
}

phi_status phi_plan_check(phi_plan p, void* stream) {
  if (!p) return PHI_ERR_ARG;
  if (!p->bound) return PHI_ERR_STATE;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  int flag[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpy(flag, p->ws + p->off_flag, sizeof(flag), hipMemcpyDeviceToHost));
  if (flag[0]) {
    const int zero[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpy(p->ws + p->off_flag, zero, sizeof(zero), hipMemcpyHostToDevice));
    return PHI_ERR_NONFINITE;
  }
  return PHI_OK;
}

phi_status phi_plan_set_flags(phi_plan p, int32_t flags) {
  if (!p) return PHI_ERR_ARG;
  if (flags & ~(PHI_PER_CHANNEL | PHI_GRAPH | PHI_PERSISTENT | PHI_FUSED_GH | PHI_DR)) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  p->flags = (flags & ~PHI_DR) | (p->flags & PHI_DR);  // PHI_DR is fixed at creation
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  return PHI_OK;
}

phi_status phi_plan_set_tuning(phi_plan p, int32_t tile, int32_t persist_blocks, void* stream) {
  if (!p) return PHI_ERR_ARG;
  if (persist_blocks < 0) return PHI_ERR_ARG;
  int c = -1;
  for (int i = 0; i < (int)p->cands.size(); ++i)
    if (p->cands[i].T == tile) c = i;
  if (c < 0) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  p->persist = persist_blocks;
  p->flags = persist_blocks ? (p->flags | PHI_PERSISTENT) : (p->flags & ~PHI_PERSISTENT);
  if (c != p->cur) {
    p->cur = c;
    if (p->bound && upload_worklist(p, (hipStream_t)stream) != hipSuccess) return PHI_ERR_HIP;
  }
  return PHI_OK;
}

phi_status phi_plan_set_timing(phi_plan p, int32_t enable) {
  if (!p) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  p->timing = enable != 0;
  return PHI_OK;
}

phi_status phi_plan_get_timing(phi_plan p, int32_t max_stages, double* ms, const char** names, int32_t* n_stages,
                               int64_t* n_calls) {
  if (!p) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  for (auto& pe : p->timer.pending) {
    HIP_TRY(hipEventSynchronize(pe.second.second));
    float t = 0.f;
    if (hipEventElapsedTime(&t, pe.second.first, pe.second.second) == hipSuccess) p->timer.ms[pe.first] += t;
  }
  p->timer.pending.clear();
  p->timer.next = 0;
  const int n = std::min<int>(max_stages, kNumStages);
  for (int i = 0; i < n; ++i) {
    if (ms) ms[i] = p->timer.ms[i];
    if (names) names[i] = kStageNames[i];
  }
  if (n_stages) *n_stages = kNumStages;
  if (n_calls) *n_calls = p->timer.calls;
  for (double& v : p->timer.ms) v = 0.0;
  p->timer.calls = 0;
  return PHI_OK;
}

phi_status phi_plan_autotune(phi_plan p, void* stream, int32_t reps) {
  const phi_status st = ready(p);
  if (st != PHI_OK) return st;
  std::lock_guard<std::mutex> lk(p->mu);
  hipStream_t s = (hipStream_t)stream;
  if (reps < 1) reps = 3;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  // finite grid values for the timed gathers (contents are otherwise unused)
  HIP_TRY(hipMemsetAsync(p->ws + p->off_grid, 0, (size_t)p->L * p->Ky * p->Kx * 8, s));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int saved_flags = p->flags, saved_persist = p->persist;
  float2* vs = p->at<float2>(p->off_vscr);
  // time `reps` rounds of the selected G stages with the current settings
  // (fused: the one-pass dual-step kernel instead of the two passes, on the
  // scratch visibilities as both v and y; the values it writes are unused)
  auto time_stages = [&](bool g, bool sc, double& ms_out, bool fused = false) -> bool {
    Runner r{p, s, false};
    auto once = [&] {
      const GArgs a = r.gargs();
      if (fused && r.err == hipSuccess) r.err = r.gather(2, a, vs, vs, 0, p->L);
      if (!fused && g && r.err == hipSuccess) r.err = r.gather(0, a, vs, nullptr, 0, p->L);
      if (!fused && sc && r.err == hipSuccess) r.err = r.scatter(0, a, vs, 0, p->L);
      if ((sc || fused) && r.err == hipSuccess) r.err = r.merge(0, p->L, nullptr, nullptr);
    };
    once();
    (void)hipEventRecord(e0, s);
    for (int k = 0; k < reps && r.err == hipSuccess; ++k) once();
    (void)hipEventRecord(e1, s);
    float ms = 0.f;
    if (r.err != hipSuccess || hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return false;
    ms_out = ms;
    return true;
  };
  double best = 1e30;
  int best_c = p->cur, best_p = 0;
  bool best_one = false;
  phi_status rc = PHI_OK;
  // tile edge x launch shape x (two passes, or one pass where its LDS fits):
  // the fastest of all (a tile that loses in two passes may win in one)
  for (int c = 0; c < (int)p->cands.size() && rc == PHI_OK; ++c) {
    p->cur = c;
    if (upload_worklist(p, s) != hipSuccess) {
      rc = PHI_ERR_HIP;
      break;
    }
    const bool one_fits = p->gprec == PHI_G_KB ? kb_fused_lds_bytes(p->W().max_pitch) > 0
                                               : fused_lds_bytes(p->W().max_pitch) > 0;
    for (int pb : {0, 4 * cus}) {
      p->persist = pb;
      p->flags = (pb ? (saved_flags | PHI_PERSISTENT) : (saved_flags & ~PHI_PERSISTENT)) & ~PHI_FUSED_GH;
      for (bool one : {false, true}) {
        if (one && !one_fits) continue;
        double ms = 0;
        if (!(one ? time_stages(false, false, ms, true) : time_stages(true, true, ms))) {
          rc = PHI_ERR_HIP;
          break;
        }
        if (ms < best) {
          best = ms;
          best_c = c;
          best_p = pb;
          best_one = one;
        }
      }
      if (rc != PHI_OK) break;
    }
  }
  p->cur = best_c;
  p->persist = best_p ? best_p : saved_persist;
  p->flags = best_p ? (saved_flags | PHI_PERSISTENT) : (saved_flags & ~PHI_PERSISTENT);
  p->flags = best_one ? (p->flags | PHI_FUSED_GH) : (p->flags & ~PHI_FUSED_GH);
  if (rc == PHI_OK && upload_worklist(p, s) != hipSuccess) rc = PHI_ERR_HIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}


// ------------------------------------------------------- analysis calls
// Phi_l^dagger Phi_l x for every channel into out (visibility scratch between)
static hipError_t normal_op(phi_plan_s* p, hipStream_t s, const float* x, float* out) {
  float2* vs = p->at<float2>(p->off_vscr);
  Runner r{p, s, false};
  if (p->flags & PHI_PER_CHANNEL) {
    for (int l = 0; l < p->L && r.err == hipSuccess; ++l) {
      r.forward(x, vs, l, l + 1);
      r.adjoint(vs, out, l, l + 1);
    }
  } else {
    r.forward(x, vs, 0, p->L);
    r.adjoint(vs, out, 0, p->L);
  }
  return r.err;
}

phi_status phi_psf(phi_plan p, float* d_psf, double* d_peak, void* stream) {
  const phi_status st = ready(p);
  if (st != PHI_OK) return st;
  if (!d_psf) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  hipStream_t s = (hipStream_t)stream;
  // delta into the output buffer, then Phi^dagger Phi in place (the forward
  // pass has read x before the adjoint writes)
  HIP_TRY(launch_delta(d_psf, p->L, p->Ny, p->Nx, s));
  HIP_TRY(normal_op(p, s, d_psf, d_psf));
  if (d_peak) HIP_TRY(launch_centre_value(d_psf, p->L, p->Ny, p->Nx, d_peak, s));
  return PHI_OK;
}

phi_status phi_residual_image(phi_plan p, const float* d_x, const void* d_y, const double* d_eta, float* d_r,
                              void* stream) {
  const phi_status st = ready(p);
  if (st != PHI_OK) return st;
  if (!d_x || !d_r || (p->M > 0 && !d_y)) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  hipStream_t s = (hipStream_t)stream;
  float2* vs = p->at<float2>(p->off_vscr);
  Runner r{p, s, false};
  auto body = [&](int l0, int l1) {
    r.forward(d_x, vs, l0, l1);
    if (r.err == hipSuccess) r.err = launch_vis_residual(vs, (const float2*)d_y, p->M, s);
    r.adjoint(vs, d_r, l0, l1);
  };
  if (p->flags & PHI_PER_CHANNEL) {
    // the residual kernel covers every visibility; run it once, after all forwards
    for (int l = 0; l < p->L && r.err == hipSuccess; ++l) r.forward(d_x, vs, l, l + 1);
    if (r.err == hipSuccess) r.err = launch_vis_residual(vs, (const float2*)d_y, p->M, s);
    for (int l = 0; l < p->L && r.err == hipSuccess; ++l) r.adjoint(vs, d_r, l, l + 1);
  } else {
    body(0, p->L);
  }
  if (r.err != hipSuccess) return PHI_ERR_HIP;
  if (d_eta) HIP_TRY(launch_chan_scale(d_r, d_eta, p->L, (int64_t)p->Ny * p->Nx, s));
  return PHI_OK;
}

phi_status phi_power_iteration(phi_plan p, float* d_x, float* d_tmp, int32_t n_iter, double* d_nu, void* stream) {
  return power_iteration_impl(p, d_x, d_tmp, n_iter, d_nu, stream);
}

}  // extern "C"

phi_status power_iteration_impl(phi_plan_s* p, float* d_x, float* d_tmp, int32_t n_iter, double* d_nu,
                                void* stream) {
  const phi_status st = ready(p);
  if (st != PHI_OK) return st;
  if (!d_x || !d_tmp || !d_nu || d_x == d_tmp) return PHI_ERR_ARG;
  if (n_iter < 1) return PHI_ERR_RANGE;
  std::lock_guard<std::mutex> lk(p->mu);
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = (int64_t)p->Ny * p->Nx;
  double* part = p->at<double>(p->off_anal);
  double* inv = part + (size_t)p->L * kNormChunks;
  float* a = d_x;
  float* b = d_tmp;
  HIP_TRY(launch_chan_norm(a, p->L, n, part, nullptr, inv, s));
  HIP_TRY(launch_chan_scale(a, inv, p->L, n, s));
  for (int k = 0; k < n_iter; ++k) {
    HIP_TRY(normal_op(p, s, a, b));
    HIP_TRY(launch_chan_norm(b, p->L, n, part, d_nu, inv, s));
    HIP_TRY(launch_chan_scale(b, inv, p->L, n, s));
    std::swap(a, b);
  }
  if (a != d_x) HIP_TRY(hipMemcpyAsync(d_x, a, (size_t)p->L * n * sizeof(float), hipMemcpyDeviceToDevice, s));
  return PHI_OK;
}

extern "C" {

// ------------------------------------------------------------- PDFB loop
static bool rule_ok(const phi_eps_rule* r) {
  const double v[4] = {r->lambda_lo, r->lambda_hi, r->lambda_mix, r->var_tol};
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return r->lambda_lo > 0.0 && r->lambda_lo <= 1.0 && r->lambda_hi >= 1.0 && r->lambda_mix > 0.0 &&
         r->lambda_mix <= 1.0 && r->var_tol >= 0.0 && r->min_gap >= 0;
}

static phi_status primal_locked(phi_plan_s* p, hipStream_t s, float* d_x, float* d_xt, const float* d_grad,
                                const double* d_tau, double* d_var) {
  Runner r{p, s, p->timing};
  r.stage(8, [&] {
    return launch_pdfb_primal(d_x, d_xt, d_grad, d_tau, p->L, (int64_t)p->Ny * p->Nx,
                              p->at<double>(p->off_anal), d_var, s);
  });
  return r.err == hipSuccess ? PHI_OK : PHI_ERR_HIP;
}

static phi_status eps_locked(phi_plan_s* p, hipStream_t s, const double* d_res, const double* d_var,
                             const phi_eps_rule* rule, double* d_eps, int32_t* d_state) {
  EpsRule er;
  er.lo = rule->lambda_lo;
  er.hi = rule->lambda_hi;
  er.mix = rule->lambda_mix;
  er.var_tol = rule->var_tol;
  er.min_gap = rule->min_gap;
  er.freeze = rule->freeze != 0;
  Runner r{p, s, p->timing};
  r.stage(9, [&] {
    return launch_eps_update(d_res, d_var, p->at<BlockInfo>(p->off_binfo), (int)p->nblk, er, d_eps, d_state, s);
  });
  return r.err == hipSuccess ? PHI_OK : PHI_ERR_HIP;
}

phi_status phi_pdfb_primal(phi_plan p, float* d_x, float* d_xt, const float* d_grad, const double* d_tau,
                           double* d_var, void* stream) {
  const phi_status st = ready(p);
  if (st != PHI_OK) return st;
  if (!d_x || !d_xt || !d_grad || !d_tau) return PHI_ERR_ARG;
  if (d_x == d_xt || (const float*)d_x == d_grad || (const float*)d_xt == d_grad) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  return primal_locked(p, (hipStream_t)stream, d_x, d_xt, d_grad, d_tau, d_var);
}

phi_status phi_eps_update(phi_plan p, const double* d_res, const double* d_var, const phi_eps_rule* rule,
                          double* d_eps, int32_t* d_state, void* stream) {
  if (!p || !d_res || !d_var || !rule || !d_eps || !d_state) return PHI_ERR_ARG;
  if (!rule_ok(rule)) return PHI_ERR_RANGE;
  const phi_status st = ready(p);
  if (st != PHI_OK) return st;
  std::lock_guard<std::mutex> lk(p->mu);
  return eps_locked(p, (hipStream_t)stream, d_res, d_var, rule, d_eps, d_state);
}

phi_status phi_pdfb_run(phi_plan p, float* d_x, float* d_xt, void* d_v, const void* d_y, double* d_eps,
                        const double* d_sigma, const double* d_tau, int32_t n_iter, const phi_eps_rule* rule,
                        int32_t* d_state, float* d_grad, double* d_rho, double* d_res, double* d_var,
                        void* stream) {
  if (!p) return PHI_ERR_ARG;
  if (rule && !rule_ok(rule)) return PHI_ERR_RANGE;
  if (n_iter < 1) return PHI_ERR_RANGE;
  const phi_status st = ready(p);
  if (st != PHI_OK) return st;
  if (!d_x || !d_xt || !d_grad || !d_tau || !d_eps || !d_var || (p->M > 0 && (!d_v || !d_y))) return PHI_ERR_ARG;
  if (d_x == d_xt || d_x == d_grad || d_xt == d_grad) return PHI_ERR_ARG;
  if (rule && (!d_state || !d_res)) return PHI_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  for (int k = 0; k < n_iter; ++k) {
    phi_status e = l2ball_dual_step(p, d_xt, d_v, d_y, d_eps, d_sigma, d_grad, d_rho, d_res, stream);
    if (e != PHI_OK) return e;
    std::lock_guard<std::mutex> lk(p->mu);
    e = primal_locked(p, s, d_x, d_xt, d_grad, d_tau, d_var);
    if (e == PHI_OK && rule) e = eps_locked(p, s, d_res, d_var, rule, d_eps, d_state);
    if (e != PHI_OK) return e;
  }
  return PHI_OK;
}

// ------------------------------------------------------------- G builder
static double host_i0(double z) {  // power series sum_k ((z/2)^k / k!)^2
  const double h = z / 2.0;
  double sum = 0.0, term = 1.0;
  for (int k = 0; k < 400; ++k) {
    if (k > 0) term *= (h / k) * (h / k);
    sum += term;
    if (k > 0 && term < 1e-18 * sum) break;
  }
  return sum;
}

phi_status phi_plan_build_g(phi_plan p, int64_t block, const phi_gbuild* desc, const double* d_kappa,
                            const int32_t* d_h, const double* d_a, const int32_t* d_ant, const void* d_dde,
                            void* stream) {
  if (!p || !desc) return PHI_ERR_ARG;
  if (block < 0 || block >= p->nblk) return PHI_ERR_RANGE;
  if (p->gprec == PHI_G_KB || p->dr_parent) return PHI_ERR_STATE;
  if (desc->J < 3 || desc->J > 11 || (desc->J & 1) == 0) return PHI_ERR_RANGE;
  if ((d_ant == nullptr) != (d_dde == nullptr)) return PHI_ERR_ARG;
  if (d_ant && (desc->n_ant < 1 || desc->sa < 1 || desc->sa > 7 || (desc->sa & 1) == 0)) return PHI_ERR_RANGE;
  const int64_t n = p->blk_n[block];
  if (n > 0 && (!d_kappa || !d_h || !d_a)) return PHI_ERR_ARG;
  if (!p->bound) return PHI_ERR_STATE;
  std::lock_guard<std::mutex> lk(p->mu);
  hipStream_t s = (hipStream_t)stream;
  p->g_loaded[block] = 0;
  if (n == 0) {
    p->g_loaded[block] = 1;
    return PHI_OK;
  }
  BuildArgs a;
  a.items = p->at<Item>(p->off_items);
  a.meta = p->at<uint32_t>(p->off_meta);
  a.perm = p->at<int32_t>(p->off_perm);
  a.G = p->ws + p->off_G;
  a.gprec = p->gprec;
  a.kappa = d_kappa;
  a.h = d_h;
  a.a = d_a;
  a.ant = d_ant;
  a.dde = static_cast<const double*>(d_dde);
  a.n_ant = d_ant ? desc->n_ant : 0;
  a.sa = d_ant ? desc->sa : 1;
  a.J = desc->J;
  const double J = desc->J;
  a.beta = M_PI * std::sqrt((J / 2.0) * (J / 2.0) * 1.5 * 1.5 - 0.8);
  a.inv_i0b = 1.0 / host_i0(a.beta);
  a.Ky = p->Ky;
  a.Kx = p->Kx;
  a.u0 = p->blk_u0[block];
  a.flag = p->at<int>(p->off_flag) + 2;
  const int zero = 0;
  HIP_TRY(hipMemcpyAsync(a.flag, &zero, sizeof(int), hipMemcpyHostToDevice, s));
  const BlockInfo& bi = p->W().binfo[block];
  HIP_TRY(launch_build_g(a, bi.item0, bi.item1, s));
  int bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, a.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (bad) return PHI_ERR_RANGE;
  p->g_loaded[block] = 1;
  return PHI_OK;
}

phi_status phi_plan_read_g(phi_plan p, int64_t block, void* h_windows, int32_t host_type, void* stream) {
  if (!p) return PHI_ERR_ARG;
  if (block < 0 || block >= p->nblk) return PHI_ERR_RANGE;
  if (host_type != PHI_HOST_C128 && host_type != PHI_HOST_C64) return PHI_ERR_ARG;
  if (p->gprec == PHI_G_KB || !p->bound || !p->g_loaded[block]) return PHI_ERR_STATE;
  const int64_t u0 = p->blk_u0[block], n = p->blk_n[block];
  if (n == 0) return PHI_OK;
  if (!h_windows) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  hipStream_t s = (hipStream_t)stream;
  const size_t eb = p->g_elem_bytes();
  const int64_t t0 = p->tap_off[u0], nt = p->tap_off[u0 + n] - t0;
  std::vector<unsigned char> raw((size_t)nt * eb);
  HIP_TRY(hipMemcpyAsync(raw.data(), p->ws + p->off_G + (size_t)t0 * eb, raw.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<int64_t> uoff(n + 1, 0);
  std::vector<int32_t> uS(n);
  for (int64_t k = 0; k < n; ++k) uS[p->perm[u0 + k] - u0] = p->S_plan[u0 + k];
  for (int64_t i = 0; i < n; ++i) uoff[i + 1] = uoff[i] + (int64_t)uS[i] * uS[i];
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t k = lo; k < hi; ++k) {
      const int64_t ui = p->perm[u0 + k] - u0, src0 = p->tap_off[u0 + k] - t0;
      for (int64_t e = 0; e < uoff[ui + 1] - uoff[ui]; ++e) {
        const unsigned char* r = raw.data() + (size_t)(src0 + e) * eb;
        double re, im;
        if (p->gprec == PHI_G_C64) {
          float f[2];
          std::memcpy(f, r, 8);
          re = f[0];
          im = f[1];
        } else if (p->gprec == PHI_G_F16) {
          _Float16 hv[2];
          std::memcpy(hv, r, 4);
          re = (double)hv[0];
          im = (double)hv[1];
        } else {
          uint16_t b[2];
          std::memcpy(b, r, 4);
          const uint32_t ur = (uint32_t)b[0] << 16, ui2 = (uint32_t)b[1] << 16;
          float fr, fi;
          std::memcpy(&fr, &ur, 4);
          std::memcpy(&fi, &ui2, 4);
          re = fr;
          im = fi;
        }
        const int64_t d = uoff[ui] + e;
        if (host_type == PHI_HOST_C128) {
          static_cast<double*>(h_windows)[2 * d] = re;
          static_cast<double*>(h_windows)[2 * d + 1] = im;
        } else {
          static_cast<float*>(h_windows)[2 * d] = (float)re;
          static_cast<float*>(h_windows)[2 * d + 1] = (float)im;
        }
      }
    }
  });
  return PHI_OK;
}

}  // extern "C"
