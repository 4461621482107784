// Visibility-gridding dimensionality reduction (Section 3.4, eqs. 4-5) of
// every data block, computed on the device from the plan's stored G:
//
//   H     = G^H Theta^H Theta G     (holographic matrix, K x K, Hermitian)
//   S_b   = {p : H_pp > 0}          (the block's support: M'_b gridded cells)
//   Lam_p = H_pp^(-1/2) on S_b
//   y'    = Lam G^H Theta^H y       (gridded data)
//   Phi'  = Lam H F Z               (reduced operator)
//
// Plan creation (host, geometry only): the support of each block is the set
// of cells covered by at least one window, and row p of H can only be
// nonzero at cells q inside a window that also covers p.  Each reduced row is
// therefore stored like a row of G: a dense s x s window whose origin and
// edge are the smallest odd square bounding the union of the windows that
// cover p (s between S and 2 S - 1; isolated windows give s = S).  The rows
// form a second plan (the reduced plan) with the same channels, blocks and
// theta, which shares this plan's workspace and grid buffers.  Because H is
// Hermitian, (Lam H)^H = H Lam and Phi'^H v' is the G^H of those rows, so
// every stage of the ordinary dual step applies to the reduced plan.
//
// phi_dr_setup (device): the row values Lam0 H0 and y' (k_dr_setup), from the
// plan's G kept in complex64; the rows are rounded once to the requested
// precision.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "phi.h"
#include "phi_internal.h"
#include "phi_plan.h"

using namespace phi;

namespace {

struct BlockRows {
  std::vector<uint32_t> cell;  // p_y | p_x << 13, increasing cell index p_y Kx + p_x
  std::vector<int32_t> base;   // [n][2] window origin
  std::vector<uint8_t> s;      // window edge
};

// Cells of one block covered by a window, and per cell the bounding offsets
// (relative to the cell, in [-(S-1), S-1]) of the windows covering it.
phi_status block_rows(const phi_plan_s* p, int b, BlockRows& out) {
  const int Ky = p->Ky, Kx = p->Kx;
  const int64_t K = (int64_t)Ky * Kx;
  std::vector<int8_t> ly(K, 1), lx(K, 1), hy(K, -1), hx(K, -1);  // ly = 1: not covered
  const int64_t v0 = p->blk_u0[b], v1 = v0 + p->blk_n[b];          // plan order is block-major
  for (int64_t v = v0; v < v1; ++v) {
    const uint32_t m = p->meta[v];
    const int S = p->S_plan[v], by = (int)(m & 8191u), bx = (int)((m >> 13) & 8191u);
    for (int i = 0; i < S; ++i) {
      const int cy = by + i < Ky ? by + i : by + i - Ky;
      for (int j = 0; j < S; ++j) {
        const int cx = bx + j < Kx ? bx + j : bx + j - Kx;
        const int64_t c = (int64_t)cy * Kx + cx;
        ly[c] = std::min<int8_t>(ly[c], (int8_t)-i);
        hy[c] = std::max<int8_t>(hy[c], (int8_t)(S - 1 - i));
        lx[c] = std::min<int8_t>(lx[c], (int8_t)-j);
        hx[c] = std::max<int8_t>(hx[c], (int8_t)(S - 1 - j));
      }
    }
  }
  for (int64_t c = 0; c < K; ++c) {
    if (ly[c] > 0) continue;
    int s = std::max(hy[c] - ly[c], hx[c] - lx[c]) + 1;
    if (!(s & 1)) ++s;
    if (s > kMaxS) return PHI_ERR_UNSUPPORTED;
    const int cy = (int)(c / Kx), cx = (int)(c % Kx);
    int oy = cy + ly[c], ox = cx + lx[c];
    if (oy < 0) oy += Ky;
    if (ox < 0) ox += Kx;
    out.cell.push_back((uint32_t)cy | ((uint32_t)cx << 13));
    out.base.push_back(oy);
    out.base.push_back(ox);
    out.s.push_back((uint8_t)s);
  }
  return PHI_OK;
}

}  // namespace

// Reduced plan and set-up tables of a plan created with PHI_DR (after the
// plan's own layout).  Host only.
phi_status dr_build(phi_plan_s* p, const phi_desc* d) {
  if (p->gprec == PHI_G_KB) return PHI_ERR_ARG;  // needs stored G
  if (p->Ky < 2 * kMaxS || p->Kx < 2 * kMaxS) return PHI_ERR_UNSUPPORTED;
  std::vector<BlockRows> br(p->nblk);
  std::atomic<int> next{0};
  std::atomic<int> bad{PHI_OK};
  {
    const int nt = std::max(1, std::min<int>({16, (int)std::thread::hardware_concurrency(), p->nblk}));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&] {
        for (int b; (b = next.fetch_add(1)) < p->nblk;) {
          const phi_status st = block_rows(p, b, br[b]);
          if (st != PHI_OK) bad = st;
        }
      });
    for (auto& x : th) x.join();
  }
  if (bad != PHI_OK) return (phi_status)bad.load();
  // the reduced plan: one row per support cell, in cell order per block
  std::vector<int64_t> n_red(p->nblk);
  std::vector<int32_t> base;
  std::vector<uint8_t> sten;
  for (int b = 0; b < p->nblk; ++b) {
    n_red[b] = (int64_t)br[b].s.size();
    base.insert(base.end(), br[b].base.begin(), br[b].base.end());
    sten.insert(sten.end(), br[b].s.begin(), br[b].s.end());
  }
  phi_desc cd = *d;
  cd.h_n_vis = n_red.data();
  cd.h_base = base.data();
  cd.h_stencil = sten.data();
  cd.flags = d->flags & ~PHI_DR;
  phi_plan_s* c = nullptr;
  const phi_status st = phi_plan_create(&cd, &c);
  if (st != PHI_OK) return st;
  c->dr_parent = p;
  p->dr = c;
  // set-up tables over the parent's work list with the smallest tile edge
  int wl = 0;
  for (int i = 1; i < (int)p->cands.size(); ++i)
    if (p->cands[i].T < p->cands[wl].T) wl = i;
  const WorkList& w = p->cands[wl];
  const int T = w.T, nty = p->Ky / T, ntx = p->Kx / T;
  const int64_t ntiles = (int64_t)nty * ntx;
  // items of one (block, origin tile) are consecutive in plan order
  std::unordered_map<int64_t, std::pair<int32_t, int32_t>> tile_items;
  for (int32_t i = 0; i < (int32_t)w.items.size(); ++i) {
    const Item& it = w.items[i];
    const int64_t key = (int64_t)it.blk * ntiles + (int64_t)(it.ty0 / T) * ntx + it.tx0 / T;
    auto f = tile_items.find(key);
    if (f == tile_items.end())
      tile_items.emplace(key, std::make_pair(i, i + 1));
    else
      f->second.second = i + 1;
  }
  std::vector<int32_t> pos_of(c->M);
  for (int64_t k = 0; k < c->M; ++k) pos_of[c->perm[k]] = (int32_t)k;
  DrTables& t = p->drt;
  t.rows.clear();
  t.groups.clear();
  t.cands.clear();
  t.cell_by_pos.assign(c->M, 0);
  for (int b = 0; b < p->nblk; ++b) {
    int smax = 1;
    for (int64_t v = p->blk_u0[b]; v < p->blk_u0[b] + p->blk_n[b]; ++v) smax = std::max<int>(smax, p->S_plan[v]);
    const int h = (smax - 1 + T - 1) / T;  // origin tiles up to h tiles up/left can reach a cell
    const BlockRows& r = br[b];
    const int64_t n = (int64_t)r.cell.size();
    // rows by cell tile (counting sort; cell order inside a tile)
    std::vector<int64_t> cnt(ntiles + 1, 0);
    auto tile_of = [&](uint32_t cell) {
      return (int64_t)((cell & 8191u) / T) * ntx + ((cell >> 13) & 8191u) / T;
    };
    for (int64_t i = 0; i < n; ++i) cnt[tile_of(r.cell[i]) + 1]++;
    for (int64_t q = 0; q < ntiles; ++q) cnt[q + 1] += cnt[q];
    std::vector<int64_t> order(n), fill(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < n; ++i) order[fill[tile_of(r.cell[i])]++] = i;
    const int64_t u0 = c->blk_u0[b];
    for (int64_t q = 0; q < ntiles; ++q) {
      if (cnt[q] == cnt[q + 1]) continue;
      DrGroup g{};
      g.row0 = (int32_t)t.rows.size();
      for (int64_t k = cnt[q]; k < cnt[q + 1]; ++k) {
        const int64_t i = order[k];
        DrRow row{};
        row.cell = r.cell[i];
        row.pos = pos_of[u0 + i];
        row.tap = c->tap_off[row.pos];
        t.cell_by_pos[row.pos] = (int64_t)(r.cell[i] & 8191u) * p->Kx + ((r.cell[i] >> 13) & 8191u);
        t.rows.push_back(row);
      }
      g.row1 = (int32_t)t.rows.size();
      g.cand0 = (int32_t)t.cands.size();
      const int ty = (int)(q / ntx), tx = (int)(q % ntx);
      std::vector<int64_t> seen;
      for (int a = 0; a <= h; ++a)
        for (int e = 0; e <= h; ++e) {
          const int sy = ((ty - a) % nty + nty) % nty, sx = ((tx - e) % ntx + ntx) % ntx;
          const int64_t key = (int64_t)b * ntiles + (int64_t)sy * ntx + sx;
          if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
          seen.push_back(key);
          auto f = tile_items.find(key);
          if (f == tile_items.end()) continue;
          DrCand cand{};
          cand.v0 = w.items[f->second.first].v0;
          cand.v1 = w.items[f->second.second - 1].v1;
          cand.tap0 = w.items[f->second.first].tap0;
          t.cands.push_back(cand);
        }
      g.cand1 = (int32_t)t.cands.size();
      t.groups.push_back(g);
    }
  }
  if (t.rows.size() > (size_t)INT32_MAX || t.cands.size() > (size_t)INT32_MAX) return PHI_ERR_UNSUPPORTED;
  return PHI_OK;
}

extern "C" {

phi_status phi_dr_plan(phi_plan p, phi_plan* out) {
  if (!p || !out) return PHI_ERR_ARG;
  *out = nullptr;
  if (!p->dr) return PHI_ERR_STATE;
  *out = p->dr;
  return PHI_OK;
}

phi_status phi_dr_rows(phi_plan p, int64_t* h_cells, int32_t* h_base, uint8_t* h_stencil) {
  if (!p) return PHI_ERR_ARG;
  if (!p->dr) return PHI_ERR_STATE;
  const phi_plan_s* c = p->dr;
  for (int64_t k = 0; k < c->M; ++k) {
    if (h_cells) h_cells[k] = p->drt.cell_by_pos[k];
    const uint32_t m = c->meta[k];
    if (h_base) {
      h_base[2 * k] = (int32_t)(m & 8191u);
      h_base[2 * k + 1] = (int32_t)((m >> 13) & 8191u);
    }
    if (h_stencil) h_stencil[k] = c->S_plan[k];
  }
  return PHI_OK;
}

phi_status phi_dr_setup(phi_plan p, const void* d_y, void* d_yred, int64_t* h_m_red, void* stream) {
  if (!p) return PHI_ERR_ARG;
  if (!p->dr) return PHI_ERR_STATE;
  if (!p->bound) return PHI_ERR_STATE;
  for (char c : p->g_loaded)
    if (!c) return PHI_ERR_STATE;
  phi_plan_s* c = p->dr;
  if (c->M > 0 && !d_yred) return PHI_ERR_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  DrArgs a;
  a.meta = p->at<uint32_t>(p->off_meta);
  a.G = p->ws + p->off_G;
  a.rmeta = c->at<uint32_t>(c->off_meta);
  a.H = c->ws + c->off_G;
  a.gprec_g = p->gprec;
  a.gprec_h = c->gprec;
  a.rows = p->at<DrRow>(p->off_drrow);
  a.groups = p->at<DrGroup>(p->off_drgrp);
  a.cands = p->at<DrCand>(p->off_drcand);
  a.y = static_cast<const float2*>(d_y);
  a.yred = static_cast<float2*>(d_yred);
  a.Ky = p->Ky;
  a.Kx = p->Kx;
  if (launch_dr_setup(a, (int)p->drt.groups.size(), (hipStream_t)stream) != hipSuccess) return PHI_ERR_HIP;
  {
    std::lock_guard<std::mutex> lc(c->mu);
    std::fill(c->g_loaded.begin(), c->g_loaded.end(), 1);
  }
  if (h_m_red)
    for (int b = 0; b < p->nblk; ++b) h_m_red[b] = c->blk_n[b];
  return PHI_OK;
}

phi_status l2ball_dual_step_dr(phi_plan p, const float* d_xt, void* d_vred, const void* d_yred,
                               const double* d_eps_red, const double* d_sigma, float* d_grad, double* d_rho,
                               double* d_res, void* stream) {
  if (!p) return PHI_ERR_ARG;
  if (!p->dr) return PHI_ERR_STATE;
  return l2ball_dual_step(p->dr, d_xt, d_vred, d_yred, d_eps_red, d_sigma, d_grad, d_rho, d_res, stream);
}

}  // extern "C"
