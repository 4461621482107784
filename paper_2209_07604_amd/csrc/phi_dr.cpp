// Visibility-gridding dimensionality reduction of one data block
// (Section 3.4, eqs. 4-5), computed on the host at plan time in FP64.
//
//   H     = G^H Theta^H Theta G     (holographic matrix, K x K, Hermitian)
//   S     = {p : H_pp > 0}          (its nonzero rows, M' cells)
//   Lam_p = H_pp^(-1/2) on S
//   y'    = Lam G^H Theta^H y       (gridded data)
//   Phi'  = Lam H F Z               (reduced operator)
//
// Row p of Lam H is nonzero only for cells q with q - p in [-(S-1), S-1]^2
// (both cells in one window), so it is stored like a row of G: a dense
// (2 Smax - 1)^2 window anchored at p - (Smax - 1).  Since H is Hermitian,
// (Lam H)^H = H Lam and Phi'^H v' is the G^H of those rows: a reduced block
// is an ordinary plan block with theta = 1, and every GPU kernel applies.
//
// H is accumulated per 16 x 16 output tile of cells: each window's S^4 tap
// pairs (p, q) are added to the row of p when p lies in the tile; tiles run
// in parallel and visibilities are taken in input order, so the sums have a
// fixed order.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "phi.h"

namespace {

using cd = std::complex<double>;
constexpr int kTile = 16;

struct Row {
  int64_t cell;
  cd y;
  double lam;
  size_t off;  // into the window store
};

}  // namespace

struct phi_dr_s {
  int ky = 0, kx = 0, smax = 1, w = 1;
  std::vector<Row> rows;         // sorted by cell
  std::vector<cd> win;           // rows' windows, w*w each (in `rows` order after sort: see copy)
};

extern "C" {

phi_status phi_dr_create(int32_t ky, int32_t kx, int64_t n_vis, const int32_t* h_base, const uint8_t* h_stencil,
                         const void* h_windows, int32_t host_type, double theta, const void* h_y, phi_dr* out) {
  if (!out) return PHI_ERR_ARG;
  *out = nullptr;
  if (n_vis < 0) return PHI_ERR_SHAPE;
  if (n_vis > 0 && (!h_base || !h_stencil || !h_windows)) return PHI_ERR_ARG;
  if (host_type != PHI_HOST_C128 && host_type != PHI_HOST_C64) return PHI_ERR_ARG;
  if (!(theta > 0.0) || !std::isfinite(theta)) return PHI_ERR_RANGE;
  if (ky < 2 * kTile || kx < 2 * kTile || ky % kTile || kx % kTile || ky > 8192 || kx > 8192)
    return PHI_ERR_UNSUPPORTED;
  int smax = 1;
  std::vector<int64_t> off(n_vis + 1, 0);
  for (int64_t m = 0; m < n_vis; ++m) {
    const int S = h_stencil[m];
    if (S < 1 || !(S & 1) || S > 11) return PHI_ERR_RANGE;  // reduced windows 2S-1 <= 21
    const int by = h_base[2 * m], bx = h_base[2 * m + 1];
    if (by < 0 || by >= ky || bx < 0 || bx >= kx) return PHI_ERR_RANGE;
    smax = std::max(smax, S);
    off[m + 1] = off[m] + (int64_t)S * S;
  }
  const int W = 2 * smax - 1;
  if (ky < 2 * W || kx < 2 * W) return PHI_ERR_UNSUPPORTED;
  phi_dr_s* d = new (std::nothrow) phi_dr_s();
  if (!d) return PHI_ERR_ARG;
  d->ky = ky;
  d->kx = kx;
  d->smax = smax;
  d->w = W;
  auto gval = [&](int64_t e) -> cd {
    if (host_type == PHI_HOST_C128) {
      const double* p = static_cast<const double*>(h_windows) + 2 * e;
      return cd(p[0], p[1]);
    }
    const float* p = static_cast<const float*>(h_windows) + 2 * e;
    return cd(p[0], p[1]);
  };
  auto yval = [&](int64_t m) -> cd {
    if (!h_y) return cd(0.0, 0.0);
    const double* p = static_cast<const double*>(h_y) + 2 * m;
    return cd(p[0], p[1]);
  };
  // (output tile, visibility) pairs, counting-sorted by tile
  const int nty = ky / kTile, ntx = kx / kTile;
  const int64_t ntiles = (int64_t)nty * ntx;
  std::vector<int64_t> cnt(ntiles + 1, 0);
  // the (at most 2 x 2, since S <= 11 < 16) output tiles a window touches
  auto tiles_of = [&](int64_t m, int64_t* t, int& nt) {
    const int S = h_stencil[m], by = h_base[2 * m], bx = h_base[2 * m + 1];
    int ty[2], tx[2], ny = 0, nx = 0;
    for (int i = 0; i < S; ++i) {
      const int r = ((by + i) % ky) / kTile;
      bool seen = false;
      for (int a = 0; a < ny; ++a) seen |= ty[a] == r;
      if (!seen && ny < 2) ty[ny++] = r;
    }
    for (int j = 0; j < S; ++j) {
      const int c = ((bx + j) % kx) / kTile;
      bool seen = false;
      for (int b = 0; b < nx; ++b) seen |= tx[b] == c;
      if (!seen && nx < 2) tx[nx++] = c;
    }
    nt = 0;
    for (int a = 0; a < ny; ++a)
      for (int b = 0; b < nx; ++b) t[nt++] = (int64_t)ty[a] * ntx + tx[b];
  };
  for (int64_t m = 0; m < n_vis; ++m) {
    int64_t t[4];
    int nt;
    tiles_of(m, t, nt);
    for (int k = 0; k < nt; ++k) cnt[t[k] + 1]++;
  }
  for (int64_t t = 0; t < ntiles; ++t) cnt[t + 1] += cnt[t];
  std::vector<int64_t> list(cnt[ntiles]);
  {
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t m = 0; m < n_vis; ++m) {
      int64_t t[4];
      int nt;
      tiles_of(m, t, nt);
      for (int k = 0; k < nt; ++k) list[fill[t[k]]++] = m;
    }
  }
  const int nthreads = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
  std::vector<std::vector<Row>> trows(nthreads);
  std::vector<std::vector<cd>> twin(nthreads);
  std::atomic<int64_t> next{0};
  const double th2 = theta * theta;
  auto worker = [&](int tid) {
    std::vector<cd> acc((size_t)kTile * kTile * W * W);
    std::vector<cd> yacc(kTile * kTile);
    std::vector<char> touched(kTile * kTile);
    for (int64_t t; (t = next.fetch_add(1)) < ntiles;) {
      if (cnt[t] == cnt[t + 1]) continue;
      const int ty0 = (int)(t / ntx) * kTile, tx0 = (int)(t % ntx) * kTile;
      std::fill(acc.begin(), acc.end(), cd(0.0, 0.0));
      std::fill(yacc.begin(), yacc.end(), cd(0.0, 0.0));
      std::fill(touched.begin(), touched.end(), 0);
      cd gw[11 * 11];
      for (int64_t k = cnt[t]; k < cnt[t + 1]; ++k) {
        const int64_t m = list[k];
        const int S = h_stencil[m], by = h_base[2 * m], bx = h_base[2 * m + 1];
        const cd ym = yval(m);
        for (int e = 0; e < S * S; ++e) gw[e] = gval(off[m] + e);
        for (int i = 0; i < S; ++i) {
          const int r = (by + i) % ky;
          if (r < ty0 || r >= ty0 + kTile) continue;
          for (int j = 0; j < S; ++j) {
            const int c = (bx + j) % kx;
            if (c < tx0 || c >= tx0 + kTile) continue;
            const int li = (r - ty0) * kTile + (c - tx0);
            const cd gp = std::conj(gw[i * S + j]);
            const cd a = th2 * gp;
            cd* row = &acc[(size_t)li * W * W];
            for (int i2 = 0; i2 < S; ++i2) {
              cd* rr = row + (size_t)(i2 - i + smax - 1) * W + (smax - 1 - j);
              for (int j2 = 0; j2 < S; ++j2) rr[j2] += a * gw[i2 * S + j2];
            }
            yacc[li] += theta * gp * ym;
            touched[li] = 1;
          }
        }
      }
      const size_t center = (size_t)(smax - 1) * W + (smax - 1);
      for (int li = 0; li < kTile * kTile; ++li) {
        if (!touched[li]) continue;
        const cd* row = &acc[(size_t)li * W * W];
        const double hpp = row[center].real();
        if (!(hpp > 0.0)) continue;
        const double lam = 1.0 / std::sqrt(hpp);
        Row rw;
        rw.cell = (int64_t)(ty0 + li / kTile) * kx + (tx0 + li % kTile);
        rw.y = lam * yacc[li];
        rw.lam = lam;
        rw.off = twin[tid].size();
        for (int e = 0; e < W * W; ++e) twin[tid].push_back(lam * row[e]);
        trows[tid].push_back(rw);
      }
    }
  };
  {
    std::vector<std::thread> th;
    for (int i = 0; i < nthreads; ++i) th.emplace_back(worker, i);
    for (auto& x : th) x.join();
  }
  // gather, sorted by cell
  std::vector<std::pair<int64_t, std::pair<int, size_t>>> idx;
  for (int t = 0; t < nthreads; ++t)
    for (size_t k = 0; k < trows[t].size(); ++k) idx.push_back({trows[t][k].cell, {t, k}});
  std::sort(idx.begin(), idx.end());
  d->rows.reserve(idx.size());
  d->win.resize(idx.size() * (size_t)W * W);
  for (size_t k = 0; k < idx.size(); ++k) {
    Row rw = trows[idx[k].second.first][idx[k].second.second];
    std::memcpy(&d->win[k * (size_t)W * W], &twin[idx[k].second.first][rw.off], sizeof(cd) * W * W);
    rw.off = k * (size_t)W * W;
    d->rows.push_back(rw);
  }
  *out = d;
  return PHI_OK;
}

phi_status phi_dr_size(phi_dr d, int64_t* n_red, int32_t* s_red) {
  if (!d) return PHI_ERR_ARG;
  if (n_red) *n_red = (int64_t)d->rows.size();
  if (s_red) *s_red = d->w;
  return PHI_OK;
}

phi_status phi_dr_copy(phi_dr d, int32_t* h_base, uint8_t* h_stencil, void* h_windows, void* h_y, double* h_lam,
                       int64_t* h_cell) {
  if (!d) return PHI_ERR_ARG;
  const int W = d->w, h = d->smax - 1;
  for (size_t k = 0; k < d->rows.size(); ++k) {
    const Row& rw = d->rows[k];
    const int r = (int)(rw.cell / d->kx), c = (int)(rw.cell % d->kx);
    if (h_base) {
      h_base[2 * k] = (r - h + d->ky) % d->ky;
      h_base[2 * k + 1] = (c - h + d->kx) % d->kx;
    }
    if (h_stencil) h_stencil[k] = (uint8_t)W;
    if (h_y) {
      double* p = static_cast<double*>(h_y) + 2 * k;
      p[0] = rw.y.real();
      p[1] = rw.y.imag();
    }
    if (h_lam) h_lam[k] = rw.lam;
    if (h_cell) h_cell[k] = rw.cell;
  }
  if (h_windows) std::memcpy(h_windows, d->win.data(), sizeof(cd) * d->win.size());
  return PHI_OK;
}

phi_status phi_dr_destroy(phi_dr d) {
  if (!d) return PHI_ERR_ARG;
  delete d;
  return PHI_OK;
}

}  // extern "C"
