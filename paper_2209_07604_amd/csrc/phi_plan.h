// The plan object behind phi_plan (host only): geometry, plan order, work
// lists, workspace layout and launch state.  Shared by the sources that
// implement the C ABI; not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <cstddef>
#include <cstdint>
#include <mutex>
#include <utility>
#include <vector>

#include "phi.h"
#include "phi_internal.h"

namespace phi {

struct StageTimer {
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  size_t next = 0;
  double ms[16] = {0};
  int64_t calls = 0;
  hipEvent_t get() {
    if (next == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[next++];
  }
};

// The work lists of one tile edge T (G items, block ranges, merge lists).
struct WorkList {
  int T = 32, halo = 1, max_pitch = 0;
  int64_t partial_elems = 0;
  std::vector<Item> items;
  std::vector<BlockInfo> binfo;
  std::vector<int32_t> tile_ptr;
  std::vector<TileEntry> entries;
  std::vector<int32_t> chan_item0;          // [L + 1]
  // the merge's regions (merge_rk x merge_rk tiles) that some partial
  // covers, by channel, as channel-major region indices; channel l's are
  // [chan_live0[l], chan_live0[l + 1])
  int merge_rk = 1;
  std::vector<int32_t> live;
  std::vector<int32_t> chan_live0;          // [L + 1]
  // the live regions as bits: word (l * (Ky / R) + ry) * live_wpr + rx / 32,
  // bit rx % 32 (R = merge_rk * T)
  int live_wpr = 1;
  std::vector<uint32_t> live_bits;
  // the items again, by pitch (largest first), for launches whose LDS is
  // sized per pitch; runs of equal pitch as (pitch, first, end)
  std::vector<Item> items_by_pitch;
  std::vector<std::array<int32_t, 3>> pitch_runs;
};

// Host copies of the gridding reduction's set-up tables (plans created with
// PHI_DR): rows in set-up order, their groups and candidate ranges, and the
// cell of every reduced row by its position in the reduced plan.
struct DrTables {
  std::vector<DrRow> rows;
  std::vector<DrGroup> groups;
  std::vector<DrCand> cands;
  std::vector<int64_t> cell_by_pos;
};

}  // namespace phi

struct phi_plan_s {
  using WorkList = phi::WorkList;
  using StageTimer = phi::StageTimer;
  // geometry
  int L = 0, Ny = 0, Nx = 0, Ky = 0, Kx = 0, nblk = 0;
  int gprec = 0, flags = 0, persist = 0;
  int64_t M = 0, ntaps = 0;
  std::vector<int32_t> n_blocks, blk_chan, chan_blk0;
  std::vector<int64_t> blk_u0, blk_n;       // user order start / count per block
  std::vector<double> theta, sy, sx;
  // plan order
  std::vector<int32_t> perm;                // plan -> user (global)
  std::vector<uint32_t> meta;
  std::vector<int64_t> tap_off;             // [M + 1]
  std::vector<uint8_t> S_plan;
  int smax = 1;
  // work lists: one per candidate tile edge, `cur` is in use on the device
  std::vector<WorkList> cands;
  int cur = 0;
  WorkList& W() { return cands[cur]; }
  const WorkList& W() const { return cands[cur]; }
  // workspace layout
  size_t off_bpart = 0, off_G = 0, off_meta = 0, off_perm = 0, off_items = 0, off_items_p = 0, off_live_bits = 0,
         off_binfo = 0, off_tptr = 0, off_ent = 0,
         off_theta = 0, off_part = 0, off_norms = 0, off_scale = 0, off_flag = 0, off_grid = 0, off_half = 0,
         off_twx = 0, off_twy = 0, off_sy = 0, off_sx = 0, off_vscr = 0, off_anal = 0, off_frac = 0, ws_bytes = 0,
         off_grid_a = 0, off_live = 0;
  // the adjoint's grid is a region of its own, kept zero outside the tiles the
  // merge writes (sparse merge), or the forward grid (every tile written)
  bool sparse_merge = false;
  char* ws = nullptr;
  bool bound = false;
  std::vector<char> g_loaded;
  hipStream_t cap_stream = nullptr;
  // graph cache for the dual step
  hipGraphExec_t gexec = nullptr;
  const void* gkey[9] = {nullptr};
  // timing
  bool timing = false;
  StageTimer timer;
  std::mutex mu;

  // G store bytes per tap (none in the Kaiser-Bessel mode, where taps are
  // evaluated in the kernels from per-visibility fractional coordinates)
  size_t g_elem_bytes() const { return gprec == PHI_G_KB ? 0 : gprec == PHI_G_C64 ? 8 : 4; }
  // the dual step reads each G tap once (gather and G^H in one pass)
  bool fused() const;
  int kb_J = 0;                 // window width of the Kaiser-Bessel mode
  double kb_beta = 0.0, kb_inv_i0b = 0.0;
  // gridding reduction (PHI_DR): the reduced plan lives in this plan's
  // workspace after its own regions (ws_total covers both and the set-up
  // tables) and shares its grid, half grid, twiddles and Z scales
  phi_plan_s* dr = nullptr;          // owned by this plan
  phi_plan_s* dr_parent = nullptr;   // set on a reduced plan
  phi::DrTables drt;
  size_t off_drrow = 0, off_drgrp = 0, off_drcand = 0, ws_total = 0;
  template <typename T_>
  T_* at(size_t off) const { return reinterpret_cast<T_*>(ws + off); }
};

// Reduced plan and set-up tables of a plan created with PHI_DR (phi_dr.cpp).
phi_status dr_build(phi_plan_s* p, const phi_desc* d);

// phi_power_iteration with its scratch image d_tmp given (phi_host.cpp).
phi_status power_iteration_impl(phi_plan_s* p, float* d_x, float* d_tmp, int32_t n_iter, double* d_nu,
                                void* stream);
