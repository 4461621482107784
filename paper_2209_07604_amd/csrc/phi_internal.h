// Internal types shared by the host planner (phi_host.cpp) and the HIP
// kernels (phi_kernels.hip).  Not part of the public ABI.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace phi {

constexpr int kMaxS = 21;          // largest window edge
constexpr int kMaxK = 8192;        // largest grid edge (13-bit cell index)
constexpr int kWave = 64;

// Per-visibility metadata word: b_y (13 bits) | b_x (13 bits) | (S-1)/2 (4 bits)
__host__ __device__ inline uint32_t pack_meta(int by, int bx, int S) {
  return (uint32_t)by | ((uint32_t)bx << 13) | ((uint32_t)((S - 1) >> 1) << 26);
}

// A G work item: a run of plan-order visibilities of one block whose window
// origins fall in one T x T uv tile.  Its G^H contributions accumulate in a
// pitch x pitch LDS tile anchored at (ty0, tx0); pitch = T + Smax_item - 1.
struct Item {
  int64_t tap0;    // first G tap of the run
  int64_t poff;    // float2 offset of its tile partial
  int32_t v0, v1;  // plan-order visibility range
  int32_t blk;     // global block index
  int32_t chan;    // channel
  int32_t ty0, tx0;
  int32_t pitch;
  int32_t ntap;    // taps of the run (sum of S^2)
  int32_t sub[3];  // taps before visibility wv[w - 1], w = 1..3
  int32_t slot;    // the item's index in plan order (its norm slot)
  int32_t wv[3];   // plan-order visibility where the gather's wave w = 1..3
                   // starts (W <= 4 waves; equal shares of S^2 + 64 per window)
  int32_t pad2;
};
static_assert(sizeof(Item) == 80, "Item layout");
#ifndef PHI_GATHER_WAVES
#define PHI_GATHER_WAVES 2
#endif
constexpr int kGatherWaves = PHI_GATHER_WAVES;

// Merge-list entry: one tile partial that overlaps a tile.
struct TileEntry {
  int64_t poff;
  int32_t pitch;
  int32_t blk;  // block of the item (its merge factor in the fused dual step)
};

struct BlockInfo {
  int32_t chan;
  int32_t item0, item1;   // items of the block
  int32_t pad;
  int64_t v0, v1;         // plan-order visibility range
};

// Arguments common to the G stages.
struct GArgs {
  const Item* items;
  const uint32_t* meta;
  const void* G;
  const float* theta;       // [nblk]
  const double* sigma;      // [nblk] or null (=> 1)
  const double* scale;      // [nblk] projection scale (dual step)
  float2* grid;             // [L][Ky][Kx]
  int Ky, Kx;
  int T;                    // tile edge of the items (pitch = T + Smax - 1)
  // Kaiser-Bessel mode: per-visibility (kappa_y - b_y, kappa_x - b_x) in plan
  // order, the width J, beta and 1 / I0(beta)
  const float2* frac;
  int kb_J;
  float kb_beta, kb_inv_i0b;
  float2* partials;         // per-item tile partials (written by the fused dual step)
};

// Kernel launchers (phi_kernels.hip).  All asynchronous on `s`.
hipError_t launch_rowfft_fwd(int Kx, const float* x, float2* half, const float* sy, const float* sx,
                             const float2* tw, int Ny, int Nx, int l0, int nl, hipStream_t s);
hipError_t launch_colfft_fwd(int Ky, const float2* half, float2* grid, const float2* tw, int Ny,
                             int Kx, int l0, int nl, hipStream_t s);
hipError_t launch_colfft_inv(int Ky, const float2* grid, float2* half, const float2* tw, int Ny,
                             int Kx, int l0, int nl, hipStream_t s);
hipError_t launch_rowfft_inv(int Kx, const float2* half, float* x, const float* sy, const float* sx,
                             const float2* tw, int Ny, int Nx, int l0, int nl, hipStream_t s);
// Image-first order for grids whose columns take two passes (Ky = 3072 ...
// 8192, Nx / 2 a multiple of 8): columns of the image first (zp: packed
// scratch [L][Ky][Nx/2], T: [L][Ky][Nx]), then the Ky rows of T into the
// grid; the adjoint runs the mirror.
bool fft_image_first(int Ky, int Nx);
hipError_t launch_rowc_fwd(int Kx, const float2* T, float2* grid, const float2* tw, int Ky, int l0, int nl,
                           hipStream_t s);
hipError_t launch_colr_fwd(int Ky, const float* x, float2* zp, float2* T, const float* sy, const float* sx,
                           const float2* tw, int Ny, int Nx, int l0, int nl, hipStream_t s);

// Regions of R x R grid cells known to be zero outside the live ones: bit
// rx % 32 of word (l * (Ky / R) + ry) * wpr + rx / 32 marks region (ry, rx)
// of channel l live; bits null: every cell is read.
struct LiveRegions {
  const uint32_t* bits;
  int R, wpr;
};
// The inverse row pass reads only the live regions' cells when live.bits is
// set (the others are zero).
hipError_t launch_rowc_inv(int Kx, const float2* grid, float2* T, const float2* tw, int Ky, int l0, int nl,
                           LiveRegions live, hipStream_t s);
hipError_t launch_colr_inv(int Ky, const float2* T, float2* zp, float* x, const float* sy, const float* sx,
                           const float2* tw, int Ny, int Nx, int l0, int nl, hipStream_t s);

// mode: 0 forward (write y), 1 residual (c = v/sigma + phi - y into v; norms)
hipError_t launch_gather(int gprec, int mode, const GArgs& a, float2* vis, const float2* y,
                         double* item_norms, int max_pitch, int it0, int it1, int grid_blocks, hipStream_t s);
// Fused dual step (mode 2 of the gather): c per visibility and, with the same
// G taps, G^H c into per-item tile partials; the per-block factors
// sigma * scale * theta (merge) and sigma * scale (launch_vscale) come after
// the norms.  LDS bytes it
// needs for the largest pitch; 0 if it does not fit a work-group.
size_t fused_lds_bytes(int max_pitch);
// LDS of the Kaiser-Bessel one-pass kernel (k_dual_kb), or 0 if it does not fit.
size_t kb_fused_lds_bytes(int max_pitch);
// v <- sigma_b * scale_b * v over the visibilities of items [it0, it1)
hipError_t launch_vscale(const BlockInfo* blocks, float2* vis, const double* sigma, const double* scale, int b0,
                         int nb, hipStream_t s);
// mode: 0 adjoint (read v), 1 dual (v+ = sigma*scale*c, written back)
hipError_t launch_scatter(int gprec, int mode, const GArgs& a, float2* vis, float2* partials,
                          int max_pitch, int it0, int it1, int grid_blocks, hipStream_t s);
// sigma/scale/theta: per-block factors sigma_b * scale_b * theta_b applied to
// each item's partial (entry .blk) after the one-pass dual step (sigma null:
// 1), or scale null for factor 1.  A work-group merges a region of rk x rk
// tiles (rk 1, 2 or 4).  live: the regions to write, live[live0 .. live0 +
// n_live) (channel-major region indices), or null for every region of
// channels [l0, l0 + nl).
hipError_t launch_merge(float2* grid, const float2* partials, const int32_t* tile_ptr,
                        const TileEntry* entries, const int32_t* live, int live0, int n_live, int Ky, int Kx, int T,
                        int halo, int rk, int l0, int nl, const double* sigma, const double* scale,
                        const float* theta, hipStream_t s);
// True where the inverse 2-D transform leaves its input grid unchanged (it
// runs in place on it for rows-first grids whose columns take two passes).
bool fft_inverse_reads_grid_only(int Ky, int Nx);
// block_part: [nblk][kFinChunks][2] scratch
constexpr int kFinChunks = 64;
hipError_t launch_finalize(const double* item_norms, const BlockInfo* blocks, double* block_part, const double* eps,
                           double* rho, double* res, double* scale, int* flag, int b0, int nb, hipStream_t s);
hipError_t launch_permute(const float2* src, float2* dst, const int32_t* perm, int64_t n,
                          int to_plan, hipStream_t s);

// Device G builder (rows from per-visibility tables, FP64)
struct BuildArgs {
  const Item* items;
  const uint32_t* meta;
  const int32_t* perm;     // plan position -> user index (global)
  void* G;
  int gprec;               // 0 c64, 1 f16, 2 bf16
  const double* kappa;     // [n][2], user order within the block
  const int32_t* h;        // [n]
  const double* a;         // [n]
  const int32_t* ant;      // [n][2] or null
  const double* dde;       // complex128 [n_ant][sa][sa] as (re, im) pairs, or null
  int n_ant, sa, J;
  double beta, inv_i0b;
  int Ky, Kx;
  int64_t u0;              // the block's first plan / user position
  int* flag;               // set to 1 on a row that does not match its declared window
};
hipError_t launch_build_g(const BuildArgs& a, int it0, int it1, hipStream_t s);

// Visibility-gridding reduction (Section 3.4, eqs. 4-5) computed on the
// device from the plan's stored G.  A reduced row is one gridded cell p of a
// block's support; it is stored like a row of G: an s x s window (its
// origin and s in the reduced plan's metadata word) that bounds every cell q
// with H_pq possibly nonzero.
struct DrRow {       // one reduced row, in set-up order (block, cell tile, cell)
  uint32_t cell;     // p_y | p_x << 13
  int32_t pos;       // its position in the reduced plan's order
  int64_t tap;       // its first tap in the reduced plan's G store
};
struct DrGroup {     // the rows of one block in one T x T tile of cells
  int32_t row0, row1;
  int32_t cand0, cand1;  // candidate visibility ranges [cand0, cand1)
};
struct DrCand {      // a plan-order range of the block's visibilities whose
  int32_t v0, v1;    // window origins lie in a tile that can reach the group
  int64_t tap0;      // first G tap of visibility v0
};
struct DrArgs {
  const uint32_t* meta;     // plan's metadata (plan order)
  const void* G;            // plan's stored G
  const uint32_t* rmeta;    // reduced plan's metadata
  void* H;                  // reduced plan's G store (rows Lam0 H0, rounded once)
  int gprec_g, gprec_h;     // storage of G and of the rows: 0 c64, 1 f16, 2 bf16
  const DrRow* rows;
  const DrGroup* groups;
  const DrCand* cands;
  const float2* y;          // whitened data, plan order (may be null: y' = 0)
  float2* yred;             // y' in the reduced plan's order
  int Ky, Kx;
};
hipError_t launch_dr_setup(const DrArgs& a, int n_groups, hipStream_t s);

// Zero taps kept behind G: a window's fetch reads 64 * NK taps (NK <= 7)
// from its first tap, past the window's end.
constexpr int kGPadTaps = 7 * 64;

// analysis helpers (per-channel images are [L][n] float32)
constexpr int kNormChunks = 256;
hipError_t launch_delta(float* x, int L, int Ny, int Nx, hipStream_t s);
hipError_t launch_vis_residual(float2* v, const float2* y, int64_t n, hipStream_t s);  // v <- y - v
// part: [L][kNormChunks] scratch; norm, inv: [L] (either may be null)
hipError_t launch_chan_norm(const float* x, int L, int64_t n, double* part, double* norm, double* inv,
                            hipStream_t s);
hipError_t launch_chan_scale(float* x, const double* f, int L, int64_t n, hipStream_t s);  // x_l *= f[l]
hipError_t launch_centre_value(const float* x, int L, int Ny, int Nx, double* peak, hipStream_t s);

// PDFB primal step: x <- max(x - tau_l g, 0), xt <- 2 x+ - x; part: [L][kNormChunks][2]
// scratch, var: [L][2] (||x+ - x||^2, ||x+||^2), may be null
hipError_t launch_pdfb_primal(float* x, float* xt, const float* g, const double* tau, int L, int64_t n,
                              double* part, double* var, hipStream_t s);
// adaptive l2-bound rule over the blocks; state: [nblk][3] (since, fixed, count)
struct EpsRule {
  double lo, hi, mix, var_tol;
  int min_gap, freeze;
};
hipError_t launch_eps_update(const double* res, const double* var, const BlockInfo* blocks, int nblk,
                             EpsRule rule, double* eps, int32_t* state, hipStream_t s);

bool fft_length_supported(int n);

}  // namespace phi
