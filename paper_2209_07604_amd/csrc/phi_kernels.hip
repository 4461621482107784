// HIP kernels for gfx950 (MI355X): the stages of Phi = Theta G F Z, its
// adjoint and the l2-ball data-fidelity dual step (Sections 2.1-2.2, eqs. 1-2).
//
//   rowfft_fwd  Z + forward DFT along x of the Ny nonzero rows   (F Z, part 1)
//   colfft_fwd  forward DFT along y of every grid column          (F Z, part 2)
//   gather      theta_b * G X per visibility; optional residual    (G, eq. 1;
//               c = v/sigma + Phi x - y with FP64 partial norms     eq. 2 step)
//   finalize    per-block FP64 norms and projection scale           (eq. 2)
//   scatter     G^H theta v (or the dual update first) into LDS tiles
//   merge       fixed-order sum of tile partials into the grid      (G^H)
//   colfft_inv  inverse DFT along y, keeping the Ny rows Z^T reads  (F^H)
//   rowfft_inv  inverse DFT along x, crop, scale, real part        (Z^T F^H)
//
// Everything is FP32 except the norms and the projection scale (FP64).
// No kernel uses global atomics; the G^H accumulation is owned by one wave
// per tile partial and merged in a fixed order, so results are bitwise
// reproducible run to run.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "phi_internal.h"

namespace phi {
namespace {

// ----------------------------------------------------------------- helpers
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// multiply by -i (forward transform) or +i (inverse transform)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 z) {
  return INV ? make_float2(-z.y, z.x) : make_float2(z.y, -z.x);
}

template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ float readlane_f(float v, int i) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
}

// v_writelane_b32 (the compiler has no builtin for it; this names the LLVM
// intrinsic): lane i of the result is the wave-uniform v, the other lanes
// keep old.
extern "C" __device__ int phi_writelane_i32(int v, int i, int old) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ float writelane_f(float old, float v, int i) {
  return __int_as_float(phi_writelane_i32(__float_as_int(v), i, __float_as_int(old)));
}

// A wave-uniform 64-bit value, so that it stays in scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// LDS byte addresses: the offset of a __shared__ buffer inside the
// work-group's LDS, and complex loads / stores at such an offset.  Callers
// fold the buffer offset into their per-lane offsets once, so each access is
// a single address register with no further add.
typedef float f32x2 __attribute__((ext_vector_type(2)));
using lds_f32x2 = __attribute__((address_space(3))) f32x2;
__device__ __forceinline__ uint32_t lds_offset(const float2* p) {
  return (uint32_t)(uintptr_t)(const lds_f32x2*)(const f32x2*)p;
}
__device__ __forceinline__ float2 lds_load(uint32_t a) {
  const f32x2 v = *(const lds_f32x2*)(uintptr_t)a;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void lds_store(uint32_t a, float2 v) {
  f32x2 w;
  w.x = v.x;
  w.y = v.y;
  *(lds_f32x2*)(uintptr_t)a = w;
}

// Row and column of tap t of an S x S window: i = floor((t + 1/2) / S) in
// FP32 with the hardware reciprocal is exact for t < 441, S <= 21 (the
// quotient stays >= 1/(2S) away from an integer, the reciprocal's relative
// error is ~1e-7), so no table or integer division is needed.
__device__ __forceinline__ int tap_row(int t, float rS) { return (int)(((float)t + 0.5f) * rS); }

// Spread consecutive panels over one XCD: work-group i runs on XCD i % 8.
__device__ __forceinline__ int xcd_remap(int i, int n) {
  if (n % 8 != 0) return i;
  return (i % 8) * (n / 8) + i / 8;
}

// ------------------------------------------------------------- FFT (LDS)
// Self-sorting (Stockham) mixed-radix passes over W interleaved sequences of
// length N held in LDS: element (k, c) at buf[k * W + c].  A pass of radix R
// with span NS takes inputs k = b + r N/R, twiddles them by
// exp(-+2 pi i (b mod NS) r / (NS R)) and writes the R-point DFT to
// (b / NS) NS R + (b mod NS) + r NS.  tw[m] = exp(-2 pi i m / N) (FP32 from FP64).
template <int R, bool INV>
__device__ __forceinline__ void dft(float2* a);

template <>
__device__ __forceinline__ void dft<2, false>(float2* a) {
  const float2 t = a[0];
  a[0] = cadd(t, a[1]);
  a[1] = csub(t, a[1]);
}
template <>
__device__ __forceinline__ void dft<2, true>(float2* a) { dft<2, false>(a); }

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3);
  const float2 t3 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}
template <>
__device__ __forceinline__ void dft<4, false>(float2* a) { dft4<false>(a[0], a[1], a[2], a[3]); }
template <>
__device__ __forceinline__ void dft<4, true>(float2* a) { dft4<true>(a[0], a[1], a[2], a[3]); }

template <bool INV>
__device__ __forceinline__ void dft8(float2* a) {
  constexpr float c = 0.70710678118654752440f;
  float2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  float2 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  if (!INV) {
    o1 = make_float2(c * (o1.x + o1.y), c * (o1.y - o1.x));
    o3 = make_float2(c * (o3.y - o3.x), -c * (o3.x + o3.y));
  } else {
    o1 = make_float2(c * (o1.x - o1.y), c * (o1.x + o1.y));
    o3 = make_float2(-c * (o3.x + o3.y), c * (o3.x - o3.y));
  }
  o2 = mul_mi<INV>(o2);
  a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
}
template <>
__device__ __forceinline__ void dft<8, false>(float2* a) { dft8<false>(a); }
template <>
__device__ __forceinline__ void dft<8, true>(float2* a) { dft8<true>(a); }

template <bool INV>
__device__ __forceinline__ void dft3(float2* a) {
  constexpr float h = 0.86602540378443864676f;  // sqrt(3)/2
  const float2 s = cadd(a[1], a[2]), d = csub(a[1], a[2]);
  const float2 m = make_float2(a[0].x - 0.5f * s.x, a[0].y - 0.5f * s.y);
  const float2 t = mul_mi<INV>(cscale(d, h));
  a[0] = cadd(a[0], s);
  a[1] = cadd(m, t);
  a[2] = csub(m, t);
}
template <>
__device__ __forceinline__ void dft<3, false>(float2* a) { dft3<false>(a); }
template <>
__device__ __forceinline__ void dft<3, true>(float2* a) { dft3<true>(a); }

template <bool INV>
__device__ __forceinline__ void dft5(float2* a) {
  constexpr float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
  constexpr float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
  constexpr float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
  constexpr float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
  const float2 p1 = cadd(a[1], a[4]), d1 = csub(a[1], a[4]);
  const float2 p2 = cadd(a[2], a[3]), d2 = csub(a[2], a[3]);
  const float2 m1 = make_float2(a[0].x + c1 * p1.x + c2 * p2.x, a[0].y + c1 * p1.y + c2 * p2.y);
  const float2 m2 = make_float2(a[0].x + c2 * p1.x + c1 * p2.x, a[0].y + c2 * p1.y + c1 * p2.y);
  const float2 n1 = mul_mi<INV>(make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
  const float2 n2 = mul_mi<INV>(make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
  a[0] = cadd(a[0], cadd(p1, p2));
  a[1] = cadd(m1, n1);
  a[4] = csub(m1, n1);
  a[2] = cadd(m2, n2);
  a[3] = csub(m2, n2);
}
template <>
__device__ __forceinline__ void dft<5, false>(float2* a) { dft5<false>(a); }
template <>
__device__ __forceinline__ void dft<5, true>(float2* a) { dft5<true>(a); }

constexpr int pick_radix(int rem) {
  return rem % 5 == 0 ? 5
         : rem % 3 == 0 ? 3
         : (rem % 8 == 0 && rem != 16) ? 8
         : rem % 4 == 0 ? 4
                        : 2;
}

// LDS slot of element i of a padded buffer: one spare slot after every 16,
// so the strided writes of the first passes of a transform over one or two
// sequences (lanes 8 or 16 elements apart) do not pile onto a few banks.
template <bool PAD>
__device__ __forceinline__ int lds_i(int i) {
  return PAD ? i + (i >> 4) : i;
}

// The pass twiddles come from tab, an LDS table of each pass's base
// twiddles w = exp(-+2 pi i k / (NS R)), k < NS (tw_table), as w^r by
// squarings and one product per odd r (a few ulp from exact values), so no
// pass issues a global load (a kernel that keeps loads of its next
// transform in flight would wait for them at such a load: vmcnt is in
// order).  PAD: buf is addressed through lds_i.  tid: the thread's index
// (threadIdx.x; a loop over transforms passes a copy the compiler cannot see
// through, so the LDS addresses are formed in the loop instead of being
// hoisted out of it and held in registers).
template <int N, int W, int NT, bool INV, int R, int NS, bool PAD>
__device__ __forceinline__ void fft_pass(float2* buf, const float2* tab, int tid) {
  constexpr int STRIDE = N / R;
  constexpr int NB = STRIDE * W;
  constexpr int BPT = (NB + NT - 1) / NT;
  float2 v[BPT][R];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int j = tid + q * NT;
    if (NB % NT == 0 || j < NB) {
      const int c = j % W, b = j / W;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[lds_i<PAD>((b + r * STRIDE) * W + c)];
      if constexpr (NS > 1) {
        float2 w[R];
        w[1] = tab[b % NS];
        if (INV) w[1].y = -w[1].y;
#pragma unroll
        for (int r = 2; r < R; ++r) w[r] = (r % 2 == 0) ? cmul(w[r / 2], w[r / 2]) : cmul(w[r - 1], w[1]);
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], w[r]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int j = tid + q * NT;
    if (NB % NT == 0 || j < NB) {
      const int c = j % W, b = j / W;
      const int k = b % NS;
      dft<R, INV>(v[q]);
      const int d = (b / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lds_i<PAD>((d + r * NS) * W + c)] = v[q][r];
    }
  }
  __syncthreads();
}

template <int N, int W, int NT, bool INV, bool PAD = false, int NS = 1>
__device__ __forceinline__ void fft_run(float2* buf, const float2* tab, int tid) {
  if constexpr (NS < N) {
    constexpr int R = pick_radix(N / NS);
    fft_pass<N, W, NT, INV, R, NS, PAD>(buf, tab, tid);
    fft_run<N, W, NT, INV, PAD, NS * R>(buf, NS > 1 ? tab + NS : tab, tid);
  }
}

// Base twiddle table of fft_run: NS entries per twiddled pass,
// tw_table_size in all; tab[k] of the pass of span NS is tw[k N / (NS R) TS]
// for a table tw of exp(-2 pi i m / (N TS)) (a transform of length N reads
// every TS-th entry of a longer transform's table).
constexpr int tw_table_size(int N) {
  int s = 0;
  for (int NS = 1; NS < N;) {
    if (NS > 1) s += NS;
    NS *= pick_radix(N / NS);
  }
  return s;
}
template <int N>
constexpr int tw_tab_len() {
  return tw_table_size(N) > 0 ? tw_table_size(N) : 1;
}
template <int N, int NT, int NS, int TS>
__device__ __forceinline__ void tw_table(float2* tab, const float2* __restrict__ tw) {
  if constexpr (NS < N) {
    constexpr int R = pick_radix(N / NS), TWS = N / (NS * R);
    if constexpr (NS > 1) {
      for (int k = threadIdx.x; k < NS; k += NT) tab[k] = tw[k * TWS * TS];
      tw_table<N, NT, NS * R, TS>(tab + NS, tw);
    } else {
      tw_table<N, NT, NS * R, TS>(tab, tw);
    }
  }
}

// Z then the forward DFT of one image row (grid length N = Kx = 2 Nx).  The
// row is real, so it runs as one complex transform of half the length on
// z[m] = r[2m] + i r[2m+1]: with Z = DFT_{N/2}(z), E[k] = (Z[k] + conj(Z[-k]))/2
// and O[k] = (Z[k] - conj(Z[-k]))/(2i) are the transforms of the even and odd
// samples, and R[k] = E[k] + w^k O[k], R[k + N/2] = E[k] - w^k O[k]
// (w = exp(-2 pi i / N)).
template <int N, int NT>
__global__ __launch_bounds__(NT) void k_rowfft_fwd(const float* __restrict__ x, float2* __restrict__ half,
                                                   const float* __restrict__ sy, const float* __restrict__ sx,
                                                   const float2* __restrict__ tw, int Ny, int Nx, int l0) {
  constexpr int M = N / 2;
  __shared__ float2 buf[M + M / 16];
  __shared__ float2 tab[tw_tab_len<M>()];
  tw_table<M, NT, 1, 2>(tab, tw);
  const int p = blockIdx.x, l = l0 + blockIdx.y;
  const float* xr = x + ((size_t)l * Ny + p) * Nx;
  const float syp = sy[p];
  auto sample = [&](int n) {  // Z x at grid column n
    const int q = (n < N / 2 ? n : n - N) + Nx / 2;
    return (q >= 0 && q < Nx) ? syp * sx[q] * xr[q] : 0.f;
  };
  for (int m = threadIdx.x; m < M; m += NT) buf[lds_i<true>(m)] = make_float2(sample(2 * m), sample(2 * m + 1));
  __syncthreads();
  fft_run<M, 1, NT, false, true>(buf, tab, threadIdx.x);
  float2* out = half + ((size_t)l * Ny + p) * N;
  for (int kk = threadIdx.x; kk < M; kk += NT) {
    const float2 a = buf[lds_i<true>(kk)], b = buf[lds_i<true>(kk == 0 ? 0 : M - kk)];
    const float2 e = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));  // (Z[k] + conj(Z[-k])) / 2
    const float2 o = make_float2(0.5f * (a.y + b.y), 0.5f * (b.x - a.x));  // (Z[k] - conj(Z[-k])) / (2i)
    const float2 wo = cmul(tw[kk], o);
    out[kk] = make_float2(e.x + wo.x, e.y + wo.y);
    out[kk + M] = make_float2(e.x - wo.x, e.y - wo.y);
  }
}

// Inverse DFT of one half-grid row, then Z^T: crop, scale, real part.  Only
// Re(IDFT(H)) is kept, which is the IDFT of the Hermitian part
// Hs[k] = (H[k] + conj(H[-k]))/2, a real sequence a[n]; its even and odd
// samples come from one complex inverse transform of half the length:
// z = IDFT_{N/2}(Fe + i Fo), Fe[k] = Hs[k] + Hs[k + N/2],
// Fo[k] = (Hs[k] - Hs[k + N/2]) w^-k, a[2m] = Re z[m], a[2m+1] = Im z[m].
template <int N, int NT>
__global__ __launch_bounds__(NT) void k_rowfft_inv(const float2* __restrict__ half, float* __restrict__ x,
                                                   const float* __restrict__ sy, const float* __restrict__ sx,
                                                   const float2* __restrict__ tw, int Ny, int Nx, int l0) {
  constexpr int M = N / 2;
  __shared__ float2 buf[M + M / 16];
  __shared__ float2 tab[tw_tab_len<M>()];
  tw_table<M, NT, 1, 2>(tab, tw);
  const int p = blockIdx.x, l = l0 + blockIdx.y;
  const float2* in = half + ((size_t)l * Ny + p) * N;
  auto herm = [&](int k) {  // Hs[k]
    const float2 a = in[k], b = in[k == 0 ? 0 : N - k];
    return make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
  };
  for (int kk = threadIdx.x; kk < M; kk += NT) {
    const float2 h0 = herm(kk), h1 = herm(kk + M);
    const float2 fe = make_float2(h0.x + h1.x, h0.y + h1.y);
    float2 w = tw[kk];
    w.y = -w.y;  // w^-k
    const float2 fo = cmul(make_float2(h0.x - h1.x, h0.y - h1.y), w);
    buf[lds_i<true>(kk)] = make_float2(fe.x - fo.y, fe.y + fo.x);  // Fe + i Fo
  }
  __syncthreads();
  fft_run<M, 1, NT, true, true>(buf, tab, threadIdx.x);
  float* xr = x + ((size_t)l * Ny + p) * Nx;
  const float syp = sy[p];
  for (int q = threadIdx.x; q < Nx; q += NT) {
    int n = q - Nx / 2;
    if (n < 0) n += N;
    const float2 z = buf[lds_i<true>(n >> 1)];
    xr[q] = ((n & 1) ? z.y : z.x) * syp * sx[q];
  }
}

// Forward DFT along y of a panel of W grid columns; only the Ny centred rows
// of the input are nonzero (they come from the half grid).
template <int N, int W, int NT>
__global__ __launch_bounds__(NT) void k_colfft_fwd(const float2* __restrict__ half, float2* __restrict__ grid,
                                                   const float2* __restrict__ tw, int Ny, int Kx, int l0) {
  __shared__ float2 buf[N * W];
  __shared__ float2 tab[tw_tab_len<N>()];
  tw_table<N, NT, 1, 1>(tab, tw);
  const int np = Kx / W;
  const int c0 = xcd_remap(blockIdx.x, np) * W, l = l0 + blockIdx.y;
  const float2* in = half + (size_t)l * Ny * Kx;
  constexpr int PER = (N * W + NT - 1) / NT;
  float2 v[PER];  // all of a thread's loads go out before the first is used
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT, k = e / W, c = e % W;
    const int p = (k < N / 2 ? k : k - N) + Ny / 2;
    v[i] = make_float2(0.f, 0.f);
    if (e < N * W && p >= 0 && p < Ny) v[i] = in[(size_t)p * Kx + c0 + c];
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N * W) buf[e] = v[i];
  }
  __syncthreads();
  fft_run<N, W, NT, false, false>(buf, tab, threadIdx.x);
  float2* out = grid + (size_t)l * N * Kx;
  for (int e = threadIdx.x; e < N * W; e += NT) {
    const int k = e / W, c = e % W;
    out[(size_t)k * Kx + c0 + c] = buf[e];
  }
}

// Inverse DFT along y of a panel of W grid columns; writes the Ny rows that
// Z^T reads into the half grid.
template <int N, int W, int NT>
__global__ __launch_bounds__(NT) void k_colfft_inv(const float2* __restrict__ grid, float2* __restrict__ half,
                                                   const float2* __restrict__ tw, int Ny, int Kx, int l0) {
  __shared__ float2 buf[N * W];
  __shared__ float2 tab[tw_tab_len<N>()];
  tw_table<N, NT, 1, 1>(tab, tw);
  const int np = Kx / W;
  const int c0 = xcd_remap(blockIdx.x, np) * W, l = l0 + blockIdx.y;
  const float2* in = grid + (size_t)l * N * Kx;
  constexpr int PER = (N * W + NT - 1) / NT;
  float2 v[PER];  // all of a thread's loads go out before the first is used
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N * W) v[i] = in[(size_t)(e / W) * Kx + c0 + e % W];
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N * W) buf[e] = v[i];
  }
  __syncthreads();
  fft_run<N, W, NT, true, false>(buf, tab, threadIdx.x);
  float2* out = half + (size_t)l * Ny * Kx;
  for (int e = threadIdx.x; e < N * W; e += NT) {
    const int k = e / W, c = e % W;
    const int p = (k < N / 2 ? k : k - N) + Ny / 2;
    if (p >= 0 && p < Ny) out[(size_t)p * Kx + c0 + c] = buf[e];
  }
}

// Long columns in two passes (N = N1 N2; row n = n1 + N1 n2 of the input,
// row k = k2 + N2 k1 of the output):
//   X[k2 + N2 k1] = sum_n1 w_N1^(n1 k1) w_N^(n1 k2) sum_n2 x[n1 + N1 n2] w_N2^(n2 k2).
// Pass A takes one n1 per work-group and transforms along n2, applies
// w_N^(n1 k2) and stores row k2 + N2 n1 of the grid; pass B takes one k2 and
// transforms rows k2 + N2 j (j = n1 -> k1) in place.  A work-group holds W
// columns, so each row access is W * 8 contiguous bytes (one column per
// work-group would be 8).  The inverse runs the same passes in reverse order
// with conjugate twiddles.
template <int N1, int N2, int W, int NT>
__global__ __launch_bounds__(NT) void k_colfft2_fwd_a(const float2* __restrict__ half, float2* __restrict__ grid,
                                                      const float2* __restrict__ tw, int Ny, int Kx, int l0) {
  constexpr int N = N1 * N2, PER = (N2 * W + NT - 1) / NT;
  __shared__ float2 buf[N2 * W];
  __shared__ float2 tab[tw_tab_len<N2>()];
  tw_table<N2, NT, 1, N1>(tab, tw);
  const int np = Kx / W;
  const int n1 = blockIdx.x / np, c0 = xcd_remap(blockIdx.x % np, np) * W, l = l0 + blockIdx.y;
  float2 wst[PER];  // store twiddles w_N^(n1 k2), loaded with the data
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    wst[i] = tw[e < N2 * W ? n1 * (e / W) : 0];
  }
  const float2* in = half + (size_t)l * Ny * Kx;
  for (int e = threadIdx.x; e < N2 * W; e += NT) {
    const int n2 = e / W, c = e % W, n = n1 + N1 * n2;
    const int p = (n < N / 2 ? n : n - N) + Ny / 2;
    buf[e] = (p >= 0 && p < Ny) ? in[(size_t)p * Kx + c0 + c] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_run<N2, W, NT, false, false>(buf, tab, threadIdx.x);
  float2* out = grid + (size_t)l * N * Kx + (size_t)N2 * n1 * Kx;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N2 * W) {
      const int k2 = e / W, c = e % W;
      out[(size_t)k2 * Kx + c0 + c] = cmul(buf[e], wst[i]);
    }
  }
}

template <int N1, int N2, int W, int NT, bool INV>
__global__ __launch_bounds__(NT) void k_colfft2_b(float2* __restrict__ grid, const float2* __restrict__ tw, int Kx,
                                                  int l0) {
  constexpr int N = N1 * N2, PER = (N1 * W + NT - 1) / NT;
  __shared__ float2 buf[N1 * W];
  __shared__ float2 tab[tw_tab_len<N1>()];
  tw_table<N1, NT, 1, N2>(tab, tw);
  const int np = Kx / W;
  const int k2 = blockIdx.x / np, c0 = xcd_remap(blockIdx.x % np, np) * W, l = l0 + blockIdx.y;
  float2 wst[PER];  // inverse: conj(w_N^(n1 k2)), loaded with the data
  if (INV) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * NT;
      wst[i] = tw[e < N1 * W ? (e / W) * k2 : 0];
      wst[i].y = -wst[i].y;
    }
  }
  float2* g = grid + (size_t)l * N * Kx + (size_t)k2 * Kx;
  for (int e = threadIdx.x; e < N1 * W; e += NT) {
    const int j = e / W, c = e % W;
    buf[e] = g[(size_t)N2 * j * Kx + c0 + c];
  }
  __syncthreads();
  fft_run<N1, W, NT, INV, false>(buf, tab, threadIdx.x);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N1 * W) {
      const int j = e / W, c = e % W;
      float2 v = buf[e];
      if (INV) v = cmul(v, wst[i]);  // j = n1: conj(w_N^(n1 k2)) before the pass along k2
      g[(size_t)N2 * j * Kx + c0 + c] = v;
    }
  }
}

template <int N1, int N2, int W, int NT>
__global__ __launch_bounds__(NT) void k_colfft2_inv_a(const float2* __restrict__ grid, float2* __restrict__ half,
                                                      const float2* __restrict__ tw, int Ny, int Kx, int l0) {
  constexpr int N = N1 * N2;
  __shared__ float2 buf[N2 * W];
  __shared__ float2 tab[tw_tab_len<N2>()];
  tw_table<N2, NT, 1, N1>(tab, tw);
  const int np = Kx / W;
  const int n1 = blockIdx.x / np, c0 = xcd_remap(blockIdx.x % np, np) * W, l = l0 + blockIdx.y;
  const float2* in = grid + (size_t)l * N * Kx + (size_t)N2 * n1 * Kx;
  for (int e = threadIdx.x; e < N2 * W; e += NT) {
    const int k2 = e / W, c = e % W;
    buf[e] = in[(size_t)k2 * Kx + c0 + c];
  }
  __syncthreads();
  fft_run<N2, W, NT, true, false>(buf, tab, threadIdx.x);
  float2* out = half + (size_t)l * Ny * Kx;
  for (int e = threadIdx.x; e < N2 * W; e += NT) {
    const int n2 = e / W, c = e % W, n = n1 + N1 * n2;
    const int p = (n < N / 2 ? n : n - N) + Ny / 2;
    if (p >= 0 && p < Ny) out[(size_t)p * Kx + c0 + c] = buf[e];
  }
}

// --------------------------------------- image-first 2-D transform (Ky = N1 N2)
// Grids whose columns take two passes (Ky = N1 N2, 3072 ... 8192 points) run
// the 2-D DFT columns first, on the image itself.  Real columns 2c and 2c+1
// are packed as one complex column z = s x_2c + i s x_2c+1 (the Z scales
// applied on load), whose Ky-point DFT Z gives both real columns'
// transforms: T_2c[k] = (Z[k] + conj Z[-k]) / 2, T_2c+1[k] = (Z[k] -
// conj Z[-k]) / (2i).  Each of the Ky rows of T (Nx nonzero inputs of Kx)
// then takes a Kx-point DFT into the grid.  The adjoint mirrors it: rows
// first, keeping the Nx columns Z^T reads, then columns, of which only the
// real part is kept: that is the inverse DFT of the Hermitian part
// (t[k] + conj t[-k]) / 2, and two such real-output transforms are packed
// as one complex transform.  Per channel and direction this moves
// 4 N + 4 K (image, packed columns between the column passes: 2 K each
// way) + 4 K (T) + 12 K (rows) bytes instead of the 28 K + 4 N of rows first.
//
// Column pass A (forward): one n1 per work-group, W packed columns; rows
// n = n1 + N1 n2 of the image (centred wrap), transform along n2, twiddle
// w_N^(n1 k2), store packed row k2 + N2 n1 of zp [Ky][Nx/2].
template <int N1, int N2, int W, int NT>
__global__ __launch_bounds__(NT) void k_colr_fwd_a(const float* __restrict__ x, float2* __restrict__ zp,
                                                   const float* __restrict__ sy, const float* __restrict__ sx,
                                                   const float2* __restrict__ tw, int Ny, int Nx, int l0,
                                                   size_t zs) {
  constexpr int N = N1 * N2, PER = (N2 * W + NT - 1) / NT;
  __shared__ float2 buf[N2 * W];
  __shared__ float2 tab[tw_tab_len<N2>()];
  tw_table<N2, NT, 1, N1>(tab, tw);
  const int Nh = Nx / 2, npc = Nh / W;
  const int n1 = blockIdx.x / npc, c0 = xcd_remap(blockIdx.x % npc, npc) * W, l = l0 + blockIdx.y;
  float2 wst[PER];  // store twiddles w_N^(n1 k2), loaded with the data
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    wst[i] = tw[e < N2 * W ? n1 * (e / W) : 0];
  }
  // a thread's elements share one column pair (NT is a multiple of W); all
  // its loads go out before the first is used
  static_assert(NT % W == 0, "one column pair per thread");
  const float* xi = x + (size_t)l * Ny * Nx;
  const int q = 2 * (c0 + (int)threadIdx.x % W);
  const float sxa = sx[q], sxb = sx[q + 1];
  float2 xv[PER];
  float sv[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT, n = n1 + N1 * (e / W);
    const int p = (n < N / 2 ? n : n - N) + Ny / 2;
    xv[i] = make_float2(0.f, 0.f);
    sv[i] = 0.f;
    if (e < N2 * W && p >= 0 && p < Ny) {
      xv[i] = *reinterpret_cast<const float2*>(xi + (size_t)p * Nx + q);
      sv[i] = sy[p];
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N2 * W) buf[e] = make_float2(sv[i] * sxa * xv[i].x, sv[i] * sxb * xv[i].y);
  }
  __syncthreads();
  fft_run<N2, W, NT, false, false>(buf, tab, threadIdx.x);
  float2* out = zp + (size_t)l * zs + (size_t)N2 * n1 * Nh;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N2 * W) {
      const int k2 = e / W, c = e % W;
      out[(size_t)k2 * Nh + c0 + c] = cmul(buf[e], wst[i]);
    }
  }
}

// Entry of k = k2 + N2 k1 that holds Z[-k]: (group, k1) of the pair
// (k2a, k2b = (N2 - k2a) mod N2) a work-group holds (group 0 is k2a).
template <int N1, int N2>
__device__ __forceinline__ int mirror_k1(int k2, int k1) {
  return k2 == 0 ? (N1 - k1) % N1 : N1 - 1 - k1;
}

// Column pass B (forward): the pair of k2 groups (k2a, N2 - k2a) per
// work-group, transform along n1 -> k1 in place, then the split of each
// packed column into its two real columns' transforms, written as T rows
// k = k2 + N2 k1 [Ky][Nx].
template <int N1, int N2, int W, int NT>
__global__ __launch_bounds__(NT) void k_colr_fwd_b(const float2* __restrict__ zp, float2* __restrict__ T,
                                                   const float2* __restrict__ tw, int Nx, int l0, size_t zs) {
  constexpr int N = N1 * N2, W2 = 2 * W;
  __shared__ float2 buf[N1 * W2];  // (k1, col): col < W group a, >= W group b
  __shared__ float2 tab[tw_tab_len<N1>()];
  tw_table<N1, NT, 1, N2>(tab, tw);
  const int Nh = Nx / 2, npc = Nh / W;
  const int g = blockIdx.x / npc, c0 = xcd_remap(blockIdx.x % npc, npc) * W, l = l0 + blockIdx.y;
  const int k2a = g, k2b = (N2 - g) % N2;
  const float2* in = zp + (size_t)l * zs;
  constexpr int PER = (N1 * W2 + NT - 1) / NT;
  float2 zv[PER];  // all of a thread's loads go out before the first is used
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N1 * W2) {
      const int j = e / W2, col = e % W2, c = col % W, k2 = col < W ? k2a : k2b;
      zv[i] = in[(size_t)(N2 * j + k2) * Nh + c0 + c];
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N1 * W2) buf[e] = zv[i];
  }
  __syncthreads();
  fft_run<N1, W2, NT, false, false>(buf, tab, threadIdx.x);
  float4* out = reinterpret_cast<float4*>(T + (size_t)l * N * Nx);
  const bool two = k2b != k2a;
  for (int e = threadIdx.x; e < N1 * W2; e += NT) {
    const int k1 = e / W2, col = e % W2, grp = col / W, c = col % W;
    if (grp == 1 && !two) continue;
    const int k2 = grp ? k2b : k2a;
    // Z[-k] lives in the other group (or the same one when self-paired)
    const int mg = two ? 1 - grp : 0, mk1 = mirror_k1<N1, N2>(k2, k1);
    const float2 z = buf[e], zm = buf[mk1 * W2 + mg * W + c];
    // T_2c = (z + conj zm) / 2, T_2c+1 = (z - conj zm) / (2i)
    const float2 a = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
    const float2 b = make_float2(0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x));
    out[((size_t)(k2 + N2 * k1) * Nx) / 2 + c0 + c] = make_float4(a.x, a.y, b.x, b.y);
  }
}

// Row passes.  Forward: row k of T (Nx values, centred in Kx = N cells) to
// grid row k.  Input cell n is nonzero for n < Nx/2 or n >= N - Nx/2, so
// with M = N/2 = Nx: X[2k'] = DFT_M(u)[k'], X[2k'+1] = DFT_M(v)[k'] with
// u[m] = T[(m + Nx/2) mod Nx] and v[m] = +-u[m] w_N^m (minus for m >= Nx/2);
// u and v run interleaved, so the transformed buffer is the grid row.
// Inverse: grid row k to row k of T' (the Nx kept columns):
// x[n] = E[n mod M] + w_N^-n O[n mod M] with E, O the inverse DFTs of the
// even and odd samples, run interleaved.
//
// Both are persistent: a work-group loops over rows r = blockIdx.x +
// i gridDim.x of the nl Ky rows, with its pass twiddles in an LDS table
// (fft_run), and loads row r + gridDim.x into registers before it
// transforms row r, so the loads of one row overlap the LDS passes and the
// stores of the other.  w^m of the load (w^-n of the store) is w^tid times
// a uniform table entry (the inverse takes w^tid from an LDS table of the 64
// lane values and a uniform entry, to keep its registers for the prefetch).
template <int N>
constexpr int rowc_threads() {
  return N / 8 < 64 ? 64 : N / 8 > 1024 ? 1024 : N / 8;
}
// Waves per SIMD the LDS allows (160 KiB per CU, 8 waves per SIMD at most):
// the register budget the long rows are compiled for.
template <int N, int NT>
constexpr int rowc_waves() {
  constexpr int waves = (NT + 63) / 64, lds = (N + N / 16) * 8;
  constexpr int wgs = 163840 / lds < 32 / waves ? 163840 / lds : 32 / waves;
  constexpr int w = wgs * waves / 4;
  return N < 2048 ? 1 : w < 1 ? 1 : w > 8 ? 8 : w;
}
template <int N, int NT>
__global__ __launch_bounds__(NT, (rowc_waves<N, NT>())) void k_rowc_fwd_p(const float2* __restrict__ T,
                                                                   float2* __restrict__ grid,
                                                                   const float2* __restrict__ tw, int Ky, int l0,
                                                                   int nrows) {
  constexpr int M = N / 2, Nx = M, PT = (M + NT - 1) / NT, NW = tw_table_size(M);
  __shared__ float2 buf[N + N / 16];  // padded
  __shared__ float2 tab[NW > 0 ? NW : 1];
  const int tid = threadIdx.x;
  tw_table<M, NT, 1, 2>(tab, tw);
  const float2 wb = tid < N ? tw[tid] : make_float2(1.f, 0.f);  // w^tid
  float2 u[PT];
  auto load = [&](int r) {
    const int l = l0 + r / Ky, k = r % Ky;
    const float2* t = T + ((size_t)l * Ky + k) * Nx;
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int m = tid + q * NT;
      if (M % NT == 0 || m < M) u[q] = t[m < Nx / 2 ? m + Nx / 2 : m - Nx / 2];
    }
  };
  int r = blockIdx.x;
  if (r < nrows) load(r);
  for (; r < nrows; r += gridDim.x) {
    // per-iteration copies the compiler cannot see through (see fft_pass)
    int tl = tid;
    float2 wl = wb;
    asm volatile("" : "+v"(tl), "+v"(wl.x), "+v"(wl.y));
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int m = tl + q * NT;
      if (M % NT == 0 || m < M) {
        const float2 uw = cmul(u[q], cmul(wl, tw[q * NT]));
        buf[lds_i<true>(2 * m)] = u[q];
        buf[lds_i<true>(2 * m + 1)] = m < Nx / 2 ? uw : make_float2(-uw.x, -uw.y);
      }
    }
    if (r + (int)gridDim.x < nrows) load(r + gridDim.x);
    __syncthreads();
    fft_run<M, 2, NT, false, true>(buf, tab, tl);
    const int l = l0 + r / Ky, k = r % Ky;
    float4* out = reinterpret_cast<float4*>(grid + ((size_t)l * Ky + k) * N);
    for (int i = tl; i < M; i += NT) {
      const float2 a = buf[lds_i<true>(2 * i)], b = buf[lds_i<true>(2 * i + 1)];
      out[i] = make_float4(a.x, a.y, b.x, b.y);
    }
    __syncthreads();
  }
}

// (6144-point rows at half the threads hold 8 prefetched elements per thread
// through radix-3 passes: 3 waves per SIMD, not the 4 the LDS would allow.)
template <int N, int NT>
constexpr int rowc_inv_waves() {
  return N == 6144 && rowc_waves<N, NT>() > 3 ? 3 : rowc_waves<N, NT>();
}
template <int N, int NT>
__global__ __launch_bounds__(NT, (rowc_inv_waves<N, NT>())) void k_rowc_inv_p(const float2* __restrict__ grid,
                                                                   float2* __restrict__ T,
                                                                   const float2* __restrict__ tw, int Ky, int l0,
                                                                   int nrows, LiveRegions live) {
  constexpr int M = N / 2, Nx = M, PT = (M + NT - 1) / NT, NW = tw_table_size(M);
  __shared__ float2 buf[N + N / 16];  // padded
  __shared__ float2 tab[NW > 0 ? NW : 1];
  __shared__ float2 s_lane[64];  // w^lane
  const int tid = threadIdx.x;
  tw_table<M, NT, 1, 2>(tab, tw);
  if (tid < 64) s_lane[tid] = tid < N ? tw[tid] : make_float2(1.f, 0.f);
  float4 v[PT];
  // With live regions, a wave's 64 element pairs (128 cells) lie in
  // 128 / R <= 8 regions of one mask word (R >= 16, a power of two): where
  // none of them is live the wave loads nothing (its cells are zero); the
  // test is wave-uniform.
  const int wave_pair0 = __builtin_amdgcn_readfirstlane(tid & ~63);  // the wave's first pair (at q = 0)
  auto load = [&](int r) {
    const int l = l0 + r / Ky, k = r % Ky;
    const float4* in = reinterpret_cast<const float4*>(grid + ((size_t)l * Ky + k) * N);
    const uint32_t* mrow = live.bits ? live.bits + ((size_t)l * (Ky / live.R) + k / live.R) * live.wpr : nullptr;
    uint32_t word[PT];  // the mask words, all loaded before the first test
#pragma unroll
    for (int q = 0; q < PT; ++q) word[q] = mrow ? mrow[(2 * (wave_pair0 + q * NT) / live.R) >> 5] : ~0u;
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int i = tid + q * NT;
      if (M % NT == 0 || i < M) {
        const int reg0 = 2 * (wave_pair0 + q * NT) / live.R, nreg = 128 / live.R;
        const bool dead = mrow && ((word[q] >> (reg0 & 31)) & ((1u << nreg) - 1u)) == 0u;
        if (dead) {
          v[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
          v[q] = in[i];
        }
      }
    }
  };
  int r = blockIdx.x;
  if (r < nrows) load(r);
  for (; r < nrows; r += gridDim.x) {
    // per-iteration copy the compiler cannot see through (see fft_pass)
    int tl = tid;
    asm volatile("" : "+v"(tl));
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int i = tl + q * NT;
      if (M % NT == 0 || i < M) {
        buf[lds_i<true>(2 * i)] = make_float2(v[q].x, v[q].y);
        buf[lds_i<true>(2 * i + 1)] = make_float2(v[q].z, v[q].w);
      }
    }
    if (r + (int)gridDim.x < nrows) load(r + gridDim.x);
    __syncthreads();
    fft_run<M, 2, NT, true, true>(buf, tab, tl);
    const int l = l0 + r / Ky, k = r % Ky;
    float2* t = T + ((size_t)l * Ky + k) * Nx;
    // w^-tid = conj(w^lane w^wave_base): an LDS entry and a uniform (scalar) load
    const int wbase = __builtin_amdgcn_readfirstlane(tl & ~63);
    float2 wl = cmul(s_lane[tl & 63], tw[wbase < N ? wbase : 0]);
    wl.y = -wl.y;
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int c = tl + q * NT;
      if (Nx % NT == 0 || c < Nx) {
        // x[c] = E[m] + w^-n O[m]: n = (c - Nx/2) mod N, m = n mod M
        const int m = c >= Nx / 2 ? c - Nx / 2 : c + Nx / 2;
        float2 wu = tw[((q * NT - Nx / 2) % N + N) % N];
        wu.y = -wu.y;
        const float2 o = cmul(buf[lds_i<true>(2 * m + 1)], cmul(wl, wu)), e = buf[lds_i<true>(2 * m)];
        t[c] = make_float2(e.x + o.x, e.y + o.y);
      }
    }
    __syncthreads();
  }
}

// Column pass B (inverse): the pair (k2a, N2 - k2a), the Hermitian parts of
// the two real columns of each packed column combined as
// (t2c[k] + conj t2c[-k]) / 2 + i (t2c+1[k] + conj t2c+1[-k]) / 2, inverse
// transform along k1 -> n1, twiddle conj w_N^(n1 k2), store packed rows
// k2 + N2 n1 of zp.
template <int N1, int N2, int W, int NT>
__global__ __launch_bounds__(NT) void k_colr_inv_b(const float2* __restrict__ T, float2* __restrict__ zp,
                                                   const float2* __restrict__ tw, int Nx, int l0, size_t zs) {
  constexpr int N = N1 * N2, W2 = 2 * W, PER = (N1 * W2 + NT - 1) / NT;
  __shared__ float4 raw[N1 * W2];  // (k1, col): the two real columns' T' values
  __shared__ float2 tab[tw_tab_len<N1>()];
  tw_table<N1, NT, 1, N2>(tab, tw);
  float2* buf = reinterpret_cast<float2*>(raw);  // packed values, (k1, col), after the split
  const int Nh = Nx / 2, npc = Nh / W;
  const int g = blockIdx.x / npc, c0 = xcd_remap(blockIdx.x % npc, npc) * W, l = l0 + blockIdx.y;
  const int k2a = g, k2b = (N2 - g) % N2;
  const bool two = k2b != k2a;
  float2 wst[PER];  // store twiddles conj(w_N^(n1 k2)), loaded with the data
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    wst[i] = tw[e < N1 * W2 ? (e / W2) * ((e % W2) / W ? k2b : k2a) : 0];
    wst[i].y = -wst[i].y;
  }
  const float4* in = reinterpret_cast<const float4*>(T + (size_t)l * N * Nx);
  for (int e = threadIdx.x; e < N1 * W2; e += NT) {
    const int j = e / W2, col = e % W2, c = col % W, k2 = col < W ? k2a : k2b;
    raw[e] = in[((size_t)(k2 + N2 * j) * Nx) / 2 + c0 + c];
  }
  __syncthreads();
  float2 h[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N1 * W2) {
      const int k1 = e / W2, col = e % W2, grp = col / W, c = col % W;
      const int k2 = grp ? k2b : k2a;
      const int mg = two ? 1 - grp : 0, mk1 = mirror_k1<N1, N2>(k2, k1);
      const float4 a = raw[e], b = raw[mk1 * W2 + mg * W + c];
      // (a.xy + conj b.xy) / 2 + i (a.zw + conj b.zw) / 2
      h[i] = make_float2(0.5f * (a.x + b.x) - 0.5f * (a.w - b.w), 0.5f * (a.y - b.y) + 0.5f * (a.z + b.z));
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N1 * W2) buf[e] = h[i];
  }
  __syncthreads();
  fft_run<N1, W2, NT, true, false>(buf, tab, threadIdx.x);
  float2* out = zp + (size_t)l * zs;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N1 * W2) {
      const int n1 = e / W2, col = e % W2, grp = col / W, c = col % W;
      const int k2 = grp ? k2b : k2a;
      if (grp == 0 || two) out[(size_t)(k2 + N2 * n1) * Nh + c0 + c] = cmul(buf[e], wst[i]);
    }
  }
}

// Column pass A (inverse): one n1 per work-group, inverse transform along
// k2 -> n2, rows n = n1 + N1 n2 kept by Z^T, real and imaginary parts are the
// two real columns, times the Z scales.
template <int N1, int N2, int W, int NT>
__global__ __launch_bounds__(NT) void k_colr_inv_a(const float2* __restrict__ zp, float* __restrict__ x,
                                                   const float* __restrict__ sy, const float* __restrict__ sx,
                                                   const float2* __restrict__ tw, int Ny, int Nx, int l0,
                                                   size_t zs) {
  constexpr int N = N1 * N2, PER = (N2 * W + NT - 1) / NT;
  static_assert(NT % W == 0, "one column pair per thread");
  __shared__ float2 buf[N2 * W];
  __shared__ float2 tab[tw_tab_len<N2>()];
  tw_table<N2, NT, 1, N1>(tab, tw);
  const int Nh = Nx / 2, npc = Nh / W;
  const int n1 = blockIdx.x / npc, c0 = xcd_remap(blockIdx.x % npc, npc) * W, l = l0 + blockIdx.y;
  const float2* in = zp + (size_t)l * zs + (size_t)N2 * n1 * Nh;
  // all of a thread's loads go out before the first is used (here and for
  // the scales below)
  float2 zv[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N2 * W) zv[i] = in[(size_t)(e / W) * Nh + c0 + e % W];
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < N2 * W) buf[e] = zv[i];
  }
  const int q = 2 * (c0 + (int)threadIdx.x % W);
  const float sxa = sx[q], sxb = sx[q + 1];
  float sv[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT, n = n1 + N1 * (e / W);
    const int p = (n < N / 2 ? n : n - N) + Ny / 2;
    sv[i] = e < N2 * W && p >= 0 && p < Ny ? sy[p] : 0.f;
  }
  __syncthreads();
  fft_run<N2, W, NT, true, false>(buf, tab, threadIdx.x);
  float* xo = x + (size_t)l * Ny * Nx;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT, n = n1 + N1 * (e / W);
    const int p = (n < N / 2 ? n : n - N) + Ny / 2;
    if (e < N2 * W && p >= 0 && p < Ny) {
      const float2 v = buf[e];
      *reinterpret_cast<float2*>(xo + (size_t)p * Nx + q) = make_float2(sv[i] * sxa * v.x, sv[i] * sxb * v.y);
    }
  }
}

// ------------------------------------------------------------ G (gather)
// Raw G storage per precision: complex float, or two 16-bit halves in a word.
template <int GP>
struct GRaw {
  using T = uint32_t;
};
template <>
struct GRaw<0> {
  using T = float2;
};
// (gx, gy) of a raw tap.  The FP16 halves stay 16-bit so that the multiply
// below can take them straight into a mixed-precision FMA.
template <int GP>
__device__ __forceinline__ float g_re(typename GRaw<GP>::T r) {
  if constexpr (GP == 0) {
    return r.x;
  } else if constexpr (GP == 1) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(r & 0xFFFFu));
  } else {
    return __uint_as_float(r << 16);
  }
}
template <int GP>
__device__ __forceinline__ float g_im(typename GRaw<GP>::T r) {
  if constexpr (GP == 0) {
    return r.y;
  } else if constexpr (GP == 1) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(r >> 16));
  } else {
    return __uint_as_float(r & 0xFFFF0000u);
  }
}

// Lane sums for the gather, in a fixed order.  v_permlane32_swap folds the
// 32-lane halves of two vectors into one (lanes 0-31 carry the first vector's
// half sums, 32-63 the second's); v_permlane16_swap folds 16-lane rows the
// same way; the DPP steps then sum inside each 16-lane row.
__device__ __forceinline__ float fold32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float fold16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float row_sum16(float v) {
  v += dppf<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dppf<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dppf<0x141>(v);  // row_half_mirror
  v += dppf<0x140>(v);  // row_mirror
  return v;
}
// Sums over 64 lanes of (a0, a1) for one window: returns (sum a0, sum a1).
__device__ __forceinline__ float2 lane_sum1(float a0, float a1) {
  const float h = fold32(a0, a1);           // [a0 | a1] in 32-lane halves
  const float q = row_sum16(fold16(h, h));  // rows: a0, a0, a1, a1
  return make_float2(readlane_f(q, 0), readlane_f(q, 32));
}
// Two windows p and q as one vector: its 16-lane rows hold sum p0, sum q0,
// sum p1, sum q1 (every lane of a row the row's sum).
__device__ __forceinline__ float lane_sum2v(float p0, float p1, float q0, float q1) {
  return row_sum16(fold16(fold32(p0, p1), fold32(q0, q1)));
}
// Two windows p and q: (sum p0, sum p1, sum q0, sum q1).
__device__ __forceinline__ float4 lane_sum2(float p0, float p1, float q0, float q1) {
  const float q = lane_sum2v(p0, p1, q0, q1);
  return make_float4(readlane_f(q, 0), readlane_f(q, 32), readlane_f(q, 16), readlane_f(q, 48));
}

// One wave streams the G taps of consecutive windows of a work item.  Lanes
// span the S*S taps of a window (row-major) in NK steps of 64 (NK = steps of
// the item's largest window), so every fetch issues exactly NK loads at
// fixed per-lane offsets (k * 64 + lane taps) from the window's first tap
// (uniform).  Lanes past a smaller window read the next window's taps (or the
// zero pad behind G); their products meet the zero cell (gather) or the
// lane's spare cell (scatter), so they never reach a result.  The window's
// metadata word comes from two C-visibility chunks held one per lane (the
// fetch runs up to D <= C windows ahead).
template <int GP, int NK, int C>
struct GStream {
  using R = typename GRaw<GP>::T;
  const char* __restrict__ G;
  int64_t tap;      // next window's first tap
  int64_t tap_end;  // re-read target once the range is exhausted
  int j, v1;
  __device__ __forceinline__ void fetch(R (&g)[NK], uint32_t& m, uint32_t mcur, uint32_t mnxt, int cb, int lane) {
    const bool live = j < v1;
    const int rel = j - cb;  // < C + D
    const uint32_t ma = (uint32_t)__builtin_amdgcn_readlane((int)mcur, rel & 63);
    const uint32_t mb = (uint32_t)__builtin_amdgcn_readlane((int)mnxt, (rel - C) & 63);
    const uint32_t mt = live ? (rel < C ? ma : mb) : 0u;
    m = mt;
    const int s = 2 * (int)(mt >> 26) + 1;
    const R* __restrict__ gp = reinterpret_cast<const R*>(G) + (live ? tap : tap_end);
#pragma unroll
    for (int k = 0; k < NK; ++k) g[k] = gp[k * 64 + lane];
    tap = uniform64(tap + (live ? s * s : 0));
    ++j;
  }
};

// Windows per chunk for a prefetch depth of D windows: the largest multiple
// of D that fits a wave, so every chunk starts at ring slot 0 and the chunk
// bookkeeping (metadata rotation, per-visibility vectors, stores) sits at one
// point between groups of D windows instead of inside them.
template <int D>
constexpr int chunk_len() {
  return D * (64 / D);
}

// Per-S lane layout of a window inside a pitch-P LDS tile: the byte offset of
// each step's cell from the window origin.  Lanes past the window hold a
// large offset, and the address min(base + off, park) sends them to the fixed
// cell `park` (a zero cell for the gather, a private spare cell for the
// scatter), so no step needs a mask or a divergent branch.
template <int NK>
struct TapLayout {
  int S = -1;
  uint32_t off[NK];  // bytes; 0x40000000 past the window
  __device__ __forceinline__ void set(int s, int P, int lane) {
    S = s;
    const int S2 = s * s;
    const float rS = __builtin_amdgcn_rcpf((float)s);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int t = k * 64 + lane;
      const uint32_t cell = (uint32_t)(t + tap_row(min(t, S2 - 1), rS) * (P - s));  // row * P + column
      off[k] = t < S2 ? cell * 8u : 0x40000000u;
    }
  }
  __device__ __forceinline__ uint32_t addr(uint32_t base_b, int k, uint32_t park) const {
    return min(base_b + off[k], park);
  }
};

// One wave per work item (a run of plan-order visibilities of one block whose
// window origins lie in one T x T uv tile).  The per-visibility sum over the
// window's taps is a fixed-order lane reduction, taken for two windows at a
// time.
//
// Latency hiding: the G taps of the next D windows are loaded into registers
// while the current windows are reduced.  Each fetch issues exactly NK loads
// and the steady-state loop has no guarded fetch, so the wait before a window
// is used always leaves the later fetches in flight.  NK is a template
// parameter picked per item at run time (1..7 for S <= 21).
//
// Gather: the item's grid region (its tile plus the window halo, wrapped
// periodically) is first copied into LDS, so each window reads its S*S cells
// from LDS and only G streams through the vector memory path.  Lane i of
// each chunk keeps visibility i's result: the residual, its FP64 norms and
// the stores are lane-parallel and coalesced.
//
// Prefetch depth: about PHI_GATHER_DEPTH_REGS (gather) or
// PHI_SCATTER_DEPTH_REGS (scatter) registers of 32-bit taps in flight per
// wave (half as many windows for complex64); deeper prefetch costs
// occupancy.
#ifndef PHI_GATHER_DEPTH_REGS
#define PHI_GATHER_DEPTH_REGS 8
#endif
#ifndef PHI_SCATTER_DEPTH_REGS
#define PHI_SCATTER_DEPTH_REGS 16
#endif
// The one-pass dual step runs few waves per SIMD (its LDS holds a tile and
// an accumulator per wave) and keeps more taps in flight, except for plans
// whose windows all take one 64-tap step (S <= 8): there registers set the
// occupancy, and a shallower ring with a smaller prefetch of the next item's
// region (512 cells: a 16-cell tile with 7 x 7 windows) runs 6 waves per
// SIMD instead of 4 (16 x 4096^2 workload: 14.80 -> 12.68 ms; depth 4: 12.66,
// 2: 13.31; the deeper ring stays for larger windows, 4.85 against 4.93 ms on
// the 1024^2 workload with windows up to 17 x 17).
#ifndef PHI_FUSED_PREFETCH_CELLS
#define PHI_FUSED_PREFETCH_CELLS 1024
#endif
#ifndef PHI_FUSED_DEPTH_REGS
#define PHI_FUSED_DEPTH_REGS 16
#endif
#ifndef PHI_FUSED_PREFETCH_CELLS_S8
#define PHI_FUSED_PREFETCH_CELLS_S8 512
#endif
#ifndef PHI_FUSED_DEPTH_REGS_S8
#define PHI_FUSED_DEPTH_REGS_S8 8
#endif
template <int GP, int NK, int REGS>
struct Depth {
  static constexpr int regs = GP == 0 ? REGS / 2 : REGS;
  static constexpr int value = (regs / NK) < 2 ? 2 : regs / NK;
};

// MODE 0: y = Phi x.  MODE 1: c = v / sigma + Phi x - y with FP64 norms.
// MODE 2: as MODE 1, and each window's c is also added as conj(g) c into
// this wave's LDS accumulator (byte offset ab, pitch P, a spare cell per lane
// behind it) with the same G taps: the dual step's G^H without reading G
// again (the per-block factor sigma * scale * theta comes later, in the
// merge).
template <int GP, int MODE, int NK, int D>
__device__ __forceinline__ int64_t gather_item(const GArgs& a, const Item& item, int v0, int v1, int64_t tap0,
                                            float2* __restrict__ vis, const float2* __restrict__ yv,
                                            double& rho2, double& res2, const float2* __restrict__ tile,
                                            uint32_t ab = 0) {
  using R = typename GRaw<GP>::T;
  constexpr int C = chunk_len<D>();
  const int lane = threadIdx.x & 63;
  const int vlast = v1 - 1, P = item.pitch;
  const float th = a.theta[item.blk];
  float inv_sig = 1.f;
  if (MODE >= 1 && a.sigma) inv_sig = (float)(1.0 / a.sigma[item.blk]);
  // C-visibility chunks held one value per lane (lanes < C): metadata of
  // chunks cb and cb + C (read per window) with cb + 2C in flight; for
  // chunk cb, y and pre = v / sigma - y (c = theta sum + pre), with v and y
  // of chunk cb + C in flight.  These registers are only rotated between
  // chunks, so no wait for a chunk load falls between a window's G fetch and
  // its use (such a wait would drain the prefetch).
  int cb = v0;
  uint32_t mcur = a.meta[min(cb + lane, vlast)];
  uint32_t mnxt = a.meta[min(cb + C + lane, vlast)];
  uint32_t mstg = a.meta[min(cb + 2 * C + lane, vlast)];
  float2 pre = make_float2(0.f, 0.f), yc = pre, vstg = pre, ystg = pre;
  auto pre_of = [&](float2 v, float2 y) {
    return make_float2(__builtin_fmaf(v.x, inv_sig, -y.x), __builtin_fmaf(v.y, inv_sig, -y.y));
  };
  if (MODE >= 1) {
    yc = yv[min(cb + lane, vlast)];
    pre = pre_of(vis[min(cb + lane, vlast)], yc);
    vstg = vis[min(cb + C + lane, vlast)];
    ystg = yv[min(cb + C + lane, vlast)];
  }
  R gb[D][NK];
  uint32_t ms[D];
  GStream<GP, NK, C> gs{static_cast<const char*>(a.G), uniform64(tap0), uniform64(tap0), v0, v1};
  TapLayout<NK> lay;
  float2 res = make_float2(0.f, 0.f);  // lane i: sum for visibility cb + i (theta applied at flush)
  auto flush = [&]() {
    if (lane < C && cb + lane < v1) {
      const float px = th * res.x, py = th * res.y;
      if (MODE == 0) {
        vis[cb + lane] = make_float2(px, py);
      } else {
        const float2 c = make_float2(__builtin_fmaf(th, res.x, pre.x), __builtin_fmaf(th, res.y, pre.y));
        vis[cb + lane] = c;
        const double rx = (double)px - (double)yc.x, ry = (double)py - (double)yc.y;
        rho2 += (double)c.x * (double)c.x + (double)c.y * (double)c.y;
        res2 += rx * rx + ry * ry;
      }
    }
  };
  auto rotate = [&]() {
    cb += C;
    mcur = mnxt;
    mnxt = mstg;
    mstg = a.meta[min(cb + 2 * C + lane, vlast)];
    if (MODE >= 1) {
      pre = pre_of(vstg, ystg);
      yc = ystg;
      vstg = vis[min(cb + C + lane, vlast)];
      ystg = yv[min(cb + C + lane, vlast)];
    }
    res = make_float2(0.f, 0.f);
  };
  // lanes past a window read the zero cell behind the tile
  const uint32_t tb = lds_offset(tile);
  const uint32_t park = tb + (uint32_t)(P * P) * 8u;
  // Every window of a run has NK steps (S^2 > 64 (NK - 1)), so each step
  // holds taps and the NK cell reads go out together, without branches.
  auto cells = [&](uint32_t mt, float2(&X)[NK]) {
    const int by = mt & 8191, bx = (mt >> 13) & 8191, S = 2 * (int)(mt >> 26) + 1;
    if (S != lay.S) lay.set(S, P, lane);
    const uint32_t base_b = tb + (uint32_t)((by - item.ty0) * P + (bx - item.tx0)) * 8u;
#pragma unroll
    for (int k = 0; k < NK; ++k) X[k] = lds_load(lay.addr(base_b, k, park));
  };
  auto dot = [&](const R(&g)[NK], const float2(&X)[NK], float& ax, float& ay) {
    ax = 0.f;
    ay = 0.f;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const float gx = g_re<GP>(g[k]), gy = g_im<GP>(g[k]);
      ax = __builtin_fmaf(gx, X[k].x, ax);
      ax = __builtin_fmaf(-gy, X[k].y, ax);
      ay = __builtin_fmaf(gx, X[k].y, ay);
      ay = __builtin_fmaf(gy, X[k].x, ay);
    }
  };
  // this lane's partial (sum over its taps of g * X) for one window
  auto partial = [&](const R(&g)[NK], uint32_t mt, float& ax, float& ay) {
    float2 X[NK];
    cells(mt, X);
    dot(g, X, ax, ay);
  };
  auto place = [&](int rel, float px, float py) {  // rel = visibility - cb; rel, px, py wave-uniform
    res.x = writelane_f(res.x, px, rel);
    res.y = writelane_f(res.y, py, rel);
  };
  // MODE 2: c of a window from its sum (the same operations as the flush, so
  // the c added here is the c written to v), then conj(g) c into the
  // accumulator: read the window's cells, add, write (distinct cells); the
  // block's theta joins sigma * scale in the merge
  auto cval = [&](int rel, float sx, float sy) {
    return make_float2(__builtin_fmaf(th, sx, readlane_f(pre.x, rel)), __builtin_fmaf(th, sy, readlane_f(pre.y, rel)));
  };
  // Windows in pairs (rel, rel + 1): both c in one lane-parallel step on the
  // pair's sum vector (rows: x of the first, x of the second, y of the
  // first, y of the second), each lane taking the pre of its row's window
  // and component from that window's lane (ds_bpermute); the same operation
  // as cval, lane by lane.
  const int pair_lane_b = ((lane >> 4) & 1) * 4;  // byte offset of the row's window from rel
  const bool pair_y = lane >= 32;
  auto pre_pair = [&](int rel) {
    const int src = rel * 4 + pair_lane_b;
    const float px = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(pre.x)));
    const float py = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(pre.y)));
    return pair_y ? py : px;
  };
  const uint32_t apark = ab + (uint32_t)(P * P + lane) * 8u;  // this lane's spare cell
  // accumulator cells of a window, read ahead of its c (addresses kept for
  // the write-back; the layout may change before then)
  auto acc_cells = [&](uint32_t mt, float2(&A)[NK], uint32_t(&adr)[NK]) {
    const int by = mt & 8191, bx = (mt >> 13) & 8191, S = 2 * (int)(mt >> 26) + 1;
    if (S != lay.S) lay.set(S, P, lane);
    const uint32_t base_b = ab + (uint32_t)((by - item.ty0) * P + (bx - item.tx0)) * 8u;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      adr[k] = lay.addr(base_b, k, apark);
      A[k] = lds_load(adr[k]);
    }
  };
  auto scatter_to = [&](const R(&g)[NK], float2(&A)[NK], const uint32_t(&adr)[NK], float2 c) {
    const float vx = c.x, vy = c.y;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const float gx = g_re<GP>(g[k]), gy = g_im<GP>(g[k]);
      A[k].x = __builtin_fmaf(gx, vx, A[k].x);
      A[k].x = __builtin_fmaf(gy, vy, A[k].x);
      A[k].y = __builtin_fmaf(gx, vy, A[k].y);
      A[k].y = __builtin_fmaf(-gy, vx, A[k].y);
      lds_store(adr[k], A[k]);
    }
  };
  auto scatter = [&](const R(&g)[NK], uint32_t mt, float2 c) {
    const int by = mt & 8191, bx = (mt >> 13) & 8191, S = 2 * (int)(mt >> 26) + 1;
    if (S != lay.S) lay.set(S, P, lane);
    const uint32_t base_b = ab + (uint32_t)((by - item.ty0) * P + (bx - item.tx0)) * 8u;
    const float vx = c.x, vy = c.y;
    float2 cur[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) cur[k] = lds_load(lay.addr(base_b, k, apark));
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const float gx = g_re<GP>(g[k]), gy = g_im<GP>(g[k]);
      cur[k].x = __builtin_fmaf(gx, vx, cur[k].x);
      cur[k].x = __builtin_fmaf(gy, vy, cur[k].x);
      cur[k].y = __builtin_fmaf(gx, vy, cur[k].y);
      cur[k].y = __builtin_fmaf(-gy, vx, cur[k].y);
      lds_store(lay.addr(base_b, k, apark), cur[k]);
    }
  };
#pragma unroll
  for (int d = 0; d < D; ++d) gs.fetch(gb[d], ms[d], mcur, mnxt, cb, lane);
  // window at slot d of a group (rel = its offset in the chunk); fetch > 0
  // refills the slot with the window D ahead
  auto single = [&](int d, int rel, bool refill) {
    float ax, ay;
    partial(gb[d], ms[d], ax, ay);
    if (MODE != 2 && refill) gs.fetch(gb[d], ms[d], mcur, mnxt, cb, lane);
    const float2 s = lane_sum1(ax, ay);
    place(rel, s.x, s.y);
    if (MODE == 2) {
      scatter(gb[d], ms[d], cval(rel, s.x, s.y));
      if (refill) gs.fetch(gb[d], ms[d], mcur, mnxt, cb, lane);
    }
  };
  // A slot's refill must not be issued before the slot's old taps are
  // consumed: if both are live at once, the slot needs a second register
  // and the copy back at the end of the group waits for the refill load,
  // which drains the whole prefetch.  The partial sums are pinned here (an
  // empty statement that takes them and orders memory accesses around it).
  auto settle = [](float& x, float& y) { asm volatile("" : "+v"(x), "+v"(y) : : "memory"); };
  // one group: D windows at slots 0..D-1, reduced in pairs
  auto group = [&](int rel0) {
#pragma unroll
    for (int d = 0; d + 1 < D; d += 2) {
      float ax0, ay0, ax1, ay1;
      if constexpr (MODE == 2 && NK <= 3) {
        // The first window's accumulator cells are read with the grid cells
        // (the previous pair's writes precede them in the wave's LDS order);
        // the second window's are read after the first's write-back, since
        // the two may share cells.
        float2 X0[NK], X1[NK], A0[NK];
        uint32_t adr0[NK];
        const float pv = pre_pair(rel0 + d);
        cells(ms[d], X0);
        acc_cells(ms[d], A0, adr0);
        cells(ms[d + 1], X1);
        dot(gb[d], X0, ax0, ay0);
        settle(ax0, ay0);
        dot(gb[d + 1], X1, ax1, ay1);
        settle(ax1, ay1);
        const float qv = lane_sum2v(ax0, ay0, ax1, ay1);
        const float cv = __builtin_fmaf(th, qv, pv);
        place(rel0 + d, readlane_f(qv, 0), readlane_f(qv, 32));
        scatter_to(gb[d], A0, adr0, make_float2(readlane_f(cv, 0), readlane_f(cv, 32)));
        gs.fetch(gb[d], ms[d], mcur, mnxt, cb, lane);
        place(rel0 + d + 1, readlane_f(qv, 16), readlane_f(qv, 48));
        scatter(gb[d + 1], ms[d + 1], make_float2(readlane_f(cv, 16), readlane_f(cv, 48)));
        gs.fetch(gb[d + 1], ms[d + 1], mcur, mnxt, cb, lane);
        continue;
      } else if constexpr (NK <= 3) {  // both windows' cell reads in flight together
        float2 X0[NK], X1[NK];
        cells(ms[d], X0);
        cells(ms[d + 1], X1);
        dot(gb[d], X0, ax0, ay0);
        settle(ax0, ay0);
        if (MODE != 2) gs.fetch(gb[d], ms[d], mcur, mnxt, cb, lane);
        dot(gb[d + 1], X1, ax1, ay1);
      } else {
        partial(gb[d], ms[d], ax0, ay0);
        settle(ax0, ay0);
        if (MODE != 2) gs.fetch(gb[d], ms[d], mcur, mnxt, cb, lane);
        partial(gb[d + 1], ms[d + 1], ax1, ay1);
      }
      settle(ax1, ay1);
      if (MODE != 2) gs.fetch(gb[d + 1], ms[d + 1], mcur, mnxt, cb, lane);
      if constexpr (MODE == 2) {
        const float qv = lane_sum2v(ax0, ay0, ax1, ay1);
        const float cv = __builtin_fmaf(th, qv, pre_pair(rel0 + d));
        place(rel0 + d, readlane_f(qv, 0), readlane_f(qv, 32));
        scatter(gb[d], ms[d], make_float2(readlane_f(cv, 0), readlane_f(cv, 32)));
        gs.fetch(gb[d], ms[d], mcur, mnxt, cb, lane);
        place(rel0 + d + 1, readlane_f(qv, 16), readlane_f(qv, 48));
        scatter(gb[d + 1], ms[d + 1], make_float2(readlane_f(cv, 16), readlane_f(cv, 48)));
        gs.fetch(gb[d + 1], ms[d + 1], mcur, mnxt, cb, lane);
      } else {
        const float4 s = lane_sum2(ax0, ay0, ax1, ay1);
        place(rel0 + d, s.x, s.y);
        place(rel0 + d + 1, s.z, s.w);
      }
    }
    if constexpr (D & 1) single(D - 1, rel0 + D - 1, true);
  };
  for (;;) {
    const int n = min(C, v1 - cb);  // windows of this chunk
    const int full = n - n % D;     // in whole groups
    for (int rel = 0; rel < full; rel += D) group(rel);
    if (n < C) {  // last chunk: the rest (< D windows) is already fetched
#pragma unroll
      for (int d = 0; d < D - 1; ++d)
        if (full + d < n) single(d, full + d, false);
      flush();
      break;
    }
    flush();
    if (cb + C >= v1) break;
    rotate();
  }
  return gs.tap;
}

// Step count (64-tap loads) of a window from its metadata word, and the end
// of the run of windows from r0 that share step count k0 (scanned 64 windows
// at a time).  Plans sort windows by S inside each 16 x 16 uv sub-tile, so a
// wave's range holds a few such runs; each run is processed with its own
// step count instead of the item's largest.
__device__ __forceinline__ int meta_steps(uint32_t m) {
  const int s = 2 * (int)(m >> 26) + 1;
  return (s * s + 63) >> 6;
}
__device__ __forceinline__ int steps_run_end(const uint32_t* __restrict__ meta, int r0, int v1, int k0, int lane) {
  for (int c = r0; c < v1; c += 64) {
    const int i = c + lane;
    const bool other = i < v1 && meta_steps(meta[min(i, v1 - 1)]) != k0;
    const uint64_t b = __ballot(other);
    if (b) return c + (int)__builtin_ctzll(b);
  }
  return v1;
}

// kGatherWaves waves per work-group share one LDS copy of the item's grid
// region; wave w takes the w-th quarter of the item's visibilities.  NKM is
// the largest step count instantiated (from the plan's largest window), so a
// plan of small windows does not pay the registers of the 21 x 21 path.
template <int GP, int MODE, int NKM>
__global__ __launch_bounds__(64 * kGatherWaves) void k_gather(GArgs a, float2* __restrict__ vis,
                                                              const float2* __restrict__ yv,
                                                              double* __restrict__ item_norms, int it0, int it1) {
  extern __shared__ float2 tile[];  // P*P cells, a zero cell, then the wave norms
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  constexpr int kThreads = 64 * kGatherWaves;
  // One-pass mode (LDS sets its occupancy, so registers are spare): the next
  // item's grid region is loaded into registers while the current item runs
  // (its loads travel with the first G fetches, which an item waits for
  // anyway), so an item starts with LDS writes instead of a memory round
  // trip.  Item descriptors come two items ahead as one dword per lane,
  // read with readlane, so no scalar load is waited for either.  Regions
  // beyond kPre cells per thread (pitch above 32) are copied at the start.
  constexpr int kPre =
      MODE == 2 ? (NKM == 1 ? PHI_FUSED_PREFETCH_CELLS_S8 : PHI_FUSED_PREFETCH_CELLS) / kThreads : 1;
  constexpr int kFusedRegs = NKM == 1 ? PHI_FUSED_DEPTH_REGS_S8 : PHI_FUSED_DEPTH_REGS;
  constexpr int kWords = (int)(sizeof(Item) / 4);
  const int G = gridDim.x;
  auto cell = [&](int chan, int ty0, int tx0, int P, int e) {  // cell e of a region (rows ty0.., wrapped)
    const int r = e / P, c = e - (e / P) * P;
    int gr = ty0 + r, gc = tx0 + c;
    gr -= (gr >= a.Ky) ? a.Ky : 0;
    gc -= (gc >= a.Kx) ? a.Kx : 0;
    return a.grid[((size_t)chan * a.Ky + gr) * a.Kx + gc];
  };
  auto desc = [&](int i) -> int {
    return (i < it1 && lane < kWords) ? reinterpret_cast<const int*>(a.items + i)[lane] : 0;
  };
  auto field = [](int d, int k) { return __builtin_amdgcn_readlane(d, k); };
  static_assert(offsetof(Item, tap0) == 0 && offsetof(Item, poff) == 8 && offsetof(Item, v0) == 16 &&
                    offsetof(Item, blk) == 24 && offsetof(Item, chan) == 28 && offsetof(Item, ty0) == 32 &&
                    offsetof(Item, tx0) == 36 && offsetof(Item, pitch) == 40 && offsetof(Item, sub) == 48 &&
                    offsetof(Item, slot) == 60 && offsetof(Item, wv) == 64 && sizeof(Item) == 80,
                "descriptor words");
  auto unpack = [&](int d) {
    Item t;
    t.tap0 = (int64_t)(((uint64_t)(uint32_t)field(d, 1) << 32) | (uint32_t)field(d, 0));
    t.poff = (int64_t)(((uint64_t)(uint32_t)field(d, 3) << 32) | (uint32_t)field(d, 2));
    t.v0 = field(d, 4);
    t.v1 = field(d, 5);
    t.blk = field(d, 6);
    t.chan = field(d, 7);
    t.ty0 = field(d, 8);
    t.tx0 = field(d, 9);
    t.pitch = field(d, 10);
    t.ntap = field(d, 11);
    t.sub[0] = field(d, 12);
    t.sub[1] = field(d, 13);
    t.sub[2] = field(d, 14);
    t.slot = field(d, 15);
    t.wv[0] = field(d, 16);
    t.wv[1] = field(d, 17);
    t.wv[2] = field(d, 18);
    t.pad2 = 0;
    return t;
  };
  float2 pre[kPre];
  auto prefetch = [&](int d) {
    const int chan = field(d, 7), ty0 = field(d, 8), tx0 = field(d, 9), P = field(d, 10);
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
      const int e = tid + q * kThreads;
      pre[q] = e < P * P ? cell(chan, ty0, tx0, P, e) : make_float2(0.f, 0.f);
    }
  };
  int it = it0 + blockIdx.x;
  int d0 = 0, d1 = 0;
  if constexpr (MODE == 2) {
    d0 = desc(it);
    d1 = desc(it + G);
    if (it < it1) prefetch(d0);
  }
  for (; it < it1; it += G) {
    const Item item = MODE == 2 ? unpack(d0) : a.items[it];
    const int P = item.pitch;
    double* s_norm = reinterpret_cast<double*>(tile + P * P + 1);
    if constexpr (MODE == 2) {
#pragma unroll
      for (int q = 0; q < kPre; ++q) {
        const int e = tid + q * kThreads;
        if (e < P * P) tile[e] = pre[q];
      }
      for (int e = tid + kPre * kThreads; e < P * P; e += kThreads) tile[e] = cell(item.chan, item.ty0, item.tx0, P, e);
    } else {
      for (int e = tid; e < P * P; e += kThreads) tile[e] = cell(item.chan, item.ty0, item.tx0, P, e);
    }
    if (tid == 0) tile[P * P] = make_float2(0.f, 0.f);  // the zero cell
    // MODE 2: one accumulator per wave (P*P cells and 64 spare cells) behind
    // the tile, its zero cell and the norms
    const int acells = P * P + 64, a0 = P * P + 16;
    if (MODE == 2)
      for (int e = tid; e < kGatherWaves * acells; e += kThreads) tile[a0 + e] = make_float2(0.f, 0.f);
    __syncthreads();
    int d2 = 0;
    if constexpr (MODE == 2) {  // the next item's region and the descriptor after it
      d2 = desc(it + 2 * G);
      if (it + G < it1) prefetch(d1);
    }
    const uint32_t ab = lds_offset(tile) + (uint32_t)(a0 + w * acells) * 8u;
    // (selects, not indexing: a run-time index would move the item to scratch)
    const int wv0 = w == 0 ? item.v0 : w == 1 ? item.wv[0] : w == 2 ? item.wv[1] : item.wv[2];
    const int wv1 = w == kGatherWaves - 1 ? item.v1 : w == 0 ? item.wv[0] : w == 1 ? item.wv[1] : item.wv[2];
    int64_t wtap = item.tap0 + (w == 0 ? 0 : w == 1 ? item.sub[0] : w == 2 ? item.sub[1] : item.sub[2]);
    double rho2 = 0.0, res2 = 0.0;
    for (int r0 = wv0; r0 < wv1;) {
      const int k0 = meta_steps(a.meta[r0]);
      const int r1 = steps_run_end(a.meta, r0, wv1, k0, lane);
      switch (k0) {
#define PHI_G_CASE(K)                                                                                  \
  case K:                                                                                              \
    if constexpr (K <= NKM)                                                                            \
      wtap = gather_item<GP, MODE, K, Depth<GP, K, MODE == 2 ? kFusedRegs : PHI_GATHER_DEPTH_REGS>::value>( \
          a, item, r0, r1, wtap, vis, yv, rho2, res2, tile, ab);                                      \
    break;
        PHI_G_CASE(1)
        PHI_G_CASE(2)
        PHI_G_CASE(3)
        PHI_G_CASE(4)
        PHI_G_CASE(5)
        PHI_G_CASE(6)
        PHI_G_CASE(7)
#undef PHI_G_CASE
        default:
          break;
      }
      r0 = r1;
    }
    if (MODE >= 1) {
      rho2 = wave_sum_d(rho2);
      res2 = wave_sum_d(res2);
      if (lane == 0) {
        s_norm[2 * w] = rho2;
        s_norm[2 * w + 1] = res2;
      }
      __syncthreads();
      if (tid == 0) {
        double r0 = 0.0, r1 = 0.0;
        for (int k = 0; k < kGatherWaves; ++k) {
          r0 += s_norm[2 * k];
          r1 += s_norm[2 * k + 1];
        }
        item_norms[2 * (int64_t)item.slot] = r0;
        item_norms[2 * (int64_t)item.slot + 1] = r1;
      }
    }
    if (MODE == 2) {  // the item's partial: the waves' accumulators in a fixed order
      float2* __restrict__ out = a.partials + item.poff;
      for (int e = tid; e < P * P; e += 64 * kGatherWaves) {
        float2 s = tile[a0 + e];
        for (int q = 1; q < kGatherWaves; ++q) {
          const float2 t = tile[a0 + q * acells + e];
          s.x += t.x;
          s.y += t.y;
        }
        out[e] = s;
      }
    }
    __syncthreads();
    d0 = d1;
    d1 = d2;
  }
}

// ----------------------------------------------------------- G^H (scatter)
// One wave owns one pitch x pitch LDS accumulator (the item's tile plus the
// window halo) and adds conj(g) theta v for its visibilities in plan order.
// The taps of one window are distinct cells, so each read-add-write step has
// no two lanes on one address; no atomics are needed and the order is fixed.
// Lanes past the window add into 64 spare cells behind the accumulator (one
// per lane), so no step needs a divergent branch.  The G taps are prefetched
// exactly as in the gather.
template <int GP, int MODE, int NK, int D>
__device__ __forceinline__ int64_t scatter_item(const GArgs& a, const Item& item, int v0, int v1, int64_t tap0,
                                                float2* __restrict__ vis, float2* __restrict__ acc) {
  using R = typename GRaw<GP>::T;
  constexpr int C = chunk_len<D>();
  const int lane = threadIdx.x;
  const int vlast = v1 - 1, P = item.pitch;
  const uint32_t ab = lds_offset(acc);
  const uint32_t park = ab + (uint32_t)(P * P + lane) * 8u;  // this lane's spare cell
  const float th = a.theta[item.blk];
  float sc = 1.f;
  if (MODE == 1) sc = (float)((a.sigma ? a.sigma[item.blk] : 1.0) * a.scale[item.blk]);
  // theta * v for a chunk (dual form: v+ = sigma * scale * c, written back;
  // lanes past the chunk hold the next chunk's visibilities and leave them)
  auto take_av = [&](float2 v, int c0) -> float2 {
    if (MODE == 1) {
      v = make_float2(sc * v.x, sc * v.y);
      if (lane < C && c0 + lane < v1) vis[c0 + lane] = v;
    }
    return make_float2(th * v.x, th * v.y);
  };
  // chunks as in the gather: metadata of chunks cb, cb + C and (in flight)
  // cb + 2C; theta v of chunk cb (read per window) and raw v of cb + C, all
  // rotated between chunks only
  int cb = v0;
  uint32_t mcur = a.meta[min(cb + lane, vlast)];
  uint32_t mnxt = a.meta[min(cb + C + lane, vlast)];
  uint32_t mstg = a.meta[min(cb + 2 * C + lane, vlast)];
  float2 avc = take_av(vis[min(cb + lane, vlast)], cb);
  float2 vraw = vis[min(cb + C + lane, vlast)];
  R gb[D][NK];
  uint32_t ms[D];
  GStream<GP, NK, C> gs{static_cast<const char*>(a.G), uniform64(tap0), uniform64(tap0), v0, v1};
  TapLayout<NK> lay;
  auto step = [&](const R(&g)[NK], uint32_t mt, int rel) {
    const int by = mt & 8191, bx = (mt >> 13) & 8191, S = 2 * (int)(mt >> 26) + 1;
    if (S != lay.S) lay.set(S, P, lane);
    const float vx = readlane_f(avc.x, rel), vy = readlane_f(avc.y, rel);
    const uint32_t base_b = ab + (uint32_t)((by - item.ty0) * P + (bx - item.tx0)) * 8u;
    // all steps of one window touch distinct cells: read them all, then add
    // and write, so the window costs one LDS round trip, not one per step
    // (every window of a run has NK steps: S^2 > 64 (NK - 1))
    float2 cur[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) cur[k] = lds_load(lay.addr(base_b, k, park));
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const float gx = g_re<GP>(g[k]), gy = g_im<GP>(g[k]);
      cur[k].x = __builtin_fmaf(gx, vx, cur[k].x);
      cur[k].x = __builtin_fmaf(gy, vy, cur[k].x);
      cur[k].y = __builtin_fmaf(gx, vy, cur[k].y);
      cur[k].y = __builtin_fmaf(-gy, vx, cur[k].y);
      lds_store(lay.addr(base_b, k, park), cur[k]);
    }
  };
#pragma unroll
  for (int d = 0; d < D; ++d) gs.fetch(gb[d], ms[d], mcur, mnxt, cb, lane);
  for (;;) {
    const int n = min(C, v1 - cb);  // windows of this chunk
    const int full = n - n % D;     // in whole groups of D (slots 0..D-1)
    for (int rel = 0; rel < full; rel += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        step(gb[d], ms[d], rel + d);
        gs.fetch(gb[d], ms[d], mcur, mnxt, cb, lane);
      }
    }
    if (n < C) {  // last chunk: the rest (< D windows) is already fetched
#pragma unroll
      for (int d = 0; d < D - 1; ++d)
        if (full + d < n) step(gb[d], ms[d], full + d);
      break;
    }
    if (cb + C >= v1) break;
    cb += C;
    mcur = mnxt;
    mnxt = mstg;
    mstg = a.meta[min(cb + 2 * C + lane, vlast)];
    avc = take_av(vraw, cb);
    vraw = vis[min(cb + C + lane, vlast)];
  }
  return gs.tap;
}

template <int GP, int MODE, int NKM>
__global__ __launch_bounds__(64) void k_scatter(GArgs a, float2* __restrict__ vis, float2* __restrict__ partials,
                                                int it0, int it1) {
  extern __shared__ float2 acc[];  // pitch^2 cells, then 64 spare cells
  const int lane = threadIdx.x;
  for (int it = it0 + blockIdx.x; it < it1; it += gridDim.x) {
    const Item item = a.items[it];
    const int P = item.pitch, PP = P * P;
    for (int e = lane; e < PP; e += 64) acc[e] = make_float2(0.f, 0.f);
    __syncthreads();
    int64_t tap = item.tap0;
    for (int r0 = item.v0; r0 < item.v1;) {
      const int k0 = meta_steps(a.meta[r0]);
      const int r1 = steps_run_end(a.meta, r0, item.v1, k0, lane);
      switch (k0) {
#define PHI_S_CASE(K)                                                                                   \
  case K:                                                                                               \
    if constexpr (K <= NKM)                                                                             \
      tap = scatter_item<GP, MODE, K, Depth<GP, K, PHI_SCATTER_DEPTH_REGS>::value>(a, item, r0, r1, tap, vis, \
                                                                                   acc);              \
    break;
        PHI_S_CASE(1)
        PHI_S_CASE(2)
        PHI_S_CASE(3)
        PHI_S_CASE(4)
        PHI_S_CASE(5)
        PHI_S_CASE(6)
        PHI_S_CASE(7)
#undef PHI_S_CASE
        default:
          break;
      }
      r0 = r1;
    }
    __syncthreads();
    float2* out = partials + item.poff;
    for (int e = lane; e < PP; e += 64) out[e] = acc[e];
    __syncthreads();
  }
}

// ------------------------------------------- Kaiser-Bessel rows in-kernel
// G rows of direction-independent data are separable Kaiser-Bessel taps,
// g(i, j) = psi(f_y - i) psi(f_x - j) with f = kappa - b the position of the
// visibility relative to its window origin (f in [J/2 - 1, J/2)) and
// psi(d) = I0(beta sqrt(1 - (2d/J)^2)) / I0(beta).  The taps are evaluated
// here instead of being read from HBM.
//
// I0 (z >= 0) by the polynomial approximations of Abramowitz & Stegun
// (Handbook of Mathematical Functions, 9.8.1 for z <= 3.75 and 9.8.2
// above, |relative error| < 2e-7); both are evaluated and one is selected,
// so lanes do not diverge.
__device__ __forceinline__ float bessel_i0(float z) {
  const float t = z * (1.f / 3.75f), u = t * t;
  const float small =
      1.f + u * (3.5156229f + u * (3.0899424f + u * (1.2067492f + u * (0.2659732f + u * (0.0360768f + u * 0.0045813f)))));
  const float r = 3.75f / fmaxf(z, 3.75f);
  const float p = 0.39894228f +
                  r * (0.01328592f +
                       r * (0.00225319f +
                            r * (-0.00157565f +
                                 r * (0.00916281f +
                                      r * (-0.02057706f + r * (0.02635537f + r * (-0.01647633f + r * 0.00392377f)))))));
  const float large = p * __expf(fminf(z, 80.f)) * rsqrtf(fmaxf(z, 3.75f));
  return z <= 3.75f ? small : large;
}

// The J taps psi(f - i), i = 0..J-1, of one axis.
template <int J>
__device__ __forceinline__ void kb_axis(float f, float beta, float inv_i0b, float (&w)[J]) {
#pragma unroll
  for (int i = 0; i < J; ++i) {
    const float d = (f - (float)i) * (2.f / (float)J);
    const float t = fmaxf(1.f - d * d, 0.f);
    w[i] = bessel_i0(beta * sqrtf(t)) * inv_i0b;
  }
}

// Gather, one lane per visibility: each lane evaluates its 2J taps once and
// sums its J x J window from the LDS copy of the item's grid region as
// sum_i psi_y(i) sum_j psi_x(j) X(i, j).  kGatherWaves waves per work-group
// share the tile and take 64-visibility chunks of the item in turn.
template <int MODE, int J>
__global__ __launch_bounds__(64 * kGatherWaves) void k_gather_kb(GArgs a, float2* __restrict__ vis,
                                                                 const float2* __restrict__ yv,
                                                                 double* __restrict__ item_norms, int it0, int it1) {
  extern __shared__ float2 tile[];  // P*P cells, a zero cell, then the wave norms
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  for (int it = it0 + blockIdx.x; it < it1; it += gridDim.x) {
    const Item item = a.items[it];
    const int P = item.pitch;
    double* s_norm = reinterpret_cast<double*>(tile + P * P + 1);
    const float2* __restrict__ grid = a.grid + (size_t)item.chan * a.Ky * a.Kx;
    for (int e = tid; e < P * P; e += 64 * kGatherWaves) {
      const int r = e / P, c = e - (e / P) * P;
      int gr = item.ty0 + r, gc = item.tx0 + c;
      gr -= (gr >= a.Ky) ? a.Ky : 0;
      gc -= (gc >= a.Kx) ? a.Kx : 0;
      tile[e] = grid[(size_t)gr * a.Kx + gc];
    }
    __syncthreads();
    const float th = a.theta[item.blk];
    float inv_sig = 1.f;
    if (MODE == 1 && a.sigma) inv_sig = (float)(1.0 / a.sigma[item.blk]);
    double rho2 = 0.0, res2 = 0.0;
    for (int c0 = item.v0 + 64 * w; c0 < item.v1; c0 += 64 * kGatherWaves) {
      const bool live = c0 + lane < item.v1;
      const int v = live ? c0 + lane : item.v1 - 1;
      const uint32_t m = a.meta[v];
      const float2 fr = a.frac[v];
      float2 vv = make_float2(0.f, 0.f), yy = vv;
      if (MODE == 1) {
        vv = vis[v];
        yy = yv[v];
      }
      float py[J], px[J];
      kb_axis<J>(fr.x, a.kb_beta, a.kb_inv_i0b, py);
      kb_axis<J>(fr.y, a.kb_beta, a.kb_inv_i0b, px);
      const char* t0 = reinterpret_cast<const char*>(tile) +
                       (size_t)(((int)(m & 8191) - item.ty0) * P + ((int)((m >> 13) & 8191) - item.tx0)) * 8;
      float ax = 0.f, ay = 0.f;
#pragma unroll
      for (int i = 0; i < J; ++i) {
        const float2* row = reinterpret_cast<const float2*>(t0 + (size_t)i * P * 8);
        float rx = 0.f, ry = 0.f;
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const float2 X = row[j];
          rx = __builtin_fmaf(px[j], X.x, rx);
          ry = __builtin_fmaf(px[j], X.y, ry);
        }
        ax = __builtin_fmaf(py[i], rx, ax);
        ay = __builtin_fmaf(py[i], ry, ay);
      }
      if (live) {
        const float sx = th * ax, sy = th * ay;
        if (MODE == 0) {
          vis[v] = make_float2(sx, sy);
        } else {
          const float2 cc = make_float2(vv.x * inv_sig + sx - yy.x, vv.y * inv_sig + sy - yy.y);
          vis[v] = cc;
          const double rx = (double)sx - (double)yy.x, ry = (double)sy - (double)yy.y;
          rho2 += (double)cc.x * (double)cc.x + (double)cc.y * (double)cc.y;
          res2 += rx * rx + ry * ry;
        }
      }
    }
    if (MODE == 1) {
      rho2 = wave_sum_d(rho2);
      res2 = wave_sum_d(res2);
      if (lane == 0) {
        s_norm[2 * w] = rho2;
        s_norm[2 * w + 1] = res2;
      }
      __syncthreads();
      if (tid == 0) {
        double r0 = 0.0, r1 = 0.0;
        for (int k = 0; k < kGatherWaves; ++k) {
          r0 += s_norm[2 * k];
          r1 += s_norm[2 * k + 1];
        }
        item_norms[2 * (int64_t)it] = r0;
        item_norms[2 * (int64_t)it + 1] = r1;
      }
    }
    __syncthreads();
  }
}

// Adds conj(g) a of a chunk's n visibilities (a = theta v for the scatter, c
// for the one pass), in order, into a wave's LDS
// accumulator (byte base accb): for each visibility the lanes span its J x J
// window (tap t = q 64 + lane at byte offset off[q] from the window origin,
// weights from the table psi; lanes past the window use their spare cell)
// and read-add-write distinct cells.  (Taking two windows whose squares do
// not overlap together, with one LDS round trip, measured slower: the
// per-step overlap test costs more than the round trip it saves.)
template <int J, int NKJ>
__device__ __forceinline__ void kb_accumulate(char* accb, const float (*psi)[2 * J], int n, float avx, float avy,
                                              uint32_t base_b, const uint32_t (&off)[NKJ], const int (&ti)[NKJ],
                                              const int (&tj)[NKJ], const bool (&on)[NKJ], uint32_t spare) {
  for (int k = 0; k < n; ++k) {
    const float vx = readlane_f(avx, k), vy = readlane_f(avy, k);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)base_b, k);
    float2 cur[NKJ];
    uint32_t ad[NKJ];
    float g[NKJ];
#pragma unroll
    for (int q = 0; q < NKJ; ++q) {
      g[q] = psi[k][ti[q]] * psi[k][J + tj[q]];
      ad[q] = on[q] ? b + off[q] : spare;
      cur[q] = *reinterpret_cast<float2*>(accb + ad[q]);
    }
#pragma unroll
    for (int q = 0; q < NKJ; ++q) {
      cur[q].x = __builtin_fmaf(g[q], vx, cur[q].x);
      cur[q].y = __builtin_fmaf(g[q], vy, cur[q].y);
      *reinterpret_cast<float2*>(accb + ad[q]) = cur[q];
    }
  }
}

// Adjoint: one wave per item owns its LDS accumulator as in k_scatter.  Per
// 64-visibility chunk, lane l evaluates visibility l's 2J taps into an LDS
// table; then for each visibility in order the lanes span its J x J window
// (lane t on tap (t / J, t mod J), a second step for J > 8) and read-add-write
// distinct cells, with g = psi_y(i) psi_x(j) read from the table.
template <int MODE, int J>
__global__ __launch_bounds__(64) void k_scatter_kb(GArgs a, float2* __restrict__ vis, float2* __restrict__ partials,
                                                   int it0, int it1) {
  constexpr int NKJ = (J * J + 63) / 64;
  extern __shared__ float2 acc[];  // pitch^2 cells, then 64 spare cells
  __shared__ float psi[64][2 * J];
  const int lane = threadIdx.x;
  for (int it = it0 + blockIdx.x; it < it1; it += gridDim.x) {
    const Item item = a.items[it];
    const int P = item.pitch, PP = P * P;
    for (int e = lane; e < PP; e += 64) acc[e] = make_float2(0.f, 0.f);
    const float th = a.theta[item.blk];
    float sc = 1.f;
    if (MODE == 1) sc = (float)((a.sigma ? a.sigma[item.blk] : 1.0) * a.scale[item.blk]);
    // this lane's taps (t / J, t mod J) per step, as LDS byte offsets from the
    // window origin; lanes past the window use their spare cell
    uint32_t off[NKJ];
    int ti[NKJ], tj[NKJ];
    bool on[NKJ];
#pragma unroll
    for (int k = 0; k < NKJ; ++k) {
      const int t = k * 64 + lane;
      on[k] = t < J * J;
      ti[k] = on[k] ? t / J : 0;
      tj[k] = on[k] ? t - (t / J) * J : 0;
      off[k] = (uint32_t)(ti[k] * P + tj[k]) * 8u;
    }
    const uint32_t spare = (uint32_t)(PP + lane) * 8u;
    char* accb = reinterpret_cast<char*>(acc);
    for (int c0 = item.v0; c0 < item.v1; c0 += 64) {
      const int n = min(64, item.v1 - c0);
      const bool live = lane < n;
      const int v = live ? c0 + lane : c0 + n - 1;
      const uint32_t m = a.meta[v];
      const float2 fr = a.frac[v];
      float2 vv = vis[v];
      if (MODE == 1) {
        vv = make_float2(sc * vv.x, sc * vv.y);
        if (live) vis[v] = vv;
      }
      const float avx = th * vv.x, avy = th * vv.y;
      const uint32_t base_b =
          (uint32_t)(((int)(m & 8191) - item.ty0) * P + ((int)((m >> 13) & 8191) - item.tx0)) * 8u;
      float py[J], px[J];
      kb_axis<J>(fr.x, a.kb_beta, a.kb_inv_i0b, py);
      kb_axis<J>(fr.y, a.kb_beta, a.kb_inv_i0b, px);
      __syncthreads();  // previous chunk's table reads are done
#pragma unroll
      for (int i = 0; i < J; ++i) {
        psi[lane][i] = py[i];
        psi[lane][J + i] = px[i];
      }
      __syncthreads();
      kb_accumulate<J, NKJ>(accb, psi, n, avx, avy, base_b, off, ti, tj, on, spare);
    }
    __syncthreads();
    float2* out = partials + item.poff;
    for (int e = lane; e < PP; e += 64) out[e] = acc[e];
    __syncthreads();
  }
}

// One-pass dual step of the Kaiser-Bessel mode (PHI_G_KB with
// PHI_FUSED_GH): one wave per item, with the item's grid tile and its
// accumulator in LDS.  Per 64-visibility chunk each lane evaluates its
// visibility's 2J taps once, forms c = v / sigma + theta Phi x - y from the
// tile (k_gather_kb's sum), writes c and its FP64 norm terms; then the taps
// go to an LDS table and the wave adds conj(g) c of each visibility, in
// order, into the accumulator (k_scatter_kb's read-add-write of distinct
// cells).  The partial holds G^H c; sigma_b * scale_b comes in v+ (k_vscale)
// and, times theta_b, in the merge, as for stored G.
template <int J>
__global__ __launch_bounds__(64) void k_dual_kb(GArgs a, float2* __restrict__ vis, const float2* __restrict__ yv,
                                                double* __restrict__ item_norms, int it0, int it1) {
  constexpr int NKJ = (J * J + 63) / 64;
  extern __shared__ float2 lds[];  // tile (P*P cells), then the accumulator (P*P + 64 cells)
  __shared__ float psi[64][2 * J];
  const int lane = threadIdx.x;
  for (int it = it0 + blockIdx.x; it < it1; it += gridDim.x) {
    const Item item = a.items[it];
    const int P = item.pitch, PP = P * P;
    float2* tile = lds;
    float2* acc = lds + PP;
    char* accb = reinterpret_cast<char*>(acc);
    const float2* __restrict__ grid = a.grid + (size_t)item.chan * a.Ky * a.Kx;
    for (int e = lane; e < PP; e += 64) {
      const int r = e / P, c = e - (e / P) * P;
      int gr = item.ty0 + r, gc = item.tx0 + c;
      gr -= (gr >= a.Ky) ? a.Ky : 0;
      gc -= (gc >= a.Kx) ? a.Kx : 0;
      tile[e] = grid[(size_t)gr * a.Kx + gc];
    }
    for (int e = lane; e < PP + 64; e += 64) acc[e] = make_float2(0.f, 0.f);
    const float th = a.theta[item.blk];
    const float inv_sig = a.sigma ? (float)(1.0 / a.sigma[item.blk]) : 1.f;
    // this lane's taps (t / J, t mod J) per step, as accumulator byte offsets
    // from the window origin; lanes past the window use their spare cell
    uint32_t off[NKJ];
    int ti[NKJ], tj[NKJ];
    bool on[NKJ];
#pragma unroll
    for (int k = 0; k < NKJ; ++k) {
      const int t = k * 64 + lane;
      on[k] = t < J * J;
      ti[k] = on[k] ? t / J : 0;
      tj[k] = on[k] ? t - (t / J) * J : 0;
      off[k] = (uint32_t)(ti[k] * P + tj[k]) * 8u;
    }
    const uint32_t spare = (uint32_t)(PP + lane) * 8u;
    double rho2 = 0.0, res2 = 0.0;
    __syncthreads();
    for (int c0 = item.v0; c0 < item.v1; c0 += 64) {
      const int n = min(64, item.v1 - c0);
      const bool live = lane < n;
      const int v = live ? c0 + lane : c0 + n - 1;
      const uint32_t m = a.meta[v];
      const float2 fr = a.frac[v];
      const float2 vv = vis[v], yy = yv[v];
      float py[J], px[J];
      kb_axis<J>(fr.x, a.kb_beta, a.kb_inv_i0b, py);
      kb_axis<J>(fr.y, a.kb_beta, a.kb_inv_i0b, px);
      const uint32_t base_b =
          (uint32_t)(((int)(m & 8191) - item.ty0) * P + ((int)((m >> 13) & 8191) - item.tx0)) * 8u;
      const char* t0 = reinterpret_cast<const char*>(tile) + base_b;
      float ax = 0.f, ay = 0.f;
#pragma unroll
      for (int i = 0; i < J; ++i) {
        const float2* row = reinterpret_cast<const float2*>(t0 + (size_t)i * P * 8);
        float rx = 0.f, ry = 0.f;
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const float2 X = row[j];
          rx = __builtin_fmaf(px[j], X.x, rx);
          ry = __builtin_fmaf(px[j], X.y, ry);
        }
        ax = __builtin_fmaf(py[i], rx, ax);
        ay = __builtin_fmaf(py[i], ry, ay);
      }
      const float sx = th * ax, sy = th * ay;
      const float2 cc = make_float2(vv.x * inv_sig + sx - yy.x, vv.y * inv_sig + sy - yy.y);
      if (live) {
        vis[v] = cc;
        const double rx = (double)sx - (double)yy.x, ry = (double)sy - (double)yy.y;
        rho2 += (double)cc.x * (double)cc.x + (double)cc.y * (double)cc.y;
        res2 += rx * rx + ry * ry;
      }
      const float avx = cc.x, avy = cc.y;  // theta joins sigma * scale in the merge
      __syncthreads();  // the previous chunk's table reads are done
#pragma unroll
      for (int i = 0; i < J; ++i) {
        psi[lane][i] = py[i];
        psi[lane][J + i] = px[i];
      }
      __syncthreads();
      kb_accumulate<J, NKJ>(accb, psi, n, avx, avy, base_b, off, ti, tj, on, spare);
    }
    rho2 = wave_sum_d(rho2);
    res2 = wave_sum_d(res2);
    if (lane == 0) {
      item_norms[2 * (int64_t)item.slot] = rho2;
      item_norms[2 * (int64_t)item.slot + 1] = res2;
    }
    __syncthreads();
    float2* out = a.partials + item.poff;
    for (int e = lane; e < PP; e += 64) out[e] = acc[e];
    __syncthreads();
  }
}

// One work-group per (channel, region): a region is rk x rk tiles of edge T
// (rk = 1, 2 or 4), and cell (r, c) of it is the fixed-order sum of the tile
// partials covering it: those of the tiles up to `halo` tiles above / left
// of the region and of its own tiles (with wrap), source tile by source
// tile, items in tile order.  A 2 x 2 region reads each of its own tiles'
// partials once, where four single-tile work-groups would each read the part
// that covers them.  The partial list is staged in LDS once per region;
// reads of a partial row are coalesced.
constexpr int kMergeList = 256;
constexpr int kMergeSrc = 25;  // (rk + halo)^2 source tiles at most
// Factor of an item's partial in the merge: sigma_b * scale_b * theta_b after
// the one-pass dual step (its partials hold G^H c), else 1 (exact:
// fma(1, v, s) = s + v).
__device__ __forceinline__ float merge_factor(const double* sigma, const double* scale, const float* theta,
                                              int blk) {
  return scale ? (float)((sigma ? sigma[blk] : 1.0) * scale[blk] * (double)theta[blk]) : 1.f;
}

__global__ __launch_bounds__(256) void k_merge(float2* __restrict__ grid, const float2* __restrict__ partials,
                                               const int32_t* __restrict__ tile_ptr,
                                               const TileEntry* __restrict__ ent, const int32_t* __restrict__ live,
                                               int live0, int Ky, int Kx, int T, int halo, int rk, int l0,
                                               const double* __restrict__ sigma, const double* __restrict__ scale,
                                               const float* __restrict__ theta) {
  __shared__ int64_t s_off[kMergeList];
  __shared__ int32_t s_pitch[kMergeList];
  __shared__ float s_fac[kMergeList];
  __shared__ int32_t s_oy[kMergeList], s_ox[kMergeList];
  __shared__ int s_beg[kMergeSrc], s_pre[kMergeSrc + 1];
  const int nty = Ky / T, ntx = Kx / T, R = rk * T, nry = Ky / R, nrx = Kx / R;
  int l = l0 + blockIdx.y, reg = blockIdx.x;
  if (live) {
    const int t = live[live0 + blockIdx.x];
    l = t / (nry * nrx);
    reg = t % (nry * nrx);
  }
  const int ry = reg / nrx, rx = reg % nrx;
  const int sw = rk + halo, nsrc = sw * sw;   // source tile offsets dy, dx in [-halo, rk)
  // source tile j (dy = j / sw - halo, dx = j % sw - halo) of the region
  auto src_tile = [&](int j) {
    int sty = ry * rk + j / sw - halo, stx = rx * rk + j % sw - halo;
    sty += sty < 0 ? nty : 0;
    stx += stx < 0 ? ntx : 0;
    sty -= sty >= nty ? nty : 0;
    stx -= stx >= ntx ? ntx : 0;
    return ((int64_t)l * nty + sty) * ntx + stx;
  };
  if ((int)threadIdx.x < nsrc) {
    const int64_t tile = src_tile(threadIdx.x);
    s_beg[threadIdx.x] = tile_ptr[tile];
    s_pre[threadIdx.x + 1] = tile_ptr[tile + 1] - tile_ptr[tile];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s_pre[0] = 0;
    for (int j = 0; j < nsrc; ++j) s_pre[j + 1] += s_pre[j];
  }
  __syncthreads();
  const int n = s_pre[nsrc];
  for (int e = threadIdx.x; e < n && e < kMergeList; e += 256) {
    int j = 0;
    while (e >= s_pre[j + 1]) ++j;
    const TileEntry te = ent[s_beg[j] + (e - s_pre[j])];
    s_off[e] = te.poff;
    s_pitch[e] = te.pitch;
    s_fac[e] = merge_factor(sigma, scale, theta, te.blk);
    s_oy[e] = (halo - j / sw) * T;  // partial row of region row r: r + s_oy
    s_ox[e] = (halo - j % sw) * T;
  }
  __syncthreads();
  float2* out = grid + (int64_t)l * Ky * Kx;
  // cell (r, c) of the region from the global lists (lists beyond kMergeList)
  auto cell_from_lists = [&](int r, int c, float& sx, float& sy) {
    for (int j = 0; j < nsrc; ++j) {
      const int64_t tile = src_tile(j);
      const int ly = r + (halo - j / sw) * T, lx = c + (halo - j % sw) * T;
      for (int k = tile_ptr[tile]; k < tile_ptr[tile + 1]; ++k) {
        const TileEntry te = ent[k];
        if ((unsigned)ly < (unsigned)te.pitch && (unsigned)lx < (unsigned)te.pitch) {
          const float2 v = partials[te.poff + (int64_t)ly * te.pitch + lx];
          const float f = merge_factor(sigma, scale, theta, te.blk);
          sx = __builtin_fmaf(f, v.x, sx);
          sy = __builtin_fmaf(f, v.y, sy);
        }
      }
    }
  };
  if (R >= 32) {
    // Regions of 32 or 64 cells: each wave takes 16 x 16 sub-squares, lane
    // (lr, lc) the cells (r0 + 4q + lr, c0 + lc), q < 4, and passes over the
    // entries whose partial misses the sub-square (a wave-uniform test): of
    // the (rk + halo)^2 source tiles only those next to the sub-square reach
    // it.  A skipped entry would have added exactly zero, so every cell's sum
    // keeps its terms and their order.
    const int lane = threadIdx.x & 63, lr = lane >> 4, lc = lane & 15, nsq = R / 16;
    for (int sq = (int)(threadIdx.x >> 6); sq < nsq * nsq; sq += 4) {
      const int r0 = (sq / nsq) * 16, c0 = (sq % nsq) * 16, c = c0 + lc;
      float sx[4] = {0.f, 0.f, 0.f, 0.f}, sy[4] = {0.f, 0.f, 0.f, 0.f};
      if (n <= kMergeList) {
        for (int k = 0; k < n; ++k) {
          const int oy = s_oy[k], ox = s_ox[k], P = s_pitch[k];
          if (r0 + oy >= P || r0 + 15 + oy < 0 || c0 + ox >= P || c0 + 15 + ox < 0) continue;
          const float fk = s_fac[k];
          const int64_t off = s_off[k];
          const int lx = c + ox;
          const bool inx = (unsigned)lx < (unsigned)P;
          float2 v[4];
          float f[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {  // loads first; a cell the partial misses reads its first cell, weight 0
            const int ly = r0 + 4 * q + lr + oy;
            const bool in = inx && (unsigned)ly < (unsigned)P;
            f[q] = in ? fk : 0.f;
            v[q] = partials[off + (in ? (int64_t)ly * P + lx : 0)];
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            sx[q] = __builtin_fmaf(f[q], v[q].x, sx[q]);
            sy[q] = __builtin_fmaf(f[q], v[q].y, sy[q]);
          }
        }
      } else {
        for (int q = 0; q < 4; ++q) cell_from_lists(r0 + 4 * q + lr, c, sx[q], sy[q]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        out[(int64_t)(ry * R + r0 + 4 * q + lr) * Kx + rx * R + c] = make_float2(sx[q], sy[q]);
    }
    return;
  }
  for (int e = threadIdx.x; e < R * R; e += 256) {
    const int r = e / R, c = e % R;
    float sx = 0.f, sy = 0.f;
    if (n <= kMergeList) {
      // four entries at a time, loads first: an entry that does not cover
      // this cell reads its partial's first cell and adds it with weight 0
      // (the sum keeps its order; partial cells are finite)
      int k = 0;
      for (; k + 4 <= n; k += 4) {
        float2 v[4];
        float f[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ly = r + s_oy[k + u], lx = c + s_ox[k + u], P = s_pitch[k + u];
          const bool in = (unsigned)ly < (unsigned)P && (unsigned)lx < (unsigned)P;
          f[u] = in ? s_fac[k + u] : 0.f;
          v[u] = partials[s_off[k + u] + (in ? (int64_t)ly * P + lx : 0)];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          sx = __builtin_fmaf(f[u], v[u].x, sx);
          sy = __builtin_fmaf(f[u], v[u].y, sy);
        }
      }
      for (; k < n; ++k) {
        const int ly = r + s_oy[k], lx = c + s_ox[k], P = s_pitch[k];
        if ((unsigned)ly < (unsigned)P && (unsigned)lx < (unsigned)P) {
          const float2 v = partials[s_off[k] + (int64_t)ly * P + lx];
          sx = __builtin_fmaf(s_fac[k], v.x, sx);
          sy = __builtin_fmaf(s_fac[k], v.y, sy);
        }
      }
    } else {  // long lists: same order, read from global memory
      cell_from_lists(r, c, sx, sy);
    }
    out[(int64_t)(ry * R + r) * Kx + rx * R + c] = make_float2(sx, sy);
  }
}

// Per-block FP64 norms from the item partials, in two fixed-order levels:
// kFinChunks work-groups per block sum fixed chunks of its items, then one
// wave per block sums the chunk partials and forms the projection scale:
// 0 inside the ball, 1 - eps/rho outside.
__global__ __launch_bounds__(256) void k_block_sums(const double* __restrict__ item_norms,
                                                    const BlockInfo* __restrict__ blocks, double* __restrict__ part,
                                                    int b0) {
  __shared__ double red[2][4];
  const int b = b0 + blockIdx.y, c = blockIdx.x, tid = threadIdx.x;
  const BlockInfo bi = blocks[b];
  const int n = bi.item1 - bi.item0, per = (n + kFinChunks - 1) / kFinChunks;
  const int i0 = bi.item0 + c * per, i1 = min(i0 + per, bi.item1);
  double s0 = 0.0, s1 = 0.0;
  for (int it = i0 + tid; it < i1; it += 256) {
    s0 += item_norms[2 * (int64_t)it];
    s1 += item_norms[2 * (int64_t)it + 1];
  }
  s0 = wave_sum_d(s0);
  s1 = wave_sum_d(s1);
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = s0;
    red[1][tid >> 6] = s1;
  }
  __syncthreads();
  if (tid < 2)
    part[((int64_t)b * kFinChunks + c) * 2 + tid] = (red[tid][0] + red[tid][1]) + (red[tid][2] + red[tid][3]);
}

__global__ __launch_bounds__(64) void k_finalize(const double* __restrict__ part, const double* __restrict__ eps,
                                                 double* __restrict__ rho, double* __restrict__ res,
                                                 double* __restrict__ scale, int* __restrict__ flag, int b0) {
  const int b = b0 + blockIdx.x, lane = threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (int c = lane; c < kFinChunks; c += 64) {
    s0 += part[((int64_t)b * kFinChunks + c) * 2];
    s1 += part[((int64_t)b * kFinChunks + c) * 2 + 1];
  }
  s0 = wave_sum_d(s0);
  s1 = wave_sum_d(s1);
  if (lane == 0) {
    const double rh = sqrt(s0), rs = sqrt(s1), ep = eps[b];
    double sc = (rh > ep) ? 1.0 - ep / rh : 0.0;
    if (!isfinite(rh) || !isfinite(rs) || !isfinite(ep)) {
      sc = 0.0;
      flag[0] = 1;
    }
    if (rho) rho[b] = rh;
    if (res) res[b] = rs;
    scale[b] = sc;
  }
}

__global__ __launch_bounds__(256) void k_permute(const float2* __restrict__ src, float2* __restrict__ dst,
                                                 const int32_t* __restrict__ perm, int64_t n, int to_plan) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (to_plan)
    dst[i] = src[perm[i]];
  else
    dst[perm[i]] = src[i];
}

// ---------------------------------------------------- analysis helpers
// delta image per channel: 1 at the phase centre (Ny/2, Nx/2), 0 elsewhere
__global__ __launch_bounds__(256) void k_delta(float* __restrict__ x, int Ny, int Nx) {
  const int64_t n = (int64_t)Ny * Nx;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  x[(int64_t)blockIdx.y * n + i] = (i == (int64_t)(Ny / 2) * Nx + Nx / 2) ? 1.f : 0.f;
}

// v <- y - v (complex)
__global__ __launch_bounds__(256) void k_vis_residual(float2* __restrict__ v, const float2* __restrict__ y,
                                                      int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float2 a = v[i], b = y[i];
  v[i] = make_float2(b.x - a.x, b.y - a.y);
}

// FP64 sum of squares of each channel image: work-group (c, l) sums the c-th
// of kNormChunks contiguous slices of channel l in a fixed order
__global__ __launch_bounds__(256) void k_chan_sumsq(const float* __restrict__ x, int64_t n,
                                                    double* __restrict__ part) {
  __shared__ double red[4];
  const int c = blockIdx.x, l = blockIdx.y, tid = threadIdx.x;
  const int64_t per = (n + kNormChunks - 1) / kNormChunks;
  const int64_t a = (int64_t)c * per, b = a + per < n ? a + per : n;
  const float* __restrict__ xl = x + (int64_t)l * n;
  double s = 0.0;
  for (int64_t i = a + tid; i < b; i += 256) {
    const double v = (double)xl[i];
    s += v * v;
  }
  s = wave_sum_d(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) part[(int64_t)l * kNormChunks + c] = (red[0] + red[1]) + (red[2] + red[3]);
}

// norm_l = sqrt(sum of the channel's partials), inv_l = 1 / norm_l (0 if the
// image is zero)
__global__ __launch_bounds__(64) void k_chan_norm(const double* __restrict__ part, double* __restrict__ norm,
                                                  double* __restrict__ inv) {
  const int l = blockIdx.x, lane = threadIdx.x;
  double s = 0.0;
  for (int c = lane; c < kNormChunks; c += 64) s += part[(int64_t)l * kNormChunks + c];
  s = wave_sum_d(s);
  if (lane == 0) {
    const double nv = sqrt(s);
    if (norm) norm[l] = nv;
    if (inv) inv[l] = nv > 0.0 ? 1.0 / nv : 0.0;
  }
}

// x_l <- f_l x_l
__global__ __launch_bounds__(256) void k_chan_scale(float* __restrict__ x, const double* __restrict__ f,
                                                    int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int l = blockIdx.y;
  x[(int64_t)l * n + i] *= (float)f[l];
}

// peak_l = psf_l at the phase centre
__global__ __launch_bounds__(64) void k_centre_value(const float* __restrict__ x, int L, int Ny, int Nx,
                                                     double* __restrict__ peak) {
  const int l = blockIdx.x * 64 + threadIdx.x;
  if (l < L) peak[l] = (double)x[(int64_t)l * Ny * Nx + (int64_t)(Ny / 2) * Nx + Nx / 2];
}

// ------------------------------------------------------------ PDFB loop
// Primal step of the regularizer-free iteration: x+ = P_+(x - tau_l g) with
// NaN kept (a NaN is neither < 0 nor clipped), x~ = 2 x+ - x, and FP64
// partial sums of ||x+ - x||^2 and ||x+||^2 per (channel, chunk).
__global__ __launch_bounds__(256) void k_pdfb_primal(float* __restrict__ x, float* __restrict__ xt,
                                                     const float* __restrict__ g, const double* __restrict__ tau,
                                                     int64_t n, double* __restrict__ part) {
  __shared__ double red[2][4];
  const int c = blockIdx.x, l = blockIdx.y, tid = threadIdx.x;
  const int64_t per = (n + kNormChunks - 1) / kNormChunks;
  const int64_t a = (int64_t)c * per, b = a + per < n ? a + per : n;
  const int64_t off = (int64_t)l * n;
  const float t = (float)tau[l];
  double d2 = 0.0, n2 = 0.0;
  for (int64_t i = off + a + tid; i < off + b; i += 256) {
    const float xo = x[i];
    const float u = xo - t * g[i];
    const float xn = u < 0.f ? 0.f : u;
    x[i] = xn;
    xt[i] = 2.f * xn - xo;
    const double dd = (double)xn - (double)xo;
    d2 += dd * dd;
    n2 += (double)xn * (double)xn;
  }
  d2 = wave_sum_d(d2);
  n2 = wave_sum_d(n2);
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = d2;
    red[1][tid >> 6] = n2;
  }
  __syncthreads();
  if (tid < 2) part[((int64_t)l * kNormChunks + c) * 2 + tid] = (red[tid][0] + red[tid][1]) + (red[tid][2] + red[tid][3]);
}

// var_l = fixed-order sums of the channel's chunk partials
__global__ __launch_bounds__(64) void k_pdfb_var(const double* __restrict__ part, double* __restrict__ var) {
  const int l = blockIdx.x, lane = threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (int c = lane; c < kNormChunks; c += 64) {
    s0 += part[((int64_t)l * kNormChunks + c) * 2];
    s1 += part[((int64_t)l * kNormChunks + c) * 2 + 1];
  }
  s0 = wave_sum_d(s0);
  s1 = wave_sum_d(s1);
  if (lane == 0) {
    var[2 * l] = s0;
    var[2 * l + 1] = s1;
  }
}

// Adaptive l2 bound of one block per lane (rule stated with phi_eps_rule).
__global__ __launch_bounds__(64) void k_eps_update(const double* __restrict__ res, const double* __restrict__ var,
                                                   const BlockInfo* __restrict__ blocks, int nblk, EpsRule rule,
                                                   double* __restrict__ eps, int32_t* __restrict__ state) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= nblk) return;
  int since = state[3 * b], fixed = state[3 * b + 1], count = state[3 * b + 2];
  if (fixed) return;
  since += 1;
  const double r = res[b], e = eps[b];
  if (rule.freeze && r <= rule.hi * e) {
    fixed = 1;
  } else {
    const int l = blocks[b].chan;
    const double d2 = var[2 * l], n2 = var[2 * l + 1];
    const bool settled = n2 > 0.0 && d2 < rule.var_tol * rule.var_tol * n2;
    const bool outside = r < rule.lo * e || r > rule.hi * e;
    if (settled && outside && since >= rule.min_gap) {
      eps[b] = rule.mix * r + (1.0 - rule.mix) * e;
      since = 0;
      count += 1;
    }
  }
  state[3 * b] = since;
  state[3 * b + 1] = fixed;
  state[3 * b + 2] = count;
}

// ------------------------------------------------------------- G builder
// Rows of G from per-visibility tables, in FP64 (definitions with
// phi_plan_build_g): Kaiser-Bessel taps per axis convolved with the
// normalised w-chirp, their outer product, then the antenna pair's DDE
// kernel d_i (*) conj(flip(d_j)).  One wave per work item walks its windows
// in plan order (tap offsets from the window sizes); the per-window tables
// live in LDS.  Each tap is rounded once to the stored precision.

// I0 by its power series sum_k ((z/2)^2)^k / (k!)^2 (z <= 30 here: 60 terms
// leave a tail far below FP64 rounding).
__device__ __forceinline__ double bessel_i0_series(double z) {
  const double q = 0.25 * z * z;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k <= 60; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
  }
  return sum;
}

// d rounded to `sig` significant bits (ties to even), with spacing at least
// 2^qmin (subnormals of the target); exact in FP64.
__device__ __forceinline__ double round_sig(double d, int sig, int qmin) {
  if (!(fabs(d) > 0.0) || !isfinite(d)) return d;
  int e;
  (void)frexp(d, &e);
  const int q = max(e - sig, qmin);
  return ldexp(rint(ldexp(d, -q)), q);
}

__device__ __forceinline__ void store_tap(void* G, int gprec, int64_t t, double re, double im) {
  if (gprec == 0) {
    reinterpret_cast<float2*>(G)[t] = make_float2((float)re, (float)im);
  } else if (gprec == 1) {
    // one rounding FP64 -> FP16 (11 significant bits, subnormal spacing 2^-24);
    // the rounded value converts exactly
    const _Float16 hr = (_Float16)(float)round_sig(re, 11, -24);
    const _Float16 hi = (_Float16)(float)round_sig(im, 11, -24);
    reinterpret_cast<uint32_t*>(G)[t] =
        (uint32_t)__builtin_bit_cast(uint16_t, hr) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
  } else {
    // one rounding FP64 -> BF16 (8 significant bits, subnormal spacing 2^-133)
    const uint32_t br = __float_as_uint((float)round_sig(re, 8, -133)) >> 16;
    const uint32_t bi = __float_as_uint((float)round_sig(im, 8, -133)) >> 16;
    reinterpret_cast<uint32_t*>(G)[t] = br | (bi << 16);
  }
}

constexpr int kBuildMaxU = 32;   // J + 2h <= 21 + margin
constexpr int kBuildMaxSd = 13;  // 2 sa - 1 for sa <= 7

__global__ __launch_bounds__(64) void k_build_g(BuildArgs a, int it0) {
  __shared__ double psi[2][16];
  __shared__ double2 cw[kBuildMaxU];
  __shared__ double2 u[2][kBuildMaxU];
  __shared__ double2 pk[kBuildMaxSd * kBuildMaxSd];
  const int lane = threadIdx.x;
  const Item item = a.items[it0 + blockIdx.x];
  const int J = a.J;
  int64_t tap = item.tap0;
  for (int v = item.v0; v < item.v1; ++v) {
    const uint32_t m = a.meta[v];
    const int Sd = 2 * (int)(m >> 26) + 1, byd = m & 8191, bxd = (m >> 13) & 8191;
    const int64_t uu = (int64_t)a.perm[v] - a.u0;
    const double ky = a.kappa[2 * uu], kx = a.kappa[2 * uu + 1];
    const int hh = a.h[uu];
    const double aa = a.a[uu];
    const int ai = a.ant ? a.ant[2 * uu] : -1, aj = a.ant ? a.ant[2 * uu + 1] : -1;
    const bool dde = ai >= 0;
    const int sd = dde ? 2 * a.sa - 1 : 1;
    const int Lu = J + 2 * hh, S = Lu + sd - 1, ext = hh + (sd - 1) / 2;
    const double fy = floor(ky - 0.5 * J), fx = floor(kx - 0.5 * J);
    bool ok = isfinite(ky) && isfinite(kx) && hh >= 0 && Lu <= kBuildMaxU && S == Sd &&
              (!dde || (ai < a.n_ant && aj >= 0 && aj < a.n_ant));
    if (ok) {
      int64_t by = (int64_t)fy + 1 - ext, bx = (int64_t)fx + 1 - ext;
      by %= a.Ky;
      bx %= a.Kx;
      if (by < 0) by += a.Ky;
      if (bx < 0) bx += a.Kx;
      ok = by == byd && bx == bxd;
    }
    if (!ok) {
      if (lane == 0) a.flag[0] = 1;
      tap += (int64_t)Sd * Sd;
      continue;
    }
    // Kaiser-Bessel taps: lanes 0..J-1 for y, 32..32+J-1 for x
    if ((lane & 31) < J) {
      const int i = lane & 31;
      const double d = (lane < 32 ? ky - (fy + 1.0 + i) : kx - (fx + 1.0 + i)) * (2.0 / J);
      const double t = 1.0 - d * d;
      psi[lane >> 5][i] = t >= 0.0 ? bessel_i0_series(a.beta * sqrt(t)) * a.inv_i0b : 0.0;
    }
    // w-chirp taps k = -h..h (unnormalised)
    if (lane <= 2 * hh) {
      const int k = lane - hh;
      const double c = cos(M_PI * k / (2.0 * (hh + 1)));
      const double ph = -M_PI * (double)k * k / (4.0 * fmax(aa, 0.5));
      cw[lane] = make_double2(c * c * cos(ph), c * c * sin(ph));
    }
    __syncthreads();
    // normalisation (same sum on every lane, fixed order)
    double2 cs = make_double2(0.0, 0.0);
    for (int k = 0; k <= 2 * hh; ++k) {
      cs.x += cw[k].x;
      cs.y += cw[k].y;
    }
    const double cn = cs.x * cs.x + cs.y * cs.y;
    // u = psi (*) (c / sum c): lanes 0..Lu-1 for y, 32.. for x
    if ((lane & 31) < Lu) {
      const int i = lane & 31, ax = lane >> 5;
      double2 acc = make_double2(0.0, 0.0);
      for (int j = max(0, i - 2 * hh); j <= min(i, J - 1); ++j) {
        const double2 c = cw[i - j];
        acc.x += psi[ax][j] * c.x;
        acc.y += psi[ax][j] * c.y;
      }
      // divide by the (complex) tap sum
      u[ax][i] = make_double2((acc.x * cs.x + acc.y * cs.y) / cn, (acc.y * cs.x - acc.x * cs.y) / cn);
    }
    // pair kernel p[r][c] = sum_{p,q} d_i[p][q] conj(d_j[sa-1-(r-p)][sa-1-(c-q)])
    if (dde) {
      const int sa = a.sa;
      const double2* __restrict__ di = reinterpret_cast<const double2*>(a.dde) + (int64_t)ai * sa * sa;
      const double2* __restrict__ dj = reinterpret_cast<const double2*>(a.dde) + (int64_t)aj * sa * sa;
      for (int e = lane; e < sd * sd; e += 64) {
        const int r = e / sd, c = e - (e / sd) * sd;
        double2 acc = make_double2(0.0, 0.0);
        for (int p = max(0, r - sa + 1); p <= min(r, sa - 1); ++p)
          for (int q = max(0, c - sa + 1); q <= min(c, sa - 1); ++q) {
            const double2 x = di[p * sa + q], y = dj[(sa - 1 - (r - p)) * sa + (sa - 1 - (c - q))];
            acc.x += x.x * y.x + x.y * y.y;  // x conj(y)
            acc.y += x.y * y.x - x.x * y.y;
          }
        pk[e] = acc;
      }
    }
    __syncthreads();
    for (int t = lane; t < S * S; t += 64) {
      const int r = t / S, c = t - (t / S) * S;
      double re = 0.0, im = 0.0;
      if (!dde) {
        const double2 y = u[0][r], x = u[1][c];
        re = y.x * x.x - y.y * x.y;
        im = y.x * x.y + y.y * x.x;
      } else {
        for (int p = max(0, r - Lu + 1); p <= min(r, sd - 1); ++p) {
          const double2 y = u[0][r - p];
          for (int q = max(0, c - Lu + 1); q <= min(c, sd - 1); ++q) {
            const double2 x = u[1][c - q], w = pk[p * sd + q];
            const double yr = y.x * x.x - y.y * x.y, yi = y.x * x.y + y.y * x.x;
            re += yr * w.x - yi * w.y;
            im += yr * w.y + yi * w.x;
          }
        }
      }
      store_tap(a.G, a.gprec, tap + t, re, im);
    }
    __syncthreads();  // the tables are rewritten for the next window
    tap += (int64_t)S * S;
  }
}

// ------------------------------------------------- gridding reduction (DR)
// Section 3.4, eqs. 4-5, for one block with whitening theta: H = G^H theta^2 G,
// Lam = H_pp^(-1/2) on the support, y' = Lam G^H theta y, Phi' = Lam H F Z.
// With H0 = G^H G and Lam0 = H0_pp^(-1/2) this is Lam H = theta Lam0 H0 and
// y' = Lam0 G^H y: the reduced rows store Lam0 H0 (theta-free, so FP16
// keeps its range) and the reduced plan applies theta_b like any plan.
//
// One wave per reduced row p: it scans the block's visibilities whose window
// origins lie in the tiles that can reach p (64 at a time, coverage tested
// per lane), and for each window m covering p, in plan order, adds
// conj(g_m[p]) g_m[q] to every entry q of the row's window and
// conj(g_m[p]) y_m to y', in FP64.  Lanes own fixed window entries, so the
// order of every sum is fixed.  The row is then scaled by Lam0 and rounded
// once to the stored precision.
constexpr int kDrMaxSteps = 7;  // row windows up to 21 x 21 = 441 entries

__device__ __forceinline__ double2 load_tap_d(const void* G, int gprec, int64_t t) {
  if (gprec == 0) {
    const float2 g = reinterpret_cast<const float2*>(G)[t];
    return make_double2(g.x, g.y);
  }
  const uint32_t r = reinterpret_cast<const uint32_t*>(G)[t];
  if (gprec == 1)
    return make_double2((double)(float)__builtin_bit_cast(_Float16, (uint16_t)(r & 0xFFFFu)),
                        (double)(float)__builtin_bit_cast(_Float16, (uint16_t)(r >> 16)));
  return make_double2((double)__uint_as_float(r << 16), (double)__uint_as_float(r & 0xFFFF0000u));
}

__global__ __launch_bounds__(256) void k_dr_setup(DrArgs a) {
  const DrGroup grp = a.groups[blockIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int r = grp.row0 + wv; r < grp.row1; r += 4) {
    const DrRow row = a.rows[r];
    const int py = (int)(row.cell & 8191u), px = (int)((row.cell >> 13) & 8191u);
    const uint32_t rm = a.rmeta[row.pos];
    const int s = 2 * (int)(rm >> 26) + 1, oy = (int)(rm & 8191u), ox = (int)((rm >> 13) & 8191u);
    int dy0 = py - oy, dx0 = px - ox;  // p inside the row's window
    if (dy0 < 0) dy0 += a.Ky;
    if (dx0 < 0) dx0 += a.Kx;
    const float rs = 1.0f / (float)s;
    double ar[kDrMaxSteps], ai[kDrMaxSteps];
    int ei[kDrMaxSteps], ej[kDrMaxSteps];
#pragma unroll
    for (int k = 0; k < kDrMaxSteps; ++k) {
      ar[k] = ai[k] = 0.0;
      const int e = k * 64 + lane;
      ei[k] = tap_row(e, rs);
      ej[k] = e - ei[k] * s;
    }
    double yr = 0.0, yi = 0.0;
    for (int c = grp.cand0; c < grp.cand1; ++c) {
      const DrCand cd = a.cands[c];
      int64_t tbase = cd.tap0;
      for (int v = cd.v0; v < cd.v1; v += 64) {
        const int m = v + lane;
        const bool live = m < cd.v1;
        const uint32_t mm = live ? a.meta[m] : 0u;
        const int S = live ? 2 * (int)(mm >> 26) + 1 : 0;
        // tap offsets of the 64 windows: exclusive prefix sum of S^2
        int incl = S * S;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const int t = __shfl_up(incl, off, 64);
          if (lane >= off) incl += t;
        }
        const int64_t tm = tbase + (incl - S * S);
        tbase += __shfl(incl, 63, 64);
        int ry = py - (int)(mm & 8191u), rx = px - (int)((mm >> 13) & 8191u);
        if (ry < 0) ry += a.Ky;
        if (rx < 0) rx += a.Kx;
        uint64_t cov = __ballot(live && ry < S && rx < S);
        while (cov) {
          const int i = __builtin_ctzll(cov);
          cov &= cov - 1;
          const int Si = __shfl(S, i, 64), ryi = __shfl(ry, i, 64), rxi = __shfl(rx, i, 64);
          const int64_t ti = uniform64(__shfl(tm, i, 64));
          const double2 gp = load_tap_d(a.G, a.gprec_g, ti + ryi * Si + rxi);  // g_m[p]
          if (a.y) {
            const float2 ym = a.y[v + i];
            yr += gp.x * ym.x + gp.y * ym.y;  // conj(g_m[p]) y_m
            yi += gp.x * ym.y - gp.y * ym.x;
          }
#pragma unroll
          for (int k = 0; k < kDrMaxSteps; ++k) {
            const int ty = ryi - dy0 + ei[k], tx = rxi - dx0 + ej[k];
            if (k * 64 + lane < s * s && ty >= 0 && ty < Si && tx >= 0 && tx < Si) {
              const double2 g = load_tap_d(a.G, a.gprec_g, ti + ty * Si + tx);
              ar[k] += gp.x * g.x + gp.y * g.y;  // conj(g_m[p]) g_m[q]
              ai[k] += gp.x * g.y - gp.y * g.x;
            }
          }
        }
      }
    }
    // H0_pp sits at entry dy0 * s + dx0; Lam0 = H0_pp^(-1/2) (0 off the support)
    const int ed = dy0 * s + dx0;
    double hd = 0.0;
#pragma unroll
    for (int k = 0; k < kDrMaxSteps; ++k)
      if (k == (ed >> 6)) hd = __shfl(ar[k], ed & 63, 64);
    const double lam = hd > 0.0 ? 1.0 / sqrt(hd) : 0.0;
#pragma unroll
    for (int k = 0; k < kDrMaxSteps; ++k) {
      const int e = k * 64 + lane;
      if (e < s * s) store_tap(a.H, a.gprec_h, row.tap + e, lam * ar[k], lam * ai[k]);
    }
    if (lane == 0) a.yred[row.pos] = make_float2((float)(lam * yr), (float)(lam * yi));
  }
}

// v+ = sigma_b scale_b c over each block's visibilities (fused dual step; a
// block is one plan-order range): gridDim.x work-groups per block stream it
__global__ __launch_bounds__(256) void k_vscale(const BlockInfo* __restrict__ blocks, float2* __restrict__ vis,
                                                const double* __restrict__ sigma, const double* __restrict__ scale,
                                                int b0) {
  const int b = b0 + blockIdx.y;
  const BlockInfo bi = blocks[b];
  const float f = (float)((sigma ? sigma[b] : 1.0) * scale[b]);
  for (int64_t v = bi.v0 + (int64_t)blockIdx.x * 256 + threadIdx.x; v < bi.v1; v += (int64_t)gridDim.x * 256) {
    const float2 c = vis[v];
    vis[v] = make_float2(f * c.x, f * c.y);
  }
}

// ------------------------------------------------------------- launchers
constexpr int kFftThreads = 256;
// Threads of a row transform: one per radix-8 butterfly of the half-length
// complex transform (N/16), 64 to 512.
template <int N>
constexpr int row_threads() {
  return N / 16 < 64 ? 64 : N / 16 > 512 ? 512 : N / 16;
}
// Column panels of 32 KiB or more likewise get 512 threads, 64 KiB ones 1024.
template <int CELLS>
constexpr int panel_threads() {
  return CELLS * 8 >= 65536 ? 1024 : CELLS * 8 >= 32768 ? 512 : kFftThreads;
}
constexpr int kFftCells = 8192;  // N * W per work-group: 64 KiB of LDS

template <int N>
hipError_t rowfft_fwd_n(const float* x, float2* half, const float* sy, const float* sx, const float2* tw,
                        int Ny, int Nx, int l0, int nl, hipStream_t s) {
  hipLaunchKernelGGL((k_rowfft_fwd<N, row_threads<N>()>), dim3(Ny, nl), dim3(row_threads<N>()), 0, s, x, half, sy, sx,
                     tw, Ny, Nx, l0);
  return hipGetLastError();
}
template <int N>
hipError_t rowfft_inv_n(const float2* half, float* x, const float* sy, const float* sx, const float2* tw,
                        int Ny, int Nx, int l0, int nl, hipStream_t s) {
  hipLaunchKernelGGL((k_rowfft_inv<N, row_threads<N>()>), dim3(Ny, nl), dim3(row_threads<N>()), 0, s, half, x, sy, sx,
                     tw, Ny, Nx, l0);
  return hipGetLastError();
}
template <int N>
constexpr int col_width() {
  return (kFftCells / N) > 16 ? 16 : (kFftCells / N) < 1 ? 1 : kFftCells / N;
}
// Long columns: (N1, N2) of the two-pass transform, or (0, 0) for one pass.
template <int N>
constexpr int col_split1() {
  return N == 3072 ? 48 : N == 4096 ? 64 : N == 5120 ? 40 : N == 6144 ? 48 : N == 8192 ? 64 : 0;
}
// Columns per work-group in the two-pass transform (divides every valid Kx:
// image edges are multiples of 16, so Kx is a multiple of 32; 64-column
// panels in the second pass measured slower).
constexpr int kColW2 = 32;

template <int N1, int N2, bool INV>
hipError_t colfft2_pass_b(float2* grid, const float2* tw, int Kx, int l0, int nl, hipStream_t s) {
  constexpr int W = kColW2, T = panel_threads<N1 * W>();
  hipLaunchKernelGGL((k_colfft2_b<N1, N2, W, T, INV>), dim3(N2 * (Kx / W), nl), dim3(T), 0, s, grid, tw, Kx, l0);
  return hipGetLastError();
}

template <int N>
hipError_t colfft_fwd_n(const float2* half, float2* grid, const float2* tw, int Ny, int Kx, int l0, int nl,
                        hipStream_t s) {
  constexpr int N1 = col_split1<N>();
  if constexpr (N1 > 0) {
    constexpr int N2 = N / N1, W = kColW2;
    if (Kx % W == 0) {
      constexpr int TA = panel_threads<N2 * W>();
      hipLaunchKernelGGL((k_colfft2_fwd_a<N1, N2, W, TA>), dim3(N1 * (Kx / W), nl), dim3(TA), 0, s, half, grid, tw,
                         Ny, Kx, l0);
      return colfft2_pass_b<N1, N2, false>(grid, tw, Kx, l0, nl, s);
    }
  }
  constexpr int W = col_width<N>();
  if (Kx % W) return hipErrorInvalidValue;
  constexpr int NT = panel_threads<N * W>();
  hipLaunchKernelGGL((k_colfft_fwd<N, W, NT>), dim3(Kx / W, nl), dim3(NT), 0, s, half, grid,
                     tw, Ny, Kx, l0);
  return hipGetLastError();
}
template <int N>
hipError_t colfft_inv_n(const float2* grid, float2* half, const float2* tw, int Ny, int Kx, int l0, int nl,
                        hipStream_t s) {
  constexpr int N1 = col_split1<N>();
  if constexpr (N1 > 0) {
    constexpr int N2 = N / N1, W = kColW2;
    if (Kx % W == 0) {
      // the pass along k1 runs in place on the grid, which the adjoint no
      // longer needs afterwards
      constexpr int TA = panel_threads<N2 * W>();
      const hipError_t e = colfft2_pass_b<N1, N2, true>(const_cast<float2*>(grid), tw, Kx, l0, nl, s);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_colfft2_inv_a<N1, N2, W, TA>), dim3(N1 * (Kx / W), nl), dim3(TA), 0, s, grid, half, tw,
                         Ny, Kx, l0);
      return hipGetLastError();
    }
  }
  constexpr int W = col_width<N>();
  if (Kx % W) return hipErrorInvalidValue;
  constexpr int NT = panel_threads<N * W>();
  hipLaunchKernelGGL((k_colfft_inv<N, W, NT>), dim3(Kx / W, nl), dim3(NT), 0, s, grid, half,
                     tw, Ny, Kx, l0);
  return hipGetLastError();
}

// Packed-column panel width of the image-first transform for an image width
// Nx (Nx / 2 packed columns), or 0 when the transform runs rows first.
inline int colr_width(int Nx) { return (Nx / 2) % 32 == 0 ? 32 : (Nx / 2) % 8 == 0 ? 8 : 0; }

template <int N, int W>
hipError_t colr_fwd_nw(const float* x, float2* zp, float2* T, const float* sy, const float* sx, const float2* tw,
                       int Ny, int Nx, int l0, int nl, hipStream_t s) {
  constexpr int N1 = col_split1<N>(), N2 = N / N1;
  constexpr int TA = panel_threads<N2 * W>(), TB = panel_threads<N1 * 2 * W>();
  const int npc = (Nx / 2) / W;
  const size_t zs = (size_t)N * 2 * Nx;  // each channel's packed columns in its own grid region
  hipLaunchKernelGGL((k_colr_fwd_a<N1, N2, W, TA>), dim3(N1 * npc, nl), dim3(TA), 0, s, x, zp, sy, sx, tw, Ny, Nx, l0,
                     zs);
  hipLaunchKernelGGL((k_colr_fwd_b<N1, N2, W, TB>), dim3((N2 / 2 + 1) * npc, nl), dim3(TB), 0, s, zp, T, tw, Nx, l0,
                     zs);
  return hipGetLastError();
}
template <int N, int W>
hipError_t colr_inv_nw(const float2* T, float2* zp, float* x, const float* sy, const float* sx, const float2* tw,
                       int Ny, int Nx, int l0, int nl, hipStream_t s) {
  constexpr int N1 = col_split1<N>(), N2 = N / N1;
  constexpr int TA = panel_threads<N2 * W>(), TB = panel_threads<N1 * 2 * W>();
  const int npc = (Nx / 2) / W;
  const size_t zs = (size_t)N * 2 * Nx;  // each channel's packed columns in its own grid region
  hipLaunchKernelGGL((k_colr_inv_b<N1, N2, W, TB>), dim3((N2 / 2 + 1) * npc, nl), dim3(TB), 0, s, T, zp, tw, Nx, l0,
                     zs);
  hipLaunchKernelGGL((k_colr_inv_a<N1, N2, W, TA>), dim3(N1 * npc, nl), dim3(TA), 0, s, zp, x, sy, sx, tw, Ny, Nx, l0,
                     zs);
  return hipGetLastError();
}

// Row passes of the image-first transform (Kx = N, Nx = N / 2).
// Resident work-groups of a persistent kernel over the current device (its
// occupancy per CU times the CU count); `cache` holds one value per device.
template <typename K>
int resident_groups(K kernel, int threads, int* cache) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cache[dev] == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
      return 0;
    cache[dev] = std::max(1, per_cu) * std::max(1, cus);
  }
  return cache[dev];
}
// Region masks of the inverse row pass: R a power of two >= 16 dividing Ky
// and N, one word per 32 regions of a row.
bool live_regions_fit(const LiveRegions& live, int N, int Ky) {
  return !live.bits || (live.R >= 16 && !(live.R & (live.R - 1)) && Ky % live.R == 0 && N % live.R == 0 &&
                        live.wpr * 32 >= N / live.R);
}
template <int N, int NT>
hipError_t rowc_fwd_nt(const float2* T, float2* grid, const float2* tw, int Ky, int l0, int nl, hipStream_t s) {
  static int cache[64] = {0};
  const int g = resident_groups(k_rowc_fwd_p<N, NT>, NT, cache);
  if (g <= 0) return hipErrorInvalidDevice;
  const int nrows = Ky * nl;
  hipLaunchKernelGGL((k_rowc_fwd_p<N, NT>), dim3(std::min(g, nrows)), dim3(NT), 0, s, T, grid, tw, Ky, l0, nrows);
  return hipGetLastError();
}
template <int N, int NT>
hipError_t rowc_inv_nt(const float2* grid, float2* T, const float2* tw, int Ky, int l0, int nl, LiveRegions live,
                       hipStream_t s) {
  static int cache[64] = {0};
  if (!live_regions_fit(live, N, Ky)) return hipErrorInvalidValue;
  const int g = resident_groups(k_rowc_inv_p<N, NT>, NT, cache);
  if (g <= 0) return hipErrorInvalidDevice;
  const int nrows = Ky * nl;
  hipLaunchKernelGGL((k_rowc_inv_p<N, NT>), dim3(std::min(g, nrows)), dim3(NT), 0, s, grid, T, tw, Ky, l0, nrows,
                     live);
  return hipGetLastError();
}
template <int N>
hipError_t rowc_fwd_n(const float2* T, float2* grid, const float2* tw, int Ky, int l0, int nl, hipStream_t s) {
  return rowc_fwd_nt<N, rowc_threads<N>()>(T, grid, tw, Ky, l0, nl, s);
}
// The inverse holds a whole grid row (16 bytes per element pair) in flight:
// long rows take half the threads, each with twice the registers (8192
// points: 2.83 ms against 3.11 ms with 1024 threads, which spill the prefetch;
// the forward is faster with 1024, 2.76 against 2.85 ms).
template <int N>
hipError_t rowc_inv_n(const float2* grid, float2* T, const float2* tw, int Ky, int l0, int nl, LiveRegions live,
                      hipStream_t s) {
  constexpr int NT = N >= 2048 ? rowc_threads<N>() / 2 : rowc_threads<N>();
  return rowc_inv_nt<N, NT>(grid, T, tw, Ky, l0, nl, live, s);
}

#define PHI_FFT_SIZES(X)                                                                              \
  X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(640) X(768) X(1024) X(1280) X(1536) \
      X(2048) X(2560) X(3072) X(4096) X(5120) X(6144) X(8192)

}  // namespace

bool fft_length_supported(int n) {
  switch (n) {
#define X(N) case N:
    PHI_FFT_SIZES(X)
#undef X
    return true;
    default:
      return false;
  }
}

hipError_t launch_rowfft_fwd(int Kx, const float* x, float2* half, const float* sy, const float* sx,
                             const float2* tw, int Ny, int Nx, int l0, int nl, hipStream_t s) {
  switch (Kx) {
#define X(N) \
  case N:    \
    return rowfft_fwd_n<N>(x, half, sy, sx, tw, Ny, Nx, l0, nl, s);
    PHI_FFT_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}
hipError_t launch_rowfft_inv(int Kx, const float2* half, float* x, const float* sy, const float* sx,
                             const float2* tw, int Ny, int Nx, int l0, int nl, hipStream_t s) {
  switch (Kx) {
#define X(N) \
  case N:    \
    return rowfft_inv_n<N>(half, x, sy, sx, tw, Ny, Nx, l0, nl, s);
    PHI_FFT_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}
hipError_t launch_colfft_fwd(int Ky, const float2* half, float2* grid, const float2* tw, int Ny, int Kx, int l0,
                             int nl, hipStream_t s) {
  switch (Ky) {
#define X(N) \
  case N:    \
    return colfft_fwd_n<N>(half, grid, tw, Ny, Kx, l0, nl, s);
    PHI_FFT_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}
hipError_t launch_colfft_inv(int Ky, const float2* grid, float2* half, const float2* tw, int Ny, int Kx, int l0,
                             int nl, hipStream_t s) {
  switch (Ky) {
#define X(N) \
  case N:    \
    return colfft_inv_n<N>(grid, half, tw, Ny, Kx, l0, nl, s);
    PHI_FFT_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// Step-count class of a plan: the kernels instantiate item paths up to NKM
// 64-tap steps (windows up to 7 x 7, 17 x 17 or 21 x 21).
static int nk_class(int max_pitch, int T) {
  const int smax = max_pitch - T + 1, nk = (smax * smax + 63) / 64;
  return nk <= 1 ? 1 : nk <= 5 ? 5 : 7;
}

template <int GP, int MODE>
static hipError_t gather_m(int nkc, const GArgs& a, float2* vis, const float2* y, double* norms, size_t lds,
                           int it0, int it1, int nb, hipStream_t s) {
  const dim3 g(nb), b(64 * kGatherWaves);
  if (nkc == 1)
    hipLaunchKernelGGL((k_gather<GP, MODE, 1>), g, b, lds, s, a, vis, y, norms, it0, it1);
  else if (nkc == 5)
    hipLaunchKernelGGL((k_gather<GP, MODE, 5>), g, b, lds, s, a, vis, y, norms, it0, it1);
  else
    hipLaunchKernelGGL((k_gather<GP, MODE, 7>), g, b, lds, s, a, vis, y, norms, it0, it1);
  return hipGetLastError();
}
template <int GP>
static hipError_t gather_gp(int mode, int nkc, const GArgs& a, float2* vis, const float2* y, double* norms,
                            size_t lds, int it0, int it1, int nb, hipStream_t s) {
  return mode == 0   ? gather_m<GP, 0>(nkc, a, vis, y, norms, lds, it0, it1, nb, s)
         : mode == 1 ? gather_m<GP, 1>(nkc, a, vis, y, norms, lds, it0, it1, nb, s)
                     : gather_m<GP, 2>(nkc, a, vis, y, norms, lds, it0, it1, nb, s);
}

size_t fused_lds_bytes(int max_pitch) {
  const size_t pp = (size_t)max_pitch * max_pitch;
  const size_t bytes = (pp + 16 + (size_t)kGatherWaves * (pp + 64)) * sizeof(float2);
  return bytes <= 65536 ? bytes : 0;
}

size_t kb_fused_lds_bytes(int max_pitch) {
  const size_t pp = (size_t)max_pitch * max_pitch;
  const size_t bytes = (2 * pp + 64) * sizeof(float2);  // tile, accumulator, spare cells
  return bytes <= 57344 ? bytes : 0;                   // with the static tap table, under 64 KiB
}

hipError_t launch_gather(int gprec, int mode, const GArgs& a, float2* vis, const float2* y, double* item_norms,
                         int max_pitch, int it0, int it1, int grid_blocks, hipStream_t s) {
  const int n = it1 - it0;
  if (n <= 0) return hipSuccess;
  const int nb = grid_blocks > 0 && grid_blocks < n ? grid_blocks : n;
  const size_t lds = mode == 2 ? fused_lds_bytes(max_pitch)
                               : ((size_t)max_pitch * max_pitch + 64) * sizeof(float2);  // tile, zero cell, norms
  if (lds == 0 || lds > 65536) return hipErrorInvalidValue;
  if (gprec == 3 && mode == 2) {  // one wave per item: tile and accumulator in LDS
    const size_t kb_lds = kb_fused_lds_bytes(max_pitch);
    if (kb_lds == 0) return hipErrorInvalidValue;
#define PHI_KB_D(JJ)                                                                                  \
  case JJ:                                                                                            \
    hipLaunchKernelGGL((k_dual_kb<JJ>), dim3(nb), dim3(64), kb_lds, s, a, vis, y, item_norms, it0, it1); \
    return hipGetLastError();
    switch (a.kb_J) {
      PHI_KB_D(3)
      PHI_KB_D(5)
      PHI_KB_D(7)
      PHI_KB_D(9)
      PHI_KB_D(11)
      default:
        return hipErrorInvalidValue;
    }
#undef PHI_KB_D
  }
  if (gprec == 3) {
    const dim3 g(nb), b(64 * kGatherWaves);
#define PHI_KB_G(JJ)                                                                                       \
  case JJ:                                                                                                 \
    if (mode == 0)                                                                                         \
      hipLaunchKernelGGL((k_gather_kb<0, JJ>), g, b, lds, s, a, vis, y, item_norms, it0, it1);            \
    else                                                                                                   \
      hipLaunchKernelGGL((k_gather_kb<1, JJ>), g, b, lds, s, a, vis, y, item_norms, it0, it1);            \
    return hipGetLastError();
    switch (a.kb_J) {
      PHI_KB_G(3)
      PHI_KB_G(5)
      PHI_KB_G(7)
      PHI_KB_G(9)
      PHI_KB_G(11)
      default:
        return hipErrorInvalidValue;
    }
#undef PHI_KB_G
  }
  const int nkc = nk_class(max_pitch, a.T);
  switch (gprec) {
    case 0: return gather_gp<0>(mode, nkc, a, vis, y, item_norms, lds, it0, it1, nb, s);
    case 1: return gather_gp<1>(mode, nkc, a, vis, y, item_norms, lds, it0, it1, nb, s);
    case 2: return gather_gp<2>(mode, nkc, a, vis, y, item_norms, lds, it0, it1, nb, s);
    default: return hipErrorInvalidValue;
  }
}

template <int GP, int MODE>
static hipError_t scatter_m(int nkc, const GArgs& a, float2* vis, float2* partials, size_t lds, int it0, int it1,
                            int nb, hipStream_t s) {
  const dim3 g(nb), b(64);
  if (nkc == 1)
    hipLaunchKernelGGL((k_scatter<GP, MODE, 1>), g, b, lds, s, a, vis, partials, it0, it1);
  else if (nkc == 5)
    hipLaunchKernelGGL((k_scatter<GP, MODE, 5>), g, b, lds, s, a, vis, partials, it0, it1);
  else
    hipLaunchKernelGGL((k_scatter<GP, MODE, 7>), g, b, lds, s, a, vis, partials, it0, it1);
  return hipGetLastError();
}
template <int GP>
static hipError_t scatter_gp(int mode, int nkc, const GArgs& a, float2* vis, float2* partials, size_t lds, int it0,
                             int it1, int nb, hipStream_t s) {
  return mode == 0 ? scatter_m<GP, 0>(nkc, a, vis, partials, lds, it0, it1, nb, s)
                   : scatter_m<GP, 1>(nkc, a, vis, partials, lds, it0, it1, nb, s);
}

hipError_t launch_scatter(int gprec, int mode, const GArgs& a, float2* vis, float2* partials, int max_pitch,
                          int it0, int it1, int grid_blocks, hipStream_t s) {
  const int n = it1 - it0;
  if (n <= 0) return hipSuccess;
  const int nb = grid_blocks > 0 && grid_blocks < n ? grid_blocks : n;
  const size_t lds = ((size_t)max_pitch * max_pitch + 64) * sizeof(float2);  // accumulator, spare cells
  if (lds > 65536) return hipErrorInvalidValue;
  if (gprec == 3) {
    const dim3 g(nb), b(64);
#define PHI_KB_S(JJ)                                                                                      \
  case JJ:                                                                                                \
    if (mode == 0)                                                                                        \
      hipLaunchKernelGGL((k_scatter_kb<0, JJ>), g, b, lds, s, a, vis, partials, it0, it1);               \
    else                                                                                                  \
      hipLaunchKernelGGL((k_scatter_kb<1, JJ>), g, b, lds, s, a, vis, partials, it0, it1);               \
    return hipGetLastError();
    switch (a.kb_J) {
      PHI_KB_S(3)
      PHI_KB_S(5)
      PHI_KB_S(7)
      PHI_KB_S(9)
      PHI_KB_S(11)
      default:
        return hipErrorInvalidValue;
    }
#undef PHI_KB_S
  }
  const int nkc = nk_class(max_pitch, a.T);
  switch (gprec) {
    case 0: return scatter_gp<0>(mode, nkc, a, vis, partials, lds, it0, it1, nb, s);
    case 1: return scatter_gp<1>(mode, nkc, a, vis, partials, lds, it0, it1, nb, s);
    case 2: return scatter_gp<2>(mode, nkc, a, vis, partials, lds, it0, it1, nb, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_merge(float2* grid, const float2* partials, const int32_t* tile_ptr, const TileEntry* entries,
                        const int32_t* live, int live0, int n_live, int Ky, int Kx, int T, int halo, int rk, int l0,
                        int nl, const double* sigma, const double* scale, const float* theta, hipStream_t s) {
  if (scale && !theta) return hipErrorInvalidValue;
  if (rk < 1 || rk > 4 || (rk + halo) * (rk + halo) > kMergeSrc || Ky % (rk * T) || Kx % (rk * T))
    return hipErrorInvalidValue;
  const int regions = (Ky / (rk * T)) * (Kx / (rk * T));
  if (live && n_live <= 0) return hipSuccess;
  const dim3 g = live ? dim3(n_live) : dim3(regions, nl);
  hipLaunchKernelGGL(k_merge, g, dim3(256), 0, s, grid, partials, tile_ptr, entries, live, live0, Ky, Kx, T, halo,
                     rk, l0, sigma, scale, theta);
  return hipGetLastError();
}

bool fft_inverse_reads_grid_only(int Ky, int Nx) {
  switch (Ky) {
    case 3072: case 4096: case 5120: case 6144: case 8192:
      return fft_image_first(Ky, Nx);
    default:
      return true;
  }
}

hipError_t launch_finalize(const double* item_norms, const BlockInfo* blocks, double* block_part, const double* eps,
                           double* rho, double* res, double* scale, int* flag, int b0, int nb, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_sums, dim3(kFinChunks, nb), dim3(256), 0, s, item_norms, blocks, block_part, b0);
  hipLaunchKernelGGL(k_finalize, dim3(nb), dim3(64), 0, s, block_part, eps, rho, res, scale, flag, b0);
  return hipGetLastError();
}

hipError_t launch_permute(const float2* src, float2* dst, const int32_t* perm, int64_t n, int to_plan,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, perm, n, to_plan);
  return hipGetLastError();
}

hipError_t launch_delta(float* x, int L, int Ny, int Nx, hipStream_t s) {
  const int64_t n = (int64_t)Ny * Nx;
  hipLaunchKernelGGL(k_delta, dim3((unsigned)((n + 255) / 256), L), dim3(256), 0, s, x, Ny, Nx);
  return hipGetLastError();
}

hipError_t launch_vis_residual(float2* v, const float2* y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vis_residual, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, y, n);
  return hipGetLastError();
}

hipError_t launch_chan_norm(const float* x, int L, int64_t n, double* part, double* norm, double* inv,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_chan_sumsq, dim3(kNormChunks, L), dim3(256), 0, s, x, n, part);
  hipLaunchKernelGGL(k_chan_norm, dim3(L), dim3(64), 0, s, part, norm, inv);
  return hipGetLastError();
}

hipError_t launch_chan_scale(float* x, const double* f, int L, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_chan_scale, dim3((unsigned)((n + 255) / 256), L), dim3(256), 0, s, x, f, n);
  return hipGetLastError();
}

hipError_t launch_centre_value(const float* x, int L, int Ny, int Nx, double* peak, hipStream_t s) {
  hipLaunchKernelGGL(k_centre_value, dim3((L + 63) / 64), dim3(64), 0, s, x, L, Ny, Nx, peak);
  return hipGetLastError();
}

hipError_t launch_pdfb_primal(float* x, float* xt, const float* g, const double* tau, int L, int64_t n,
                              double* part, double* var, hipStream_t s) {
  if (L <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pdfb_primal, dim3(kNormChunks, L), dim3(256), 0, s, x, xt, g, tau, n, part);
  if (var) hipLaunchKernelGGL(k_pdfb_var, dim3(L), dim3(64), 0, s, part, var);
  return hipGetLastError();
}

hipError_t launch_eps_update(const double* res, const double* var, const BlockInfo* blocks, int nblk,
                             EpsRule rule, double* eps, int32_t* state, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_eps_update, dim3((nblk + 63) / 64), dim3(64), 0, s, res, var, blocks, nblk, rule, eps,
                     state);
  return hipGetLastError();
}

hipError_t launch_build_g(const BuildArgs& a, int it0, int it1, hipStream_t s) {
  if (it1 <= it0) return hipSuccess;
  hipLaunchKernelGGL(k_build_g, dim3(it1 - it0), dim3(64), 0, s, a, it0);
  return hipGetLastError();
}

hipError_t launch_vscale(const BlockInfo* blocks, float2* vis, const double* sigma, const double* scale, int b0,
                         int nb, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  const int chunks = std::max(64, (4096 + nb - 1) / nb);  // >= 4096 work-groups over the chip
  hipLaunchKernelGGL(k_vscale, dim3(chunks, nb), dim3(256), 0, s, blocks, vis, sigma, scale, b0);
  return hipGetLastError();
}

hipError_t launch_dr_setup(const DrArgs& a, int n_groups, hipStream_t s) {
  if (n_groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dr_setup, dim3(n_groups), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Image-first 2-D transform (grids with two-pass columns): see k_colr_fwd_a.
bool fft_image_first(int Ky, int Nx) {
  switch (Ky) {
    case 3072: case 4096: case 5120: case 6144: case 8192:
      return colr_width(Nx) > 0;
    default:
      return false;
  }
}

#define PHI_COLR_SIZES(X) X(3072) X(4096) X(5120) X(6144) X(8192)

hipError_t launch_colr_fwd(int Ky, const float* x, float2* zp, float2* T, const float* sy, const float* sx,
                           const float2* tw, int Ny, int Nx, int l0, int nl, hipStream_t s) {
  const int W = colr_width(Nx);
  switch (Ky) {
#define X(N)                                                                                   \
  case N:                                                                                      \
    return W == 32 ? colr_fwd_nw<N, 32>(x, zp, T, sy, sx, tw, Ny, Nx, l0, nl, s)               \
           : W == 8 ? colr_fwd_nw<N, 8>(x, zp, T, sy, sx, tw, Ny, Nx, l0, nl, s) : hipErrorInvalidValue;
    PHI_COLR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}
hipError_t launch_colr_inv(int Ky, const float2* T, float2* zp, float* x, const float* sy, const float* sx,
                           const float2* tw, int Ny, int Nx, int l0, int nl, hipStream_t s) {
  const int W = colr_width(Nx);
  switch (Ky) {
#define X(N)                                                                                   \
  case N:                                                                                      \
    return W == 32 ? colr_inv_nw<N, 32>(T, zp, x, sy, sx, tw, Ny, Nx, l0, nl, s)               \
           : W == 8 ? colr_inv_nw<N, 8>(T, zp, x, sy, sx, tw, Ny, Nx, l0, nl, s) : hipErrorInvalidValue;
    PHI_COLR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}
hipError_t launch_rowc_fwd(int Kx, const float2* T, float2* grid, const float2* tw, int Ky, int l0, int nl,
                           hipStream_t s) {
  switch (Kx) {
#define X(N) \
  case N:    \
    return rowc_fwd_n<N>(T, grid, tw, Ky, l0, nl, s);
    PHI_FFT_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}
hipError_t launch_rowc_inv(int Kx, const float2* grid, float2* T, const float2* tw, int Ky, int l0, int nl,
                           LiveRegions live, hipStream_t s) {
  switch (Kx) {
#define X(N) \
  case N:    \
    return rowc_inv_n<N>(grid, T, tw, Ky, l0, nl, live, s);
    PHI_FFT_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace phi
