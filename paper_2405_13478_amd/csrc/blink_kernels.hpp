// HIP kernels of the dirty-imaging path for gfx950.
//
// Per timestep t (shared by all channels):
//   k_sort_run / k_merge / k_sort_finish - order the usable baselines by u in
//       metres (exact double comparison, ties by baseline index). Because
//       rint(u * s_c) is non-decreasing in u for every s_c > 0, the baselines of
//       one u cell form a contiguous run of this order at EVERY channel, so one
//       sort serves all channels of the timestep.
// Per chunk of images (t, c):
//   k_bounds  - for every signed u cell, the first sorted position at or beyond
//               it (a scan of the sorted u list at this channel's scale).
//   k_grid_cols<N, MODE> - one wavefront per u cell column: gathers the column's
//               baselines (directly and as conjugates of the mirror column),
//               accumulates sums (and counts) in LDS, applies the weighting,
//               then either writes the grid column (MODE_GRID) or runs the
//               inverse transform along v and writes the rows of the cutout
//               (MODE_IMAGE) - the grid never reaches HBM on the image path.
//   k_rows<N> - two image rows per wavefront: Hermitian extension of the half
//               spectrum (u cells 0..N/2-1), inverse transform along u, real
//               part, FFT shift, 1/W and cutout fused into the store.
// The adjoint (differentiation form) runs the same two passes transposed.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "blink_fft.hpp"
#include "twiddles.inc"

namespace blink {

constexpr double C_LIGHT = 299792458.0;   // m/s
constexpr unsigned long long KEY_MAX = ~0ull;

enum { MODE_IMAGE = 0, MODE_GRID = 1 };
enum { VT_C64 = 0, VT_F16 = 1, VT_BF16 = 2 };

// Cells per metre at frequency f: (f * (N dx)) / c, IEEE double, this order.
__device__ __forceinline__ double cells_per_metre(double f, double ndx) {
  const double p = f * ndx;
  return p / C_LIGHT;
}

// Order-preserving map of a double to an unsigned 64-bit key.
__device__ __forceinline__ unsigned long long order_key(double u) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(u);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}

// ============================================================== sort by u
struct SortArgs {
  int T, B;
  int t0;                        // first timestep of this launch (grid.y covers t0 + blockIdx.y)
  const double* uvw;             // [T][B][3]
  const uint8_t* flags;          // [T][B] or null
  unsigned long long* key[2];    // [T][B] ping-pong
  int* idx[2];                   // [T][B]
  int* n_unflagged;              // [T]
  int* n_valid;                  // [T]
  double* su;                    // [T][B] sorted u
  double* sv;                    // [T][B] v in the same order
  int* perm;                     // [T][B] baseline index in the same order
  double* sd;                    // [T][B] delay in the same order, or null (no rotation)
  double pl, pm, pn1;            // phase centre l0, m0 and n0 - 1
  int proj;                      // 1: grid the baselines re-projected onto the new centre's plane
  double eu[3], ev[3];           // with proj: u' = eu . (u, v, w), v' = ev . (u, v, w)
  const double* cable;           // [A] electrical cable lengths (m) or null
  const int* ant1;               // [B] (with cable lengths)
  const int* ant2;               // [B]
  int n_ant;                     // cable length entries; an antenna index outside [0, n_ant) adds 0
  double* vmax;                  // [T] largest |v| of the usable baselines, or null
  // single-image bounds (one channel per timestep): the cell bounds of image t
  // are formed by the sort kernel itself (see k_sort_small)
  int N, kw;                     // grid size, gridding kernel support (0: nearest cell)
  double ndx;                    // fl(N * dx)
  const double* freq;            // [1]
  int* bnd;                      // [T][N + 2]
  int* ncz;                      // [T]
};

// The (u, v) in metres that the imager grids for baseline o of the flat
// [T][B] layout: the baseline's own, or its components along the new
// centre's tangent-plane axes when re-projecting.
__device__ __forceinline__ void plane_uv(const SortArgs& a, size_t o, double& u, double& v) {
  const double* b = a.uvw + o * 3;
  if (a.proj) {
    u = a.eu[0] * b[0] + a.eu[1] * b[1] + a.eu[2] * b[2];
    v = a.ev[0] * b[0] + a.ev[1] * b[1] + a.ev[2] * b[2];
  } else {
    u = b[0];
    v = b[1];
  }
}

// u l0 + v m0 + w (n0 - 1): the path difference (metres) between the new
// phase centre and zenith for baseline uvw.
__device__ __forceinline__ double geo_delay(const double* uvw, double l0, double m0, double n1) {
  return uvw[0] * l0 + uvw[1] * m0 + uvw[2] * n1;
}

// The delay of baseline b (metres): the geometric term plus, with cable
// lengths, l_ant1 - l_ant2 (a longer path delays that antenna's voltage).
// An antenna index outside [0, n_ant) contributes no cable term, as it
// contributes a zero gain on the gains path.
__device__ __forceinline__ double cable_len(const SortArgs& a, int i) {
  return (unsigned)i < (unsigned)a.n_ant ? a.cable[i] : 0.0;
}
__device__ __forceinline__ double baseline_delay(const SortArgs& a, size_t tb, int b) {
  double d = geo_delay(a.uvw + (tb + b) * 3, a.pl, a.pm, a.pn1);
  if (a.cable != nullptr) d += cable_len(a, a.ant1[b]) - cable_len(a, a.ant2[b]);
  return d;
}

__global__ void k_sort_init(int* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

// Bitonic sort of one run of RUN (key, index) pairs in LDS; the pair order is
// total because indices are distinct, so the result equals a stable sort.
template <int RUN>
__global__ void __launch_bounds__(1024) k_sort_run(SortArgs a) {
  __shared__ unsigned long long sk[RUN];
  __shared__ int si[RUN];
  __shared__ int s_unf;
  const int t = a.t0 + blockIdx.y;
  const int base = blockIdx.x * RUN;
  const int len = min(RUN, a.B - base);
  if (threadIdx.x == 0) s_unf = 0;
  __syncthreads();
  int unf = 0;
  for (int i = threadIdx.x; i < RUN; i += blockDim.x) {
    unsigned long long k = KEY_MAX;
    int id = 0x7fffffff;
    if (i < len) {
      const int b = base + i;
      const size_t o = (size_t)t * a.B + b;
      double u, v;
      plane_uv(a, o, u, v);
      const bool flagged = a.flags != nullptr && a.flags[o] != 0;
      unf += flagged ? 0 : 1;
      if (!flagged && isfinite(u) && isfinite(v)) k = order_key(u);
      id = b;
    }
    sk[i] = k;
    si[i] = id;
  }
  if (unf) atomicAdd(&s_unf, unf);
  __syncthreads();
  for (int k = 2; k <= RUN; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < RUN / 2; i += blockDim.x) {
        const int lo = 2 * i - (i & (j - 1));
        const int hi = lo + j;
        const bool up = (lo & k) == 0;
        const unsigned long long ka = sk[lo], kb = sk[hi];
        const int ia = si[lo], ib = si[hi];
        const bool gt = ka > kb || (ka == kb && ia > ib);
        if (gt == up) {
          sk[lo] = kb; sk[hi] = ka;
          si[lo] = ib; si[hi] = ia;
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    const size_t o = (size_t)t * a.B + base + i;
    a.key[0][o] = sk[i];
    a.idx[0][o] = si[i];
  }
  if (threadIdx.x == 0 && s_unf) atomicAdd(&a.n_unflagged[t], s_unf);
}

// Cell bounds of one image from its sorted u (see k_bounds, which documents
// them): ucol(j) is the clamped u cell of sorted position j. Run by one
// workgroup; returns nothing, writes bnd[0 .. N + 1] and *ncz.
template <class UCol>
__device__ __forceinline__ void image_bounds(UCol&& ucol, int nv, int N, int kw, int* bnd, int* ncz) {
  const int H = N / 2;
  const int clast = nv == 0 ? -H - 1 : ucol(nv - 1);
  if (nv > 16 * (N + 2)) {
    for (int c = (int)threadIdx.x - H; c <= H + 1; c += blockDim.x) {
      int lo = 0, hi = nv;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ucol(mid) >= c) hi = mid; else lo = mid + 1;
      }
      bnd[c + H] = lo;
    }
  } else {
    for (int j = threadIdx.x; j < nv; j += blockDim.x) {
      const int cj = ucol(j);
      const int cp = j == 0 ? -H - 1 : ucol(j - 1);
      for (int c = cp + 1; c <= cj; ++c) bnd[c + H] = j;
    }
    for (int c = clast + 1 + (int)threadIdx.x; c <= H + 1; c += blockDim.x) bnd[c + H] = nv;
  }
  // every entry lies in a column |c| <= max(|first|, |last|) of the sorted order;
  // a gridding kernel reaches columns c with |c - x_u| <= W/2, i.e. at most
  // floor(W/2 + 1/2) columns beyond the entry's nearest one
  const int reach = kw > 0 ? (kw + 1) / 2 : 0;
  if (threadIdx.x == 0) *ncz = nv == 0 ? 0 : min(H, max(clast, -ucol(0)) + 1 + reach);
}

// Whole per-timestep order in one kernel when B <= RUN: load, bitonic sort in
// LDS, then the sorted u, v, baseline index, the two counters and the largest
// |v| of the timestep (one workgroup per timestep, so no atomics and no
// initialisation). BOUNDS (one channel per timestep): the same workgroup then
// forms the cell bounds of its image, which saves the bounds launch.
template <int RUN, bool BOUNDS = false>
__global__ void __launch_bounds__(1024) k_sort_small(SortArgs a) {
  __shared__ unsigned long long sk[RUN];
  __shared__ int si[RUN];
  __shared__ int s_unf, s_val;
  __shared__ double s_vm[1024 / WAVE];
  const int t = a.t0 + blockIdx.y;
  const size_t tb = (size_t)t * a.B;
  if (threadIdx.x == 0) { s_unf = 0; s_val = 0; }
  __syncthreads();
  int unf = 0, val = 0;
  for (int i = threadIdx.x; i < RUN; i += blockDim.x) {
    unsigned long long k = KEY_MAX;
    int id = 0x7fffffff;
    if (i < a.B) {
      double u, v;
      plane_uv(a, tb + i, u, v);
      const bool flagged = a.flags != nullptr && a.flags[tb + i] != 0;
      unf += flagged ? 0 : 1;
      if (!flagged && isfinite(u) && isfinite(v)) { k = order_key(u); ++val; }
      id = i;
    }
    sk[i] = k;
    si[i] = id;
  }
  if (unf) atomicAdd(&s_unf, unf);
  if (val) atomicAdd(&s_val, val);
  __syncthreads();
  for (int k = 2; k <= RUN; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < RUN / 2; i += blockDim.x) {
        const int lo = 2 * i - (i & (j - 1));
        const int hi = lo + j;
        const bool up = (lo & k) == 0;
        const unsigned long long ka = sk[lo], kb = sk[hi];
        const int ia = si[lo], ib = si[hi];
        const bool gt = ka > kb || (ka == kb && ia > ib);
        if (gt == up) {
          sk[lo] = kb; sk[hi] = ka;
          si[lo] = ib; si[hi] = ia;
        }
      }
      __syncthreads();
    }
  }
  double vm = 0.0;
  for (int j = threadIdx.x; j < a.B; j += blockDim.x) {
    const int b = si[j];
    double u, v;
    plane_uv(a, tb + b, u, v);
    a.su[tb + j] = u;
    a.sv[tb + j] = v;
    if (a.sd != nullptr) a.sd[tb + j] = baseline_delay(a, tb, b);
    a.perm[tb + j] = b;
    if (j < s_val) vm = fmax(vm, fabs(v));        // usable entries sort first
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) vm = fmax(vm, __shfl_xor(vm, o));
  if (threadIdx.x % WAVE == 0) s_vm[threadIdx.x / WAVE] = vm;
  __syncthreads();
  if (threadIdx.x == 0) {
    a.n_unflagged[t] = s_unf;
    a.n_valid[t] = s_val;
    if (a.vmax != nullptr) {
      double m = 0.0;
      for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) m = fmax(m, s_vm[w]);
      a.vmax[t] = m;
    }
  }
  if constexpr (BOUNDS) {
    const double s = cells_per_metre(a.freq[0], a.ndx);
    const int H = a.N / 2;
    auto ucol = [&](int j) -> int {
      double u, v;
      plane_uv(a, tb + si[j], u, v);                          // the u of sorted position j
      const double x = rint(u * s);
      return (int)fmin(fmax(x, (double)-H), (double)H);
    };
    image_bounds(ucol, s_val, a.N, a.kw, a.bnd + (size_t)t * (a.N + 2), a.ncz + t);
  }
}

// Merge neighbouring sorted runs of width w: each element's output position
// is its rank in its own run plus the number of smaller elements in the other
// run (binary search). All (key, index) pairs are distinct.
__global__ void __launch_bounds__(256) k_merge(SortArgs a, int w, int src) {
  const int t = a.t0 + blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.B) return;
  const size_t tb = (size_t)t * a.B;
  const unsigned long long* K = a.key[src] + tb;
  const int* I = a.idx[src] + tb;
  const int pb = (e / (2 * w)) * (2 * w);
  const int lend = min(pb + w, a.B);
  const int rend = min(pb + 2 * w, a.B);
  const unsigned long long mk = K[e];
  const int mi = I[e];
  const bool left = e < lend;
  int lo = left ? lend : pb, hi = left ? rend : lend;
  const int own = left ? e - pb : e - lend;
  while (lo < hi) {  // count of elements of the other run that are smaller
    const int mid = (lo + hi) >> 1;
    const unsigned long long km = K[mid];
    const bool less = km < mk || (km == mk && I[mid] < mi);
    if (less) lo = mid + 1; else hi = mid;
  }
  const int other = left ? lo - lend : lo - pb;
  const int out = pb + own + other;
  a.key[src ^ 1][tb + out] = mk;
  a.idx[src ^ 1][tb + out] = mi;
}

__global__ void __launch_bounds__(256) k_sort_finish(SortArgs a, int src) {
  const int t = a.t0 + blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.B) return;
  const size_t tb = (size_t)t * a.B;
  const unsigned long long k = a.key[src][tb + j];
  const int b = a.idx[src][tb + j];
  double u, v;
  plane_uv(a, tb + b, u, v);
  a.su[tb + j] = u;
  a.sv[tb + j] = v;
  if (a.sd != nullptr) a.sd[tb + j] = baseline_delay(a, tb, b);
  a.perm[tb + j] = b;
  const bool valid = k != KEY_MAX;
  const bool next_invalid = (j + 1 == a.B) || a.key[src][tb + j + 1] == KEY_MAX;
  if (valid && next_invalid) a.n_valid[t] = j + 1;
}

// ============================================================== cell bounds
// largest number of coefficients of the Kaiser-Bessel weight's polynomial (see kb_weight)
constexpr int KB_POLY_TERMS = 25;

struct ImgArgs {
  int T, C, B, N, M, weighting, norm, vis_type;
  double ndx;                   // fl(N * dx)
  const void* vis;              // [T][C][B] c64 or [T][C][B][2] f16/bf16
  const float* vis_scale;       // [C]
  const double* freq;           // [C]
  const int* ant1;              // [B]
  const int* ant2;              // [B]
  const float2* gains;          // [A] or null
  const double* su;             // [T][B]
  const double* sv;             // [T][B]
  const int* perm;              // [T][B]
  const double* sd;             // [T][B] sorted geometric delays (metres) or null: no rotation
  const int* n_valid;           // [T]
  const int* n_unflagged;       // [T]
  const double* vmax;           // [T] largest |v| (metres) of the usable baselines, or null
  int* bnd;                     // [T*C][N + 2]
  int* ncz;                     // [T*C] u-cell columns 0..ncz-1 may be non-empty; the rest are zero
  int ntiles;                   // column tiles per image of the current column kernel
  int* wpart;                   // [T*C][wstride] weight-sum partials, one per column tile
  int* kpart;                   // [T*C][wstride] kept-baseline partials, one per column tile
  int wstride;                  // partial slots per image (>= tiles of any producer kernel)
  int wtiles;                   // partial slots per image written by the current producer kernel
  int img0, nimg;               // this chunk: images [img0, img0 + nimg)
  float2* half;                 // [chunk][N/2][M] column-transformed half spectrum
  float2* grid;                 // MODE_GRID: [T*C][N][N]
  int* counts;                  // MODE_GRID: [T*C][N][N] or null
  float* images;                // [T*C][M][M]
  float* weight_sum;            // [T*C] or null
  int* n_dropped;               // [T*C] or null
  // adjoint
  const float* image_grad;      // [T*C][M][M]
  const float* wsum_in;         // [T*C] weight sums of the forward call, or null (count them)
  float2* gamma;                // [chunk][B] gradient w.r.t. V' per image
  float2* vis_grad;             // [T][C][B]
  float2* pacc;                 // [B] sum over images of gamma conj(V)
  float2* gain_grad;            // [A]
  float2* gfull;                // adjoint with a gridding kernel: [chunk][N/2][N] transformed columns
  int n_ant;
  // Kaiser-Bessel gridding kernel (kw = support in cells, 0 = nearest cell)
  int kw;
  float kbeta;                  // shape
  float kinv;                   // 1 / I0(kbeta)
  double kbeta_d;               // the shape in double (the correction is formed in double)
  double ktaper0_d;             // sinh(beta) / beta: the correction's value at 0 before normalising
  float k2w;                    // 2 / W
  int kpoly_on;                 // 1: weights from kpoly, 0: from cyl_bessel_i0f
  int kpoly_deg;                // degree D of that polynomial (<= KB_POLY_TERMS - 1)
  float kpoly[KB_POLY_TERMS];   // its coefficients in s = 1 - 2 (2d/W)^2, kpoly[k] of s^k, 0 above D
  // kernel gridding with uniform weighting: [chunk][B] per sorted entry, the
  // kept entries (direct and mirrored) at its nearest cell; null otherwise
  int* kdens;
};

// bnd[c + N/2] = first sorted position j with clamp(rint(u_j s)) >= c for
// c in [-N/2, N/2 + 1]; entry N + 1 is always n_valid. One workgroup per image.
// The clamped cell is non-decreasing along the sorted order (s > 0), so each
// bound is found either by one pass over the list, marking where the cell
// steps up, or - when the list is much longer than the N + 2 bounds - by a
// binary search per bound. Both give that first position. For s <= 0 or a
// non-finite s every bound still lies in [0, n_valid].
__global__ void __launch_bounds__(256) k_bounds(ImgArgs a) {
  const int img = blockIdx.x;
  const int t = img / a.C, ch = img - t * a.C;
  const double s = cells_per_metre(a.freq[ch], a.ndx);
  const int H = a.N / 2;
  const double* su = a.su + (size_t)t * a.B;
  auto ucol = [&](int j) -> int {
    const double x = rint(su[j] * s);
    return (int)fmin(fmax(x, (double)-H), (double)H);
  };
  image_bounds(ucol, a.n_valid[t], a.N, a.kw, a.bnd + (size_t)img * (a.N + 2), a.ncz + img);
}

// Largest |v| in metres over the usable baselines of each timestep (one
// workgroup per timestep). Since x -> rint(x |s|) is non-decreasing, every
// gridded row of an image at scale s satisfies |i_v| <= rint(vmax |s|), so the
// rows beyond that bound are known to be empty before the column is gridded.
__global__ void __launch_bounds__(256) k_vmax(const double* __restrict__ sv, const int* __restrict__ n_valid,
                                              int B, double* __restrict__ vmax) {
  __shared__ double red[256];
  const int t = blockIdx.x;
  const double* v = sv + (size_t)t * B;
  const int nv = n_valid[t];
  double m = 0.0;
  for (int j = threadIdx.x; j < nv; j += 256) m = fmax(m, fabs(v[j]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) vmax[t] = red[0];
}

// Zero band of an image's column transforms (see zero_band): the rows beyond
// rint(vmax |s|) are empty. Non-finite or out-of-range bounds give 0.
template <int N>
__device__ __forceinline__ int column_zero_band(const ImgArgs& a, int t, double s) {
  if (a.vmax == nullptr) return 0;
  const double vc = rint(a.vmax[t] * fabs(s));
  return (vc >= 0.0 && vc < (double)(N / 2)) ? zero_band(N, (int)vc + 1) : 0;
}

// Sum of the per-tile partials of one image (read by one wavefront; every
// slot below wtiles was written by exactly one workgroup of the producer).
__device__ __forceinline__ int sum_partials(const int* part, int img, int wstride, int wtiles, int lane) {
  int v = 0;
  for (int i = lane; i < wtiles; i += WAVE) v += part[(size_t)img * wstride + i];
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// The same for partials holding FP32 weight sums (kernel gridding).
__device__ __forceinline__ float sum_partials_f(const int* part, int img, int wstride, int wtiles, int lane) {
  float v = 0.f;
  for (int i = lane; i < wtiles; i += WAVE) v += __int_as_float(part[(size_t)img * wstride + i]);
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ============================================================== visibility load
// g[a1] conj(g[a2]); an antenna index outside [0, n_ant) gives a zero gain.
__device__ __forceinline__ float2 antenna_gain(const float2* g, int i, int n) {
  return (unsigned)i < (unsigned)n ? g[i] : make_float2(0.f, 0.f);
}
template <class A>
__device__ __forceinline__ float2 baseline_gain(const A& a, int b) {
  const float2 g1 = antenna_gain(a.gains, a.ant1[b], a.n_ant);
  const float2 g2 = antenna_gain(a.gains, a.ant2[b], a.n_ant);
  return cmul(g1, cconj(g2));
}
__device__ __forceinline__ float2 load_vis_raw(const ImgArgs& a, size_t off, int ch) {
  float2 v;
  if (a.vis_type == VT_C64) {
    v = static_cast<const float2*>(a.vis)[off];
  } else if (a.vis_type == VT_F16) {
    const __half2 h = static_cast<const __half2*>(a.vis)[off];
    v = __half22float2(h);
    const float sc = a.vis_scale[ch];
    v.x *= sc; v.y *= sc;
  } else {
    const unsigned int w = static_cast<const unsigned int*>(a.vis)[off];
    v.x = __uint_as_float(w << 16);
    v.y = __uint_as_float(w & 0xffff0000u);
    const float sc = a.vis_scale[ch];
    v.x *= sc; v.y *= sc;
  }
  return v;
}
__device__ __forceinline__ float2 load_vis(const ImgArgs& a, size_t off, int b, int ch) {
  float2 v;
  if (a.vis_type == VT_C64) {
    v = static_cast<const float2*>(a.vis)[off];
  } else if (a.vis_type == VT_F16) {
    const __half2 h = static_cast<const __half2*>(a.vis)[off];
    v = __half22float2(h);
    const float sc = a.vis_scale[ch];
    v.x *= sc; v.y *= sc;
  } else {
    const unsigned int w = static_cast<const unsigned int*>(a.vis)[off];
    v.x = __uint_as_float(w << 16);
    v.y = __uint_as_float(w & 0xffff0000u);
    const float sc = a.vis_scale[ch];
    v.x *= sc; v.y *= sc;
  }
  if (a.gains != nullptr) v = cmul(baseline_gain(a, b), v);
  return v;
}

// Geometric phase rotation of a visibility: V exp(+2 pi i d nu / c) for the
// delay d (metres) of its baseline. The phase in cycles is formed in double
// and reduced to [-1/2, 1/2] before the single-precision sine and cosine.
__device__ __forceinline__ float2 rotate_phase(float2 v, double d, double f) {
  const double cyc = d * (f / C_LIGHT);
  const float fr = (float)(cyc - rint(cyc));
  float sn, cs;
  sincospif(2.0f * fr, &sn, &cs);
  return make_float2(v.x * cs - v.y * sn, v.x * sn + v.y * cs);
}

// Grid the column's entries: sorted positions [dlo, dhi) add V' at row i_v,
// positions [clo, chi) (the mirror column) add conj(V') at row -i_v. Both
// ranges are walked as one list, GU x 64 entries per step: every step first
// issues the sorted-list loads of all its entries, then their visibility
// gathers, then the LDS adds, so a wavefront keeps GU times more loads in
// flight. Only this wavefront touches the column, so the LDS adds happen in a
// fixed order (steps in sequence; within a step, sub-steps in sequence and
// lanes in LDS order).
constexpr int GU = 2;

struct ColSpan {                 // the sorted entries of one u-cell column
  int dlo, dhi, clo, chi;        // direct range and mirror (conjugate) range
  __device__ int nd() const { return dhi - dlo; }
  __device__ int total() const { return (dhi - dlo) + (chi - clo); }
};

struct EntryStep {               // GU x 64 entries in registers
  double sv[GU];
  double dl[GU];                 // geometric delay (phase rotation only)
  int bl[GU];
  int row[GU];
  float2 val[GU];
  bool ok[GU], cj[GU];
};

// phase 1: sorted-list loads (v in metres and baseline index) of the step at i0
// (ROT: and the geometric delays for the phase rotation)
template <bool ROT>
__device__ __forceinline__ void step_keys(const ImgArgs& a, const ColSpan& c, int i0, int t, int lane,
                                          EntryStep& e) {
  const size_t tb = (size_t)t * a.B;
  const int nd = c.nd(), total = c.total();
#pragma unroll
  for (int u = 0; u < GU; ++u) {
    const int i = i0 + u * WAVE + lane;
    e.ok[u] = i < total;
    e.cj[u] = i >= nd;
    const int j = e.cj[u] ? c.clo + (i - nd) : c.dlo + i;
    e.sv[u] = e.ok[u] ? a.sv[tb + j] : 0.0;
    e.bl[u] = e.ok[u] ? a.perm[tb + j] : 0;
    if (ROT) e.dl[u] = e.ok[u] ? a.sd[tb + j] : 0.0;
  }
}

// phase 2: cell rows (FP64) and the visibility gathers of the kept entries
template <int N, bool ROT>
__device__ __forceinline__ void step_gather(const ImgArgs& a, int t, int ch, double s, EntryStep& e) {
  const size_t vb = ((size_t)t * a.C + ch) * a.B;
#pragma unroll
  for (int u = 0; u < GU; ++u) {
    const double iv = rint(e.sv[u] * s);
    e.ok[u] = e.ok[u] && fabs(iv) < (double)(N / 2);
    int r = (int)iv;
    if (e.cj[u]) r = -r;
    e.row[u] = r < 0 ? r + N : r;
    e.val[u] = e.ok[u] ? load_vis(a, vb + e.bl[u], e.bl[u], ch) : make_float2(0.f, 0.f);
    if (ROT) e.val[u] = rotate_phase(e.val[u], e.dl[u], a.freq[ch]);
  }
}

// ------------------------------------------------------ LDS accumulation
// LDS floating-point atomic adds are slow on gfx950: measured at about 190
// CU cycles per wave64 ds_add_f32, against about 5 for an integer atomic or a
// plain read-modify-write. The column being gridded is LDS that only its own
// wavefront writes, so the adds are done as plain read-modify-writes, and
// lanes that would touch the same element take turns: each turn, every
// pending lane posts a tag (turn * 64 + 64 - lane) to claim slot key mod 64
// with an integer atomic max, and the lane whose tag survives adds its value
// (and, with counts, 1 to its count). Lanes whose elements coincide share a
// slot, so no two lanes of one turn touch one element; of the lanes sharing
// a slot the lowest goes first, so each element receives its adds in lane
// order, step after step: the order of the sorted list, whatever the
// grouping into steps. Tags grow with the wavefront's turn counter, so the
// claim slots never need clearing after their initial zeroing.
constexpr int CLAIM_SLOTS = 64;

struct Claim {
  unsigned* slot;                // CLAIM_SLOTS words of this wavefront's LDS
  unsigned turn;                 // wave-uniform
};

// Zeroes this wavefront's claim slots (the caller's next wave_sync publishes them).
__device__ __forceinline__ Claim claim_init(unsigned* slots, int lane) {
  if (lane < CLAIM_SLOTS) slots[lane] = 0u;
  return Claim{slots, 0u};
}

// dst[idx] += v (and cnt[cidx] += 1 with COUNT) for every active lane; lanes
// with equal idx must pass equal key.
template <bool COUNT>
__device__ __forceinline__ void wave_add(float2* dst, int idx, int* cnt, int cidx, int key, float2 v, bool active,
                                         Claim& cl, int lane) {
  bool pending = active;
  while (__ballot(pending) != 0) {
    const unsigned tag = cl.turn * CLAIM_SLOTS + (unsigned)(CLAIM_SLOTS - lane);
    unsigned* slot = cl.slot + (key & (CLAIM_SLOTS - 1));
    if (pending) __hip_atomic_fetch_max(slot, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    wave_sync();
    if (pending && *slot == tag) {
      const float2 d = dst[idx];
      dst[idx] = make_float2(d.x + v.x, d.y + v.y);
      if (COUNT) cnt[cidx] += 1;
      pending = false;
    }
    wave_sync();
    ++cl.turn;
  }
}

// phase 3: the LDS adds; kd / kc count the kept direct / conjugate entries
template <bool COUNT>
__device__ __forceinline__ void step_add(const EntryStep& e, float2* buf, int* cnt, int& kd, int& kc, Claim& cl,
                                         int lane) {
#pragma unroll
  for (int u = 0; u < GU; ++u) {
    float2 v = e.val[u];
    if (e.cj[u]) v.y = -v.y;
    wave_add<COUNT>(buf, pad(e.row[u]), cnt, e.row[u], e.row[u], v, e.ok[u], cl, lane);
    kd += __popcll(__ballot(e.ok[u] && !e.cj[u]));
    kc += __popcll(__ballot(e.ok[u] && e.cj[u]));
  }
}

// All steps of a column from step i0 on; returns the kept direct and
// conjugate entries (added to kd / kc). The phase-rotated form is a separate
// copy of the loop, so the plain one carries none of its work.
template <int N, bool COUNT, bool ROT>
__device__ __forceinline__ void grid_steps_t(const ImgArgs& a, const ColSpan& c, int i0, float2* buf, int* cnt,
                                             int t, int ch, double s, int lane, int& kd, int& kc, Claim& cl) {
  const int total = c.total();
  for (; i0 < total; i0 += GU * WAVE) {
    EntryStep e;
    step_keys<ROT>(a, c, i0, t, lane, e);
    step_gather<N, ROT>(a, t, ch, s, e);
    step_add<COUNT>(e, buf, cnt, kd, kc, cl, lane);
  }
}
template <int N, bool COUNT>
__device__ __forceinline__ void grid_steps(const ImgArgs& a, const ColSpan& c, int i0, float2* buf, int* cnt,
                                           int t, int ch, double s, int lane, int& kd, int& kc, Claim& cl) {
  if (a.sd != nullptr) grid_steps_t<N, COUNT, true>(a, c, i0, buf, cnt, t, ch, s, lane, kd, kc, cl);
  else grid_steps_t<N, COUNT, false>(a, c, i0, buf, cnt, t, ch, s, lane, kd, kc, cl);
}

// ------------------------------------------------------------- kernel gridding
// Kaiser-Bessel weight C(d) = I0(beta sqrt(1 - (2d/W)^2)) / I0(beta), |d| <= W/2.
// I0(beta sqrt(w)) is an entire function of w = 1 - (2d/W)^2 in [0, 1], so a
// polynomial of low degree in s = 2w - 1 in [-1, 1] matches it closely: the
// host interpolates C at Chebyshev points of s and keeps the shortest
// truncation whose dropped Chebyshev terms sum below 2e-8 (degree 11 at
// W = 6 with the default shape). Its coefficients in powers of s are the
// function's expansion around w = 1/2, all positive and summing to about 1,
// so Horner's rule in FP32 loses no accuracy to cancellation. The degree
// picks one of three fixed-length forms (12, 16 or 25 coefficients, zeros
// above the degree), so that the coefficients stay in scalar registers and
// the loops unroll. Beyond 25 coefficients (beta above about 70) the weights
// come from cyl_bessel_i0f.
template <int TERMS>
__device__ __forceinline__ float kb_horner(float s, const float* c) {
  float p = c[TERMS - 1];
#pragma unroll
  for (int k = TERMS - 2; k >= 0; --k) p = fmaf(p, s, c[k]);
  return p;
}

__device__ __forceinline__ float kb_weight(float d, const ImgArgs& a) {
  const float t = d * a.k2w;
  if (a.kpoly_on) {
    const float s = fmaxf(-1.0f, fmaf(-2.0f * t, t, 1.0f));
    if (a.kpoly_deg < 12) return kb_horner<12>(s, a.kpoly);
    if (a.kpoly_deg < 16) return kb_horner<16>(s, a.kpoly);
    return kb_horner<KB_POLY_TERMS>(s, a.kpoly);
  }
  return cyl_bessel_i0f(a.kbeta * sqrtf(fmaxf(0.0f, fmaf(-t, t, 1.0f)))) * a.kinv;
}

// Reciprocal of the correction at xi cycles per cell, 1 / c(xi) with
// c(xi) = [sinh(z)/z] / [sinh(beta)/beta], z = sqrt(beta^2 - (pi W xi)^2)
// (sin(|z|)/|z| beyond pi W |xi| = beta). Formed in double: near a zero of
// c (small beta, pixels near the edge of a full-field image) FP32 would lose
// most of its digits in z.
__device__ __forceinline__ float kb_inv_taper(double xi, const ImgArgs& a) {
  const double b = a.kbeta_d;
  const double x = 3.141592653589793 * (double)a.kw * xi;
  const double z2 = b * b - x * x;
  double f = 1.0;
  if (z2 > 0.0) { const double z = sqrt(z2); f = sinh(z) / z; }
  else if (z2 < 0.0) { const double z = sqrt(-z2); f = sin(z) / z; }
  return (float)(a.ktaper0_d / f);
}

// Adds w[k] v to rows j0 + k, k < nrow, of this column for every active
// lane, with one claim per entry instead of one per row: lanes with the same
// first row j0 take turns, lowest lane first (the claim protocol of
// wave_add, keyed on j0), and lanes with different j0 never reach the same
// row at the same k, so a turn adds all of its lanes' rows in sequence over
// k. Each element receives its adds in a fixed order: step, turn, k.
template <int N, bool COUNT, int KMAX>
__device__ __forceinline__ void kb_add_rows(float2* buf, int* cnt, int j0, int nrow, const float (&w)[KMAX + 1],
                                            float2 v, bool active, int kw, Claim& cl, int lane) {
  bool pending = active;
  while (__ballot(pending) != 0) {
    const unsigned tag = cl.turn * CLAIM_SLOTS + (unsigned)(CLAIM_SLOTS - lane);
    unsigned* slot = cl.slot + (j0 & (CLAIM_SLOTS - 1));
    if (pending) __hip_atomic_fetch_max(slot, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    wave_sync();
    const bool go = pending && *slot == tag;
#pragma unroll
    for (int k = 0; k <= KMAX; ++k) {
      if (k > kw) break;
      if (go && k < nrow) {
        const int r = j0 + k < 0 ? j0 + k + N : j0 + k;
        const float2 d = buf[pad(r)];
        buf[pad(r)] = make_float2(d.x + w[k] * v.x, d.y + w[k] * v.y);
        if (COUNT) cnt[r] += 1;
      }
      wave_sync();
    }
    pending = pending && !go;
    ++cl.turn;
  }
}

// Kernel gridding of u-cell column c: the span holds the sorted entries whose
// nearest column c' lies within floor(W/2 + 1/2) of c (direct) and of -c
// (mirror): |c - x_u| <= W/2 and |x_u - c'| <= 1/2 bound |c - c'|. Each
// direct entry at exact position x adds C(c - x_u) C(j - x_v) V' to the rows j
// of its footprint, each mirror entry (its conjugate, at -x) adds
// C(c + x_u) C(j + x_v) conj(V'). One entry per lane per step; its W + 1
// row weights are formed first (KMAX >= W bounds them at compile time), then
// kb_add_rows adds them. kd / kc count kept entries whose nearest column is
// c (each baseline once); wsum collects this lane's weights.
template <int N, bool COUNT, int KMAX>
__device__ __forceinline__ void grid_steps_kb(const ImgArgs& a, const ColSpan& sp, int c, float2* buf,
                                              int* cnt, int t, int ch, double s, int lane, int& kd,
                                              int& kc, float& wsum, Claim& cl, const int* dens) {
  constexpr int H = N / 2;
  const size_t tb = (size_t)t * a.B;
  const size_t vb = ((size_t)t * a.C + ch) * a.B;
  const double hw = 0.5 * a.kw;
  const int kw = a.kw;
  const int nd = sp.nd(), total = sp.total();
  for (int i0 = 0; i0 < total; i0 += WAVE) {
    const int i = i0 + lane;
    bool ok = i < total;
    const bool cj = i >= nd;
    const int j = cj ? sp.clo + (i - nd) : sp.dlo + i;
    double xu = 0.0, xv = 0.0;
    int b = 0;
    if (ok) {
      xu = a.su[tb + j] * s;
      xv = a.sv[tb + j] * s;
      b = a.perm[tb + j];
    }
    // kept iff the whole footprint lies inside |i| < N/2 on both axes
    ok = ok && ceil(xu - hw) > (double)-H && floor(xu + hw) < (double)H &&
         ceil(xv - hw) > (double)-H && floor(xv + hw) < (double)H;
    if (cj) { xu = -xu; xv = -xv; }
    const bool home = ok && rint(xu) == (double)c;
    kd += __popcll(__ballot(home && !cj));
    kc += __popcll(__ballot(home && cj));
    const double du = (double)c - xu;
    const bool in = ok && fabs(du) <= hw;
    float2 v = make_float2(0.f, 0.f);
    float wu = 0.f;
    int j0 = 0, nrow = 0;
    if (in) {
      v = load_vis(a, vb + b, b, ch);
      if (a.sd != nullptr) v = rotate_phase(v, a.sd[tb + j], a.freq[ch]);
      if (cj) v.y = -v.y;
      wu = kb_weight((float)du, a);
      // uniform weighting: the baseline's share of its nearest cell
      if (dens != nullptr) wu = wu / (float)dens[j];
      j0 = (int)ceil(xv - hw);
      nrow = (int)floor(xv + hw) - j0 + 1;       // W or W + 1 rows
    }
    float w[KMAX + 1];
#pragma unroll
    for (int k = 0; k <= KMAX; ++k) {
      w[k] = 0.f;
      if (k > kw) break;
      if (k < nrow) {
        w[k] = wu * kb_weight((float)((double)(j0 + k) - xv), a);
        wsum += w[k];
      }
    }
    kb_add_rows<N, COUNT, KMAX>(buf, cnt, j0, nrow, w, v, in, kw, cl, lane);
  }
}

// u-cell columns (one wavefront each) per workgroup of the column kernels
__host__ __device__ constexpr int cols_per_wg(int n) { return n <= 1024 ? 8 : (n <= 2048 ? 4 : 2); }

// Uniform weighting with kernel gridding: the weight of a kept baseline is
// 1 / n, n the number of kept entries - direct and mirrored - whose nearest
// cell is the baseline's own. This pass writes n for every kept entry of each
// image of the chunk into a.kdens[li][j] (j its sorted position). One
// workgroup per image, DENS_WAVES wavefronts; a wavefront takes signed
// u-cell columns c in turn, counts the kept direct entries of column c and
// the mirrored entries of column -c per row in an LDS row array with integer
// atomics, reads the counts back for the direct entries, and clears only the
// rows it touched. Kept entries have |nearest cell| <= N/2 - 1 on both axes,
// so the columns -N/2+1 .. N/2-1 hold all of them.
constexpr int DENS_WAVES = 4;

template <int N>
__global__ void __launch_bounds__(DENS_WAVES * WAVE) k_kb_density(ImgArgs a) {
  extern __shared__ int dens_lds[];
  constexpr int H = N / 2;
  const int li = blockIdx.x;
  if (li >= a.nimg) return;
  const int img = a.img0 + li;
  const int t = img / a.C, ch = img - t * a.C;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), lane = threadIdx.x % WAVE;
  int* rc = dens_lds + wave * N;                     // rc[iv + H]: entries in row iv of the column
  for (int r = lane; r < N; r += WAVE) rc[r] = 0;
  wave_sync();
  const int* bnd = a.bnd + (size_t)img * (N + 2);
  const double s = cells_per_metre(a.freq[ch], a.ndx);
  const double hw = 0.5 * a.kw;
  const double* su = a.su + (size_t)t * a.B;
  const double* sv = a.sv + (size_t)t * a.B;
  int* out = a.kdens + (size_t)li * a.B;
  // nearest row of entry j (mirrored with mj), or N when it is not kept
  auto row_of = [&](int j, bool mj) -> int {
    const double xu = su[j] * s, xv = sv[j] * s;
    const bool kept = ceil(xu - hw) > (double)-H && floor(xu + hw) < (double)H &&
                      ceil(xv - hw) > (double)-H && floor(xv + hw) < (double)H;
    if (!kept) return N;
    const int r = (int)rint(xv);
    return mj ? -r : r;
  };
  // 64 columns per round: lane l fetches the ranges of column c0 + l
  for (int c0 = -H + 1 + wave * WAVE; c0 < H; c0 += DENS_WAVES * WAVE) {
    const int cl_ = c0 + lane;
    int d0 = 0, d1 = 0, m0 = 0, m1 = 0;
    if (cl_ < H) {
      d0 = bnd[cl_ + H]; d1 = bnd[cl_ + 1 + H];
      m0 = bnd[-cl_ + H]; m1 = bnd[-cl_ + 1 + H];
    }
    unsigned long long busy = __ballot(d1 > d0);     // columns with direct entries
    while (busy != 0ull) {
      const int k = __builtin_ctzll(busy);
      busy &= busy - 1ull;
      const int dlo = __shfl(d0, k), dhi = __shfl(d1, k), mlo = __shfl(m0, k), mhi = __shfl(m1, k);
      const int nd = dhi - dlo, total = nd + (mhi - mlo);
      for (int i = lane; i < total; i += WAVE) {
        const bool mj = i >= nd;
        const int r = row_of(mj ? mlo + (i - nd) : dlo + i, mj);
        if (r != N) atomicAdd(&rc[r + H], 1);
      }
      wave_sync();
      for (int i = lane; i < nd; i += WAVE) {
        const int r = row_of(dlo + i, false);
        if (r != N) out[dlo + i] = rc[r + H];
      }
      wave_sync();
      for (int i = lane; i < total; i += WAVE) {
        const bool mj = i >= nd;
        const int r = row_of(mj ? mlo + (i - nd) : dlo + i, mj);
        if (r != N) rc[r + H] = 0;
      }
      wave_sync();
    }
  }
}

// Twiddle table staged in LDS (one copy per workgroup) where it fits beside
// the transform buffers without lowering occupancy.
template <int N>
struct TwLds { static constexpr bool ON = N <= 1024; };

// CL: copy only the compact table (tw_entries_compact), for transforms that
// form the last stage's higher twiddle powers in registers.
template <int N, bool CL = false>
__device__ __forceinline__ const float2* stage_twiddles(float2* lds_tw) {
  if constexpr (TwLds<N>::ON) {
    const float2* g = TwTable<N>::stages();
    constexpr int NTW = CL ? tw_entries_compact(N) : tw_entries(N);
    for (int i = threadIdx.x; i < NTW; i += blockDim.x) lds_tw[i] = g[i];
    return lds_tw;      // visible after the caller's next __syncthreads
  } else {
    return TwTable<N>::stages();
  }
}

template <int N, int CPW_ = cols_per_wg(N)>
struct Cols {
  static constexpr int STRIDE = padded_len(N);                // complex per column buffer
  static constexpr int CPW = CPW_;
  static constexpr int THREADS = CPW * WAVE;
  static constexpr int TW = TwLds<N>::ON ? tw_entries(N) : 0; // complex twiddles in LDS
  static size_t lds_bytes(bool counts) {
    return (size_t)(CPW * STRIDE + TW) * sizeof(float2) + (counts ? (size_t)CPW * N * sizeof(int) : 0);
  }
  // the gridding kernel adds every wavefront's claim slots after that
  static size_t grid_lds_bytes(bool counts) { return lds_bytes(counts) + (size_t)CPW * CLAIM_SLOTS * sizeof(unsigned); }
};

// One workgroup = CPW consecutive u-cell columns of one image; one wavefront
// per column. MODE_IMAGE: columns 0..N/2-1 (the half spectrum), transform
// along v, rows of the cutout written to `half`. MODE_GRID: all N columns,
// weighted grid and counts written out.
// The 1D grid is laid out so that all column tiles of an image share one XCD
// (workgroup L runs on XCD L mod 8): the image's visibility row and the
// timestep's sorted lists are then fetched into a single L2.
// KB: Kaiser-Bessel kernel gridding instead of nearest cell; uniform weighting
// then comes from the per-entry cell occupancy of k_kb_density (a.kdens), so
// UNI (the nearest-cell division by counts) stays off.
// KMAX: largest support W the kernel gridding form handles (rows k = 0 .. W).
template <int N, int MODE, bool UNI, int CPW = cols_per_wg(N), bool KB = false, int KMAX = 16>
__global__ void __launch_bounds__((Cols<N, CPW>::THREADS)) k_grid_cols(ImgArgs a) {
  static_assert(!(KB && UNI), "kernel gridding weights uniformly through a.kdens");
  extern __shared__ float4 lds_raw[];
  __shared__ int red[2 * CPW];
  using C_ = Cols<N, CPW>;
  constexpr int H = N / 2;
  constexpr bool CNT = UNI || MODE == MODE_GRID;
  const int L = blockIdx.x;
  const int r8 = L >> 3;
  const int li = (r8 / a.ntiles) * 8 + (L & 7);
  const int tile = r8 % a.ntiles;
  if (li >= a.nimg) return;                          // padding of the last group of 8 images
  float2* lds = reinterpret_cast<float2*>(lds_raw);
  float2* ltw = lds + CPW * C_::STRIDE;
  int* lcnt = reinterpret_cast<int*>(ltw + C_::TW);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), lane = threadIdx.x % WAVE;
  const int img = a.img0 + li;
  const int t = img / a.C, ch = img - t * a.C;
  const int c0 = tile * CPW;
  const int ncols = MODE == MODE_IMAGE ? min(H, a.ncz[img]) : N;
  if (c0 >= ncols) {                                 // the whole tile is empty
    if (threadIdx.x == 0) {
      a.wpart[(size_t)img * a.wstride + tile] = 0;
      a.kpart[(size_t)img * a.wstride + tile] = 0;
    }
    return;
  }
  const int col = c0 + wave;                        // MODE_IMAGE: 0..H-1, MODE_GRID: 0..N-1
  const bool active = col < ncols;
  const int cs = MODE == MODE_IMAGE ? col : (col < H ? col : col - N);  // signed u cell
  float2* buf = lds + wave * C_::STRIDE;
  int* cnt = CNT ? lcnt + wave * N : nullptr;
  const double s = cells_per_metre(a.freq[ch], a.ndx);
  const float2* tw = MODE == MODE_IMAGE ? stage_twiddles<N>(ltw) : nullptr;

  for (int r = lane; r < C_::STRIDE; r += WAVE) buf[r] = make_float2(0.f, 0.f);
  if (CNT)
    for (int r = lane; r < N; r += WAVE) cnt[r] = 0;
  unsigned* lclaim = reinterpret_cast<unsigned*>(lcnt + (CNT ? CPW * N : 0));
  Claim cl = claim_init(lclaim + wave * CLAIM_SLOTS, lane);
  wave_sync();

  int kept_b = 0, wcontrib = 0;
  if (KB && active && cs != H && cs != -H) {
    const int* bnd = a.bnd + (size_t)img * (N + 2);
    const int hk = (a.kw + 1) / 2;                  // see grid_steps_kb
    auto at = [&](int c) { return bnd[min(max(c, -H), H + 1) + H]; };
    const ColSpan span{at(cs - hk), at(cs + hk + 1), at(-cs - hk), at(-cs + hk + 1)};
    int kd = 0, kc = 0;
    float ws = 0.f;
    const int* dens = a.kdens != nullptr ? a.kdens + (size_t)li * a.B : nullptr;
    grid_steps_kb<N, CNT, KMAX>(a, span, cs, buf, cnt, t, ch, s, lane, kd, kc, ws, cl, dens);
    wave_sync();
    kept_b = kd + ((MODE == MODE_IMAGE && cs > 0) ? kc : 0);
    for (int o = WAVE / 2; o > 0; o >>= 1) ws += __shfl_xor(ws, o);
    wcontrib = __float_as_int(((MODE == MODE_IMAGE && cs > 0) ? 2.0f : 1.0f) * ws);
  } else if (!KB && active && cs != H && cs != -H) {
    const int* bnd = a.bnd + (size_t)img * (N + 2);
    const ColSpan span{bnd[cs + H], bnd[cs + 1 + H], bnd[-cs + H], bnd[-cs + 1 + H]};
    int kd = 0, kc = 0;
    grid_steps<N, CNT>(a, span, 0, buf, cnt, t, ch, s, lane, kd, kc, cl);
    wave_sync();
    // baselines counted once: the direct entry of every cell column, plus the
    // conjugate entries of columns whose mirror the image path never visits
    kept_b = kd + ((MODE == MODE_IMAGE && cs > 0) ? kc : 0);
    const int mult = (MODE == MODE_IMAGE && cs > 0) ? 2 : 1;
    if (UNI) {
      int occ = 0;
      for (int r = lane; r < N; r += WAVE) {
        const int n = cnt[r];
        if (n > 0) {
          float2 v = buf[pad(r)];
          v.x = v.x / (float)n;
          v.y = v.y / (float)n;
          buf[pad(r)] = v;
          ++occ;
        }
      }
      for (int o = WAVE / 2; o > 0; o >>= 1) occ += __shfl_xor(occ, o);
      wcontrib = mult * occ;
      wave_sync();
    } else {
      wcontrib = mult * (kd + kc);
    }
  }
  if (lane == 0) { red[wave] = wcontrib; red[CPW + wave] = kept_b; }
  __syncthreads();                                   // also publishes the LDS twiddles
  if (threadIdx.x == 0) {
    int ws = 0, ks = 0;
    float wf = 0.f;                                  // kernel gridding: FP32 weight sums
    for (int i = 0; i < CPW; ++i) {
      ws += red[i];
      wf += __int_as_float(red[i]);
      ks += red[CPW + i];
    }
    a.wpart[(size_t)img * a.wstride + tile] = KB ? __float_as_int(wf) : ws;
    a.kpart[(size_t)img * a.wstride + tile] = ks;
  }

  if (MODE == MODE_IMAGE) {
    if (active) {
      // rows of the cutout straight from the last stage: output row m holds
      // v-frequency q = (m - M/2) mod N
      float2* dst = a.half + ((size_t)li * H + col) * a.M;
      const int hm = a.M / 2;
      wave_fft_emit<N, +1>(buf, lane, tw, [&](auto qb, float2 v) {
        cutout_block<N, decltype(qb)::value>(lane, hm, [&](unsigned m) { store_at(dst, m, v); });
      });
    }
  } else {
    // write the CPW-column tile row by row (CPW consecutive cells per row)
    float2* g = a.grid + (size_t)img * N * N;
    int* gc = a.counts ? a.counts + (size_t)img * N * N : nullptr;
    for (int e = threadIdx.x; e < N * CPW; e += blockDim.x) {
      const int r = e / CPW, w = e % CPW;
      if (c0 + w < N) {
        g[(size_t)r * N + c0 + w] = lds[w * C_::STRIDE + pad(r)];
        if (gc) gc[(size_t)r * N + c0 + w] = lcnt[w * N + r];
      }
    }
  }
}

// ------------------------------------------- column pass, half-length LDS
// The image-mode column kernel (nearest cell) with every LDS exchange of the
// column through N/2 points: the rows below N/2 are gridded (and, with
// uniform weighting, divided by their counts) and handed to the first
// stage's registers, then the rows above, and the stages exchange in two
// rounds (wave_fft_half_emit). Each row receives the same adds in the same
// order as in the full-buffer kernel.
template <int N, int CPW, bool UNI>
struct ColsHalf {
  static constexpr int STRIDE = padded_len(N / 2);
  static constexpr int THREADS = CPW * WAVE;
  // compact twiddle table in LDS: at N = 1024 and 4 columns per workgroup
  // 22.5 KB instead of 26.6 KB, so seven workgroups share a CU instead of six
  static constexpr bool CL = TwLds<N>::ON && compact_last(N);
  static constexpr int TW = TwLds<N>::ON ? tw_entries_compact(N) : 0;
  static constexpr size_t LDS = (size_t)(CPW * STRIDE + TW) * sizeof(float2) +
                                (UNI ? (size_t)CPW * (N / 2) * sizeof(int) : 0) +
                                (size_t)CPW * CLAIM_SLOTS * sizeof(unsigned);
};

// LDS adds (and counts) of the kept entries of a step whose row lies in half HF
template <int N, int HF, bool COUNT>
__device__ __forceinline__ void step_add_half(const EntryStep& e, float2* hbuf, int* hcnt, Claim& cl, int lane) {
#pragma unroll
  for (int u = 0; u < GU; ++u) {
    const bool act = e.ok[u] && (e.row[u] >= N / 2) == (HF == 1);
    float2 v = e.val[u];
    if (e.cj[u]) v.y = -v.y;
    const int r = e.row[u] - HF * (N / 2);
    wave_add<COUNT>(hbuf, pad(r), hcnt, r, r, v, act, cl, lane);
  }
}

__device__ __forceinline__ void step_count(const EntryStep& e, int& kd, int& kc) {
#pragma unroll
  for (int u = 0; u < GU; ++u) {
    kd += __popcll(__ballot(e.ok[u] && !e.cj[u]));
    kc += __popcll(__ballot(e.ok[u] && e.cj[u]));
  }
}

template <int N, bool UNI>
__device__ __forceinline__ void zero_half(float2* hbuf, int* hcnt, int lane) {
  for (int r = lane; r < padded_len(N / 2); r += WAVE) hbuf[r] = make_float2(0.f, 0.f);
  if (UNI)
    for (int r = lane; r < N / 2; r += WAVE) hcnt[r] = 0;
}

// Uniform weighting of one half: every occupied cell divided by its count;
// returns this lane's number of occupied cells.
template <int N>
__device__ __forceinline__ int uniform_half(float2* hbuf, const int* hcnt, int lane) {
  int occ = 0;
  for (int r = lane; r < N / 2; r += WAVE) {
    const int n = hcnt[r];
    if (n > 0) {
      float2 v = hbuf[pad(r)];
      v.x = v.x / (float)n;
      v.y = v.y / (float)n;
      hbuf[pad(r)] = v;
      ++occ;
    }
  }
  return occ;
}

// Grids one column in two halves and loads the first stage's inputs. A
// column of at most GU x 64 entries (the usual case) keeps its one step of
// entries in registers for both halves; longer columns load them again.
// occ: this lane's occupied cells (uniform weighting).
template <int N, bool ROT, bool UNI, int ZB>
__device__ __forceinline__ void grid_col_half(const ImgArgs& a, const ColSpan& c, float2* hbuf, int* hcnt,
                                              HalfIn<N>& in, int t, int ch, double s, int lane, int& kd,
                                              int& kc, int& occ, Claim& cl) {
  constexpr int R0 = HalfIn<N>::R;
  const int total = c.total();
  const bool one = total <= GU * WAVE;
  EntryStep e;
  zero_half<N, UNI>(hbuf, hcnt, lane);
  wave_sync();
  if (one) {
    if (total > 0) {
      step_keys<ROT>(a, c, 0, t, lane, e);
      step_gather<N, ROT>(a, t, ch, s, e);
      step_add_half<N, 0, UNI>(e, hbuf, hcnt, cl, lane);
      step_count(e, kd, kc);
    }
  } else {
    for (int i0 = 0; i0 < total; i0 += GU * WAVE) {
      EntryStep f;
      step_keys<ROT>(a, c, i0, t, lane, f);
      step_gather<N, ROT>(a, t, ch, s, f);
      step_add_half<N, 0, UNI>(f, hbuf, hcnt, cl, lane);
      step_count(f, kd, kc);
    }
  }
  wave_sync();
  if (UNI) {
    occ += uniform_half<N>(hbuf, hcnt, lane);
    wave_sync();
  }
  half_read<N, R0, 0, ZB>(hbuf, lane, in.v);
  wave_sync();
  zero_half<N, UNI>(hbuf, hcnt, lane);
  wave_sync();
  if (one) {
    if (total > 0) step_add_half<N, 1, UNI>(e, hbuf, hcnt, cl, lane);
  } else {
    for (int i0 = 0; i0 < total; i0 += GU * WAVE) {
      EntryStep f;
      step_keys<ROT>(a, c, i0, t, lane, f);
      step_gather<N, ROT>(a, t, ch, s, f);
      step_add_half<N, 1, UNI>(f, hbuf, hcnt, cl, lane);
    }
  }
  wave_sync();
  if (UNI) {
    occ += uniform_half<N>(hbuf, hcnt, lane);
    wave_sync();
  }
  half_read<N, R0, 1, ZB>(hbuf, lane, in.v);
  wave_sync();
}

// Same tiling, XCD mapping and outputs as k_grid_cols<N, MODE_IMAGE, UNI, CPW>.
// HMC > 0: the cutout half-width M/2 fixed at compile time (M = N/2 takes
// HMC = N/4), so that the last stage computes only the outputs it stores and
// the cutout tests vanish; 0: read from the arguments.
template <int N, int CPW, bool UNI, int HMC = 0>
__global__ void __launch_bounds__((ColsHalf<N, CPW, UNI>::THREADS)) k_grid_cols_half(ImgArgs a) {
  extern __shared__ float4 lds_raw[];
  using C_ = ColsHalf<N, CPW, UNI>;
  constexpr int H = N / 2;
  const int L = blockIdx.x;
  const int r8 = L >> 3;
  const int li = (r8 / a.ntiles) * 8 + (L & 7);
  const int tile = r8 % a.ntiles;
  if (li >= a.nimg) return;                          // padding of the last group of 8 images
  float2* lds = reinterpret_cast<float2*>(lds_raw);
  float2* ltw = lds + CPW * C_::STRIDE;
  int* lcnt = reinterpret_cast<int*>(ltw + C_::TW);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), lane = threadIdx.x % WAVE;
  const int img = a.img0 + li;
  const int t = img / a.C, ch = img - t * a.C;
  const int c0 = tile * CPW;
  const int ncols = min(H, a.ncz[img]);
  const int col = c0 + wave;                         // u cell 0..H-1
  // one weight / kept-baseline partial per column, written by its wavefront
  int* wslot = a.wpart + (size_t)img * a.wstride + col;
  int* kslot = a.kpart + (size_t)img * a.wstride + col;
  if (c0 >= ncols) {                                 // the whole tile is empty
    if (lane == 0 && col < H) { *wslot = 0; *kslot = 0; }
    return;
  }
  const bool active = col < ncols;
  float2* hbuf = lds + wave * C_::STRIDE;
  int* hcnt = UNI ? lcnt + wave * H : nullptr;
  unsigned* lclaim = reinterpret_cast<unsigned*>(lcnt + (UNI ? CPW * H : 0));
  const double s = cells_per_metre(a.freq[ch], a.ndx);
  const float2* tw = stage_twiddles<N, C_::CL>(ltw);
  // the only workgroup barrier: it publishes the LDS twiddles; after it every
  // wavefront grids and transforms its column without waiting for the others
  if (TwLds<N>::ON) __syncthreads();

  ColSpan span{0, 0, 0, 0};
  if (active) {
    const int* bnd = a.bnd + (size_t)img * (N + 2);
    span = ColSpan{bnd[col + H], bnd[col + 1 + H], bnd[-col + H], bnd[-col + 1 + H]};
  }
  // the rest is compiled once per zero band of the first stage and chosen per
  // workgroup (all of its columns belong to one image)
  auto body = [&](auto zbc) {
    constexpr int ZB = decltype(zbc)::value;
    HalfIn<N> in;
    int kd = 0, kc = 0, occ = 0;
    Claim cl = claim_init(lclaim + wave * CLAIM_SLOTS, lane);
    if (a.sd != nullptr) grid_col_half<N, true, UNI, ZB>(a, span, hbuf, hcnt, in, t, ch, s, lane, kd, kc, occ, cl);
    else grid_col_half<N, false, UNI, ZB>(a, span, hbuf, hcnt, in, t, ch, s, lane, kd, kc, occ, cl);
    // baselines counted once: the direct entry of every cell column, plus the
    // conjugate entries of columns whose mirror the image path never visits
    const int kept_b = kd + (col > 0 ? kc : 0);
    const int mult = col > 0 ? 2 : 1;
    int wcontrib;
    if (UNI) {
      for (int o = WAVE / 2; o > 0; o >>= 1) occ += __shfl_xor(occ, o);
      wcontrib = mult * occ;
    } else {
      wcontrib = mult * (kd + kc);
    }
    if (lane == 0 && col < H) { *wslot = wcontrib; *kslot = kept_b; }
    if (active) {
      // rows of the cutout straight from the last stage: output row m holds
      // v-frequency q = (m - M/2) mod N
      float2* dst = a.half + ((size_t)li * H + col) * a.M;
      const int hm = HMC > 0 ? HMC : a.M / 2;
      wave_fft_half_emit<N, +1, ZB, C_::CL>(hbuf, lane, tw, in, [&](auto qb, float2 v) {
        cutout_block<N, decltype(qb)::value>(lane, hm, [&](unsigned m) { store_at(dst, m, v); });
      });
    }
  };
  if (HalfIn<N>::R == 16 && column_zero_band<N>(a, t, s) >= 4) body(ic<HalfIn<N>::R == 16 ? 4 : 0>{});
  else body(ic<0>{});
}

__global__ void k_grid_finish(ImgArgs a, int n_img) {
  const int img = blockIdx.x * blockDim.x + threadIdx.x;
  if (img >= n_img) return;
  const int t = img / a.C;
  int w = 0, k = 0;
  float wf = 0.f;                                    // kernel gridding: FP32 weight sums
  for (int i = 0; i < a.wtiles; ++i) {
    w += a.wpart[(size_t)img * a.wstride + i];
    wf += __int_as_float(a.wpart[(size_t)img * a.wstride + i]);
    k += a.kpart[(size_t)img * a.wstride + i];
  }
  if (a.weight_sum) a.weight_sum[img] = a.kw > 0 ? wf : (float)w;
  if (a.n_dropped) a.n_dropped[img] = a.n_unflagged[t] - k;
}

// ============================================================== row pass
template <int N>
struct Rows {
  // buffer stride of 4 mod 32 complex: the workgroup's PPW buffers start on
  // different bank groups, so filling them side by side is conflict-free
  static constexpr int STRIDE = padded_len(N) + ((4 - padded_len(N) % 32) + 32) % 32;
  static constexpr int PPW = N <= 1024 ? 8 : (N <= 2048 ? 4 : 2);  // row pairs (waves) per WG
  static constexpr int THREADS = PPW * WAVE;
  static constexpr int TW = TwLds<N>::ON ? tw_entries(N) : 0;
  static constexpr size_t LDS = (size_t)(PPW * STRIDE + TW) * sizeof(float2);
};

// Inverse transform along u of two cutout rows per wavefront. The half
// spectrum A[k] (k < N/2) of row m and B[k] of row m+1 are packed as
// Z = A_full + i B_full with the Hermitian extensions A_full[N-k] = conj A[k]
// (A_full[N/2] = 0: the Nyquist column is never gridded), so one complex
// transform yields row m as Re z and row m+1 as Im z. The shift, 1/W and the
// cutout are applied as the rows are stored.
// Persistent form: a fixed grid of workgroups walks the (image, row tile)
// list. For N <= 1024, while the transforms of one tile run, the
// half-spectrum slice of the next tile is already in flight into registers,
// so the HBM latency of the loads hides behind the arithmetic of the previous
// tile (larger N would need too many registers and loads per tile instead).
// AL: the cutout half-width M/2 is a multiple of the wavefront width and the
// plan's last-stage blocks are aligned (blocks_aligned), so each block of 64
// output columns is stored or skipped whole.
// KB: the image was gridded with the Kaiser-Bessel kernel; the stores apply
// its correction.
template <int N, bool AL, bool KB>
__global__ void __launch_bounds__(Rows<N>::THREADS) k_rows(ImgArgs a) {
  static_assert(!AL || blocks_aligned(N), "aligned cutout needs aligned blocks");
  extern __shared__ float4 lds_raw[];
  constexpr int H = N / 2;
  constexpr int PPW = Rows<N>::PPW;
  constexpr int ST = Rows<N>::STRIDE;
  constexpr int THR = Rows<N>::THREADS;
  constexpr int EPT = (H * PPW + THR - 1) / THR;     // half-spectrum float4 loads per thread
  constexpr bool PREF = EPT <= 8;
  constexpr int NPRE = PREF ? EPT : 1;
  float2* lds = reinterpret_cast<float2*>(lds_raw);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), lane = threadIdx.x % WAVE;
  const int M = a.M;
  const int npair = M / 2;
  const int ntr = (npair + PPW - 1) / PPW;           // row tiles per image
  const int total = a.nimg * ntr;
  const float2* tw = stage_twiddles<N>(lds + PPW * ST);
  // kernel gridding: 1 / c((l - M/2) / N) per image column l (the same table
  // serves the rows: the correction is separable), published by the first
  // barrier of the loop
  float* lcorr = reinterpret_cast<float*>(lds + PPW * ST + Rows<N>::TW);
  constexpr bool kbon = KB;
  if (kbon)
    for (int l = threadIdx.x; l < a.M; l += THR) lcorr[l] = kb_inv_taper((double)(l - a.M / 2) / N, a);

  // thread t always serves pair slot t % PPW and columns t / PPW + i * (THR / PPW)
  const int kt = threadIdx.x / PPW, pt = threadIdx.x % PPW;
  auto load = [&](int tile, int i) -> float4 {
    const int li = tile / ntr, p0 = (tile % ntr) * PPW;
    const int nz = min(H, a.ncz[a.img0 + li]);
    const int k = kt + i * (THR / PPW);
    const float4* src = reinterpret_cast<const float4*>(a.half + (size_t)li * H * M) + (p0 + pt);
    return (k < nz && p0 + pt < npair) ? src[(size_t)k * (M / 2)] : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  float4 pre[NPRE];
  int tile = blockIdx.x;
  if (PREF && tile < total) {
#pragma unroll
    for (int i = 0; i < NPRE; ++i) pre[i] = load(tile, i);
  }
#pragma nounroll
  for (; tile < total; tile += gridDim.x) {
    // lane-dependent addresses are recomputed inside the loop: hoisted out of
    // it they would stay live across the transforms and cost occupancy
    int lane_i = lane, ln = threadIdx.x;
    asm volatile("" : "+v"(lane_i), "+v"(ln));
    const int li = tile / ntr, p0 = (tile % ntr) * PPW;
    const int img = a.img0 + li;
    const float W = kbon ? sum_partials_f(a.wpart, img, a.wstride, a.wtiles, lane_i)
                         : (float)sum_partials(a.wpart, img, a.wstride, a.wtiles, lane_i);
    const float scale = a.norm ? (W > 0 ? 1.0f / W : 0.0f) : 1.0f;
    if (p0 == 0 && ln == 0 && a.weight_sum) a.weight_sum[img] = W;
    const int kti = ln / PPW, pti = ln % PPW;
    __syncthreads();                                  // previous tile's rows have left LDS
    auto put = [&](int i, float4 ab) {
      const int k = kti + i * (THR / PPW);
      float2* z = lds + pti * ST;
      if (k == 0) {
        z[pad(0)] = make_float2(ab.x, ab.z);
        z[pad(H)] = make_float2(0.f, 0.f);
      } else {
        z[pad(k)] = make_float2(ab.x - ab.w, ab.y + ab.z);
        z[pad(N - k)] = make_float2(ab.x + ab.w, ab.z - ab.y);
      }
    };
    if constexpr (PREF) {
#pragma unroll
      for (int i = 0; i < NPRE; ++i)
        if (kti + i * (THR / PPW) < H) put(i, pre[i]);
    } else {
      for (int i = 0; kti + i * (THR / PPW) < H; ++i) put(i, load(tile, i));
    }
    __syncthreads();
    if (PREF && tile + (int)gridDim.x < total) {
#pragma unroll
      for (int i = 0; i < NPRE; ++i) pre[i] = load(tile + gridDim.x, i);
    }
    const int pair = p0 + wave;
    if (pair < npair) {
      float2* z = lds + wave * ST;
      float* r0 = a.images + ((size_t)img * M + 2 * pair) * M;
      float* r1 = r0 + M;
      float s0 = scale, s1 = scale;
      if (kbon) {
        s0 *= lcorr[2 * pair];
        s1 *= lcorr[2 * pair + 1];
      }
      int hm = M / 2;
      asm volatile("" : "+s"(hm));   // block tests stay inside the loop (hoisted they spill)
      // image columns of the cutout straight from the last stage: column l
      // holds u-frequency q = (l - M/2) mod N; row 2p is Re z, row 2p+1 is Im z
      wave_fft_emit<N, +1>(z, lane_i, tw, [&](auto qb, float2 v) {
        auto st = [&](unsigned l) {
          const float cl = kbon ? lcorr[l] : 1.0f;
          store_at(r0, l, v.x * s0 * cl);
          store_at(r1, l, v.y * s1 * cl);
        };
        if constexpr (AL) cutout_block_aligned<N, decltype(qb)::value>(lane_i, hm, st);
        else cutout_lane<N, decltype(qb)::value>(lane_i, hm, st);
      });
    }
  }
}

// Row pass with the transforms' exchanges through half-length LDS buffers
// (see wave_fft_half_emit): the same packing, shift, 1/W, cutout and stores
// as k_rows, and the same tiling (one workgroup per row tile, or a
// persistent grid walking the tiles). The workgroup fills the lower halves
// of its PPW packed rows (z[k], k < N/2) from one load of the half-spectrum
// slice, each wavefront takes its first stage's lower inputs, then the upper
// halves (z[N - k]) follow from the same registers. With no prefetch across
// tiles and half the LDS, three workgroups share a CU instead of two.
template <int N>
struct RowsHalf {
  static constexpr int STRIDE = padded_len(N / 2) + ((4 - padded_len(N / 2) % 32) + 32) % 32;
  static constexpr int PPW = Rows<N>::PPW;
  static constexpr int THREADS = PPW * WAVE;
  static constexpr int TW = TwLds<N>::ON ? tw_entries(N) : 0;
  static constexpr size_t LDS = (size_t)(PPW * STRIDE + TW) * sizeof(float2);
};

// HMC > 0: the cutout half-width fixed at compile time (see k_grid_cols_half).
template <int N, bool AL, bool KB, int HMC = 0>
__global__ void __launch_bounds__(RowsHalf<N>::THREADS) k_rows_half(ImgArgs a) {
  static_assert(!AL || blocks_aligned(N), "aligned cutout needs aligned blocks");
  extern __shared__ float4 lds_raw[];
  constexpr int H = N / 2;
  constexpr int PPW = RowsHalf<N>::PPW;
  __shared__ int wred[PPW];                          // per-wavefront sums of the weight partials
  constexpr int ST = RowsHalf<N>::STRIDE;
  constexpr int THR = RowsHalf<N>::THREADS;
  constexpr int EPT = (H * PPW + THR - 1) / THR;     // half-spectrum float4 loads per thread
  constexpr int R0 = HalfIn<N>::R;
  float2* lds = reinterpret_cast<float2*>(lds_raw);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), lane = threadIdx.x % WAVE;
  const int M = a.M;
  const int npair = M / 2;
  const int ntr = (npair + PPW - 1) / PPW;           // row tiles per image
  const int total = a.nimg * ntr;
  const float2* tw = stage_twiddles<N>(lds + PPW * ST);
  float* lcorr = reinterpret_cast<float*>(lds + PPW * ST + RowsHalf<N>::TW);
  if (KB)
    for (int l = threadIdx.x; l < a.M; l += THR) lcorr[l] = kb_inv_taper((double)(l - a.M / 2) / N, a);

#pragma nounroll
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    // lane-dependent addresses are formed inside the loop: hoisted out of it
    // they would stay live across the transforms and cost occupancy
    int lane_i = lane, ln = threadIdx.x;
    asm volatile("" : "+v"(lane_i), "+v"(ln));
    // thread t serves pair slot t % PPW and columns t / PPW + i * (THR / PPW)
    const int kt = ln / PPW, pt = ln % PPW;
    const int li = tile / ntr, p0 = (tile % ntr) * PPW;
    const int img = a.img0 + li;
    const int nz = min(H, a.ncz[img]);               // u cells >= nz are empty
    // the rest of the tile is compiled once per zero band of the first stage
    // and chosen per tile (all of its rows belong to one image)
    auto body = [&](auto zbc) {
      constexpr int ZB = decltype(zbc)::value;
      float4 ab[EPT];
      {
        const float4* src = reinterpret_cast<const float4*>(a.half + (size_t)li * H * M) + (p0 + pt);
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
          const int k = kt + i * (THR / PPW);
          ab[i] = (k < nz && p0 + pt < npair) ? src[(size_t)k * (M / 2)] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
      // the image's weight sum W from its partials (integers, or FP32 sums with
      // a gridding kernel), split over the workgroup and combined in LDS
      int wli = 0;
      float wlf = 0.f;
      for (int i = ln; i < a.wtiles; i += THR) {
        const int pv = a.wpart[(size_t)img * a.wstride + i];
        wli += pv;
        wlf += __int_as_float(pv);
      }
      for (int o = WAVE / 2; o > 0; o >>= 1) {
        if (KB) wlf += __shfl_xor(wlf, o);
        else wli += __shfl_xor(wli, o);
      }
      float2* zs = lds + pt * ST;                       // the packed row this thread fills
      float2* z = lds + wave * ST;                      // the packed row this wavefront transforms
      HalfIn<N> in;
      __syncthreads();                                  // previous tile's rows have left LDS
      if (lane_i == 0) wred[wave] = KB ? __float_as_int(wlf) : wli;
#pragma unroll
      for (int i = 0; i < EPT; ++i) {                   // lower half: z[k] = A[k] + i B[k]
        const int k = kt + i * (THR / PPW);
        if (k < H) {
          const float4 v = ab[i];
          zs[pad(k)] = k == 0 ? make_float2(v.x, v.z) : make_float2(v.x - v.w, v.y + v.z);
        }
      }
      __syncthreads();
      float W;
      if (KB) {
        float f = 0.f;
        for (int w = 0; w < PPW; ++w) f += __int_as_float(wred[w]);
        W = f;
      } else {
        int n = 0;
        for (int w = 0; w < PPW; ++w) n += wred[w];
        W = (float)n;
      }
      const float scale = a.norm ? (W > 0 ? 1.0f / W : 0.0f) : 1.0f;
      if (p0 == 0 && ln == 0 && a.weight_sum) a.weight_sum[img] = W;
      half_read<N, R0, 0, ZB>(z, lane_i, in.v);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < EPT; ++i) {                   // upper half: z[N - k] = conj A[k] + i conj B[k]
        const int k = kt + i * (THR / PPW);
        if (k < H) {
          const float4 v = ab[i];
          zs[pad(k == 0 ? 0 : H - k)] = k == 0 ? make_float2(0.f, 0.f) : make_float2(v.x + v.w, v.z - v.y);
        }
      }
      __syncthreads();
      half_read<N, R0, 1, ZB>(z, lane_i, in.v);
      const int pair = p0 + wave;
      if (pair < npair) {
        float* r0 = a.images + ((size_t)img * M + 2 * pair) * M;
        float* r1 = r0 + M;
        float s0 = scale, s1 = scale;
        if (KB) {
          s0 *= lcorr[2 * pair];
          s1 *= lcorr[2 * pair + 1];
        }
        int hm = HMC > 0 ? HMC : M / 2;
        // block tests stay inside the loop (hoisted they spill)
        if constexpr (HMC == 0) asm volatile("" : "+s"(hm));
        // image columns of the cutout straight from the last stage: column l
        // holds u-frequency q = (l - M/2) mod N; row 2p is Re z, row 2p+1 is Im z
        wave_fft_half_emit<N, +1, ZB>(z, lane_i, tw, in, [&](auto qb, float2 v) {
          auto st = [&](unsigned l) {
            const float cl = KB ? lcorr[l] : 1.0f;
            store_at(r0, l, v.x * s0 * cl);
            store_at(r1, l, v.y * s1 * cl);
          };
          if constexpr (AL) cutout_block_aligned<N, decltype(qb)::value>(lane_i, hm, st);
          else cutout_lane<N, decltype(qb)::value>(lane_i, hm, st);
        });
      }
    };
    if (HalfIn<N>::R == 16 && zero_band(N, nz) >= 4) body(ic<HalfIn<N>::R == 16 ? 4 : 0>{});
    else body(ic<0>{});
  }
}

// ============================================================== dynamic spectra
// Transpose of the image cube [T][C][P] to per-pixel time series [P][C][T]
// with the reference image subtracted on the way. One workgroup per tile of
// DS_TT timesteps x DS_PP pixels of one channel: the rows of the tile (and,
// for a mean over K preceding images, the K rows before it) are read with
// consecutive pixels on consecutive lanes, all loads of a thread issued
// before the first is used; the differences are formed per pixel and staged
// in LDS as [pixel][time]; each pixel's series is then written with
// consecutive timesteps on consecutive lanes. VEC moves 16 bytes per lane
// (P and T multiples of 4, 16-byte aligned arrays).
// Grid: one dimension, workgroup L on XCD L mod 8. The channel varies fastest
// among the workgroups of an XCD, and all time tiles of a pixel tile share
// its XCD, so the series of (p, c) and (p, c + 1), adjacent in the output,
// are written close together into the same L2 and leave it as whole lines.
constexpr int DS_TT = 128, DS_PP = 64, DS_THREADS = 256, DS_KMAX = 128;
constexpr int DS_ST = DS_PP + 1;                              // LDS row stride (floats)

// One LDS buffer of min(DS_TT, T) + K rows (a series shorter than a tile
// needs fewer rows, so more workgroups share a CU): the differences overwrite
// the tile's own rows once every thread has read its window, and the stores
// read them back column-wise (the odd stride keeps both directions off a
// single bank). Rows at or beyond T are never read or written.
__host__ __device__ constexpr int dynspec_rows(int t) { return t < DS_TT ? t : DS_TT; }
__host__ __device__ constexpr size_t dynspec_lds(int k, int t) {
  return (size_t)(dynspec_rows(t) + k) * DS_ST * sizeof(float);
}

template <bool VEC>
__global__ void __launch_bounds__(DS_THREADS) k_dynspec(const float* __restrict__ img, int T, int C, long long P,
                                                        int mode, int K, const float* __restrict__ ref,
                                                        float* __restrict__ out, int npt8) {
  extern __shared__ float4 lds_raw[];
  float* rows = reinterpret_cast<float*>(lds_raw);            // [DS_TT + K][DS_ST]
  const long long L = blockIdx.x;
  const long long r8 = L >> 3;
  const int c = (int)(r8 % C);
  const long long u = (r8 / C) * 8 + (L & 7);                // tile: u = time tile * npt8 + pixel tile
  const long long pt = u % npt8;
  const int tt = (int)(u / npt8);
  const long long p0 = pt * DS_PP;
  const int t0 = tt * DS_TT;
  if (p0 >= P || t0 >= T) return;                             // padding of the pixel tiles to 8
  const int r0 = t0 - K;                                      // first row held (may be < 0)
  const int nrows = dynspec_rows(T) + K;
  if constexpr (VEC) {
    constexpr int Q = DS_PP / 4;                              // float4 per row
    constexpr int MAXI = (DS_TT + DS_KMAX) * Q / DS_THREADS;
    float4 v[MAXI];
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
      const int e = threadIdx.x + i * DS_THREADS;
      const int r = e / Q, q = e % Q;
      const int t = r0 + r;
      const long long p = p0 + 4 * q;
      v[i] = (r < nrows && t >= 0 && t < T && p < P)
                 ? *reinterpret_cast<const float4*>(img + ((long long)t * C + c) * P + p)
                 : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
      const int e = threadIdx.x + i * DS_THREADS;
      const int r = e / Q, q = e % Q;
      if (r < nrows) {
        float* d = rows + r * DS_ST + 4 * q;
        d[0] = v[i].x; d[1] = v[i].y; d[2] = v[i].z; d[3] = v[i].w;
      }
    }
  } else {
    for (int e = threadIdx.x; e < nrows * DS_PP; e += DS_THREADS) {
      const int r = e / DS_PP, jj = e % DS_PP;
      const int t = r0 + r;
      const long long p = p0 + jj;
      rows[r * DS_ST + jj] = (t >= 0 && t < T && p < P) ? img[((long long)t * C + c) * P + p] : 0.0f;
    }
  }
  __syncthreads();
  // thread = (pixel j, segment g of the tile's timesteps)
  const int j = threadIdx.x % DS_PP, g = threadIdx.x / DS_PP;
  constexpr int SEG = DS_TT / (DS_THREADS / DS_PP);
  const float rv = (mode == 2 && p0 + j < P) ? ref[(long long)c * P + p0 + j] : 0.0f;
  double win = 0.0;                                           // sum of the k preceding images
  const int ta = t0 + g * SEG;
  if (mode == 1 && ta < T) {
    const int k = min(K, ta);
    for (int s = ta - k; s < ta; ++s) win += (double)rows[(s - r0) * DS_ST + j];
  }
  float dv[SEG];
#pragma unroll
  for (int i = 0; i < SEG; ++i) {
    const int t = ta + i;
    float d = 0.0f;
    if (t < T) {                                              // rows from T on are not held
      const float x = rows[(t - r0) * DS_ST + j];
      if (mode == 0) {
        d = x;
      } else if (mode == 2) {
        d = x - rv;
      } else {
        // mean of the window: 1/k is exact for k a power of two and within an
        // ulp of double otherwise, far below the final rounding to float
        const int k = min(K, t);
        d = t == 0 ? 0.0f : (float)((double)x - win * (1.0 / (double)k));
        // slide the window to end at t: add x, drop the image K behind
        win += (double)x;
        if (t - K >= 0) win -= (double)rows[(t - K - r0) * DS_ST + j];
      }
    }
    dv[i] = d;
  }
  __syncthreads();                                            // every window has been read
#pragma unroll
  for (int i = 0; i < SEG; ++i)
    if (ta + i < T) rows[(ta + i - r0) * DS_ST + j] = dv[i];
  __syncthreads();
  if constexpr (VEC) {
    constexpr int Q = DS_TT / 4;                              // float4 per pixel series
#pragma unroll
    for (int i = 0; i < DS_PP * Q / DS_THREADS; ++i) {
      const int e = threadIdx.x + i * DS_THREADS;
      const int pj = e / Q, q = e % Q;
      const long long p = p0 + pj;
      const int t = t0 + 4 * q;
      if (p < P && t < T) {
        const float* src = rows + (t - r0) * DS_ST + pj;
        *reinterpret_cast<float4*>(out + (p * C + c) * T + t) =
            make_float4(src[0], src[DS_ST], src[2 * DS_ST], src[3 * DS_ST]);
      }
    }
  } else {
    for (int e = threadIdx.x; e < DS_PP * DS_TT; e += DS_THREADS) {
      const int pj = e / DS_TT, tq = e % DS_TT;
      const long long p = p0 + pj;
      const int t = t0 + tq;
      if (p < P && t < T) out[(p * C + c) * T + t] = rows[(t - r0) * DS_ST + pj];
    }
  }
}

// ============================================================== correlator X-engine
// V_ij = sum_s x_i(s) conj(x_j(s)) for 8-bit complex voltages x[t][c][a][s]
// (real, imaginary interleaved), on the matrix cores. With x = r + i q:
//   Re V_ij = sum r_i r_j + q_i q_j,   Im V_ij = sum q_i r_j - r_i q_j,
// i.e. integer matrix products of the antenna-by-sample matrices R and Q.
// One wavefront computes a 64 x 64 tile of antenna pairs (tile row I <= tile
// column J) as 4 x 4 blocks of 16 x 16 with v_mfma_i32_16x16x64_i8, 64
// samples per step: lane (g, q) holds antenna q of a block and the 16
// samples 16 g .. 16 g + 15 of the step, so one 16-byte load instruction
// reads 16 antenna rows, 64 contiguous bytes of each (a 32 x 32 block with
// one antenna per lane would touch 64 rows per instruction, and the vector
// memory path, which handles each touched line in turn, then sets the pace).
// Each lane loads 32 bytes of each of its four row and four column antennas,
// splits real and imaginary bytes with byte permutes, and issues 64 products
// into 48 int32 accumulator sets (RR + QQ, QR, RQ per block); every operand
// feeds four blocks. The next step's loads are in flight during the
// products. A and B see the same sample order in every lane, so the dot
// products do not depend on how the matrix cores order k within a lane.
// Sums are exact in int32 for up to 65520 samples. The workgroups of one
// (t, c) run on one XCD, so its voltages are read from HBM once and served to
// every tile from L2.
typedef int xe_v4i __attribute__((ext_vector_type(4)));
constexpr int XE_BLK = 16;      // antennas per MFMA block
constexpr int XE_NB = 4;        // blocks per tile edge
constexpr int XE_TILE = XE_BLK * XE_NB;   // antennas per wavefront tile edge
constexpr int XE_STEP = 64;     // samples per MFMA step (16 per quarter-wavefront)
// RR + QQ of S samples reaches 2 S 128^2 in magnitude: below 2^31 up to this S
constexpr int XE_MAX_SAMPLES = 65520;

struct XeArgs {
  const int8_t* volt;           // [T][C][A][S][2]
  float2* vis;                  // [T][C][A(A-1)/2]
  float* autos;                 // [T][C][A] or null
  int T, C, A, S;
  int nt;                       // antenna tiles: ceil(A / 64)
  int npairs;                   // nt (nt + 1) / 2 tile pairs per (t, c)
  long long nimg;               // T * C
};

// Real and imaginary bytes of 16 interleaved complex int8 samples (32 bytes).
__device__ __forceinline__ void xe_split(const uint4 lo, const uint4 hi, xe_v4i& re, xe_v4i& im) {
  // v_perm_b32 picks bytes of the 64-bit value {a, b} (b = bytes 0-3)
  re.x = __builtin_amdgcn_perm(lo.y, lo.x, 0x06040200u);
  im.x = __builtin_amdgcn_perm(lo.y, lo.x, 0x07050301u);
  re.y = __builtin_amdgcn_perm(lo.w, lo.z, 0x06040200u);
  im.y = __builtin_amdgcn_perm(lo.w, lo.z, 0x07050301u);
  re.z = __builtin_amdgcn_perm(hi.y, hi.x, 0x06040200u);
  im.z = __builtin_amdgcn_perm(hi.y, hi.x, 0x07050301u);
  re.w = __builtin_amdgcn_perm(hi.w, hi.z, 0x06040200u);
  im.w = __builtin_amdgcn_perm(hi.w, hi.z, 0x07050301u);
}

__global__ void __launch_bounds__(WAVE) k_xengine(XeArgs a) {
  constexpr int NOP = 2 * XE_NB;                              // operand antennas per lane
  const long long L = blockIdx.x;
  const long long r8 = L >> 3;
  const long long img = (r8 / a.npairs) * 8 + (L & 7);
  if (img >= a.nimg) return;                                  // padding of the last group of 8
  int pr = (int)(r8 % a.npairs);
  int ti = 0;                                                 // tile pair -> (ti <= tj)
  while (pr >= a.nt - ti) { pr -= a.nt - ti; ++ti; }
  const int tj = ti + pr;
  const int lane = threadIdx.x;
  const int g = lane >> 4, q = lane & 15;
  const size_t rowb = (size_t)a.S * 2;                        // bytes per antenna row
  const int8_t* base = a.volt + (size_t)img * a.A * rowb;
  // operand antennas of this lane: rows ti*64 + 16k + q, columns tj*64 + 16k + q
  const uint4* pa[NOP];
  bool ok[NOP];
#pragma unroll
  for (int k = 0; k < NOP; ++k) {
    const int ant = (k < XE_NB ? ti : tj) * XE_TILE + (k % XE_NB) * XE_BLK + q;
    ok[k] = ant < a.A;
    pa[k] = reinterpret_cast<const uint4*>(base + (size_t)(ok[k] ? ant : 0) * rowb);
  }
  xe_v4i acc[XE_NB][XE_NB][3];
#pragma unroll
  for (int x = 0; x < XE_NB; ++x)
#pragma unroll
    for (int y = 0; y < XE_NB; ++y)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[x][y][k] = xe_v4i{0, 0, 0, 0};
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  // operand bytes of step s0 (zeros beyond S or beyond A). Unconditional
  // 16-byte loads from a clamped, valid address (antenna 0, first chunk),
  // zeroed afterwards, so no branches sit in the load path.
  uint4 f[2 * NOP];
  auto fetch = [&](int s0) {
    const int s = s0 + 16 * g;                                // this quarter-wavefront's 16 samples
    const bool in = s < a.S;                                  // S is a multiple of 16
    const int u = in ? s >> 3 : 0;                            // uint4 index: 8 samples per 16 bytes
#pragma unroll
    for (int k = 0; k < NOP; ++k) {
      f[2 * k] = pa[k][u];
      f[2 * k + 1] = pa[k][u + 1];
      if (!(ok[k] && in)) { f[2 * k] = z; f[2 * k + 1] = z; }
    }
  };
  xe_v4i r[NOP], qv[NOP];
  auto split = [&]() {
#pragma unroll
    for (int k = 0; k < NOP; ++k) xe_split(f[2 * k], f[2 * k + 1], r[k], qv[k]);
  };
  if (a.S > 0) {                                              // (no samples: nothing to read)
    fetch(0);
    split();
  }
  for (int s0 = 0; s0 < a.S; s0 += XE_STEP) {
    fetch(s0 + XE_STEP);
    // the two products into one accumulator set are 32 issues apart
#pragma unroll
    for (int x = 0; x < XE_NB; ++x)
#pragma unroll
      for (int y = 0; y < XE_NB; ++y)
        acc[x][y][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(r[x], r[XE_NB + y], acc[x][y][0], 0, 0, 0);
#pragma unroll
    for (int x = 0; x < XE_NB; ++x)
#pragma unroll
      for (int y = 0; y < XE_NB; ++y) {
        acc[x][y][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(qv[x], r[XE_NB + y], acc[x][y][1], 0, 0, 0);
        acc[x][y][2] = __builtin_amdgcn_mfma_i32_16x16x64_i8(r[x], qv[XE_NB + y], acc[x][y][2], 0, 0, 0);
      }
#pragma unroll
    for (int x = 0; x < XE_NB; ++x)
#pragma unroll
      for (int y = 0; y < XE_NB; ++y)
        acc[x][y][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(qv[x], qv[XE_NB + y], acc[x][y][0], 0, 0, 0);
    split();
  }
  // accumulator element e of lane (g, q) in block (x, y) holds row
  // i = ti*64 + 16x + 4g + e and column j = tj*64 + 16y + q
  const size_t nbl = (size_t)a.A * (a.A - 1) / 2;
  float2* v = a.vis + (size_t)img * nbl;
#pragma unroll
  for (int x = 0; x < XE_NB; ++x)
#pragma unroll
    for (int y = 0; y < XE_NB; ++y) {
      const int j = tj * XE_TILE + y * XE_BLK + q;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = ti * XE_TILE + x * XE_BLK + 4 * g + e;
        if (j < a.A && i < j) {
          const size_t b = (size_t)i * a.A - (size_t)i * (i + 1) / 2 + (j - i - 1);
          v[b] = make_float2((float)acc[x][y][0][e], (float)(acc[x][y][1][e] - acc[x][y][2][e]));
        } else if (a.autos != nullptr && i == j && j < a.A) {
          a.autos[(size_t)img * a.A + i] = (float)acc[x][y][0][e];
        }
      }
    }
}

// ============================================================== plain 2D FFT
template <int N>
struct Fft2 {
  static constexpr int STRIDE = padded_len(N) + 4;
  static constexpr int VPW = N <= 1024 ? 8 : (N <= 2048 ? 4 : 2);   // vectors per workgroup
  static constexpr int THREADS = VPW * WAVE;
  static constexpr size_t LDS = (size_t)VPW * STRIDE * sizeof(float2);
};

template <int N, int SIGN>
__global__ void __launch_bounds__(Fft2<N>::THREADS) k_fft_rows(const float2* in, float2* out, int nrows) {
  extern __shared__ float4 lds_raw[];
  float2* lds = reinterpret_cast<float2*>(lds_raw);
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const long row = (long)blockIdx.x * Fft2<N>::VPW + wave;
  if (row >= nrows) return;
  float2* z = lds + wave * Fft2<N>::STRIDE;
  const float2* s = in + row * N;
  for (int i = lane; i < N; i += WAVE) z[pad(i)] = s[i];
  wave_sync();
  wave_fft<N, SIGN>(z, lane, TwTable<N>::stages());
  float2* d = out + row * N;
  for (int i = lane; i < N; i += WAVE) d[i] = z[pad(i)];
}

template <int N, int SIGN>
__global__ void __launch_bounds__(Fft2<N>::THREADS) k_fft_cols(float2* data) {
  extern __shared__ float4 lds_raw[];
  constexpr int VPW = Fft2<N>::VPW;
  float2* lds = reinterpret_cast<float2*>(lds_raw);
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int c0 = blockIdx.x * VPW;
  float2* img = data + (size_t)blockIdx.y * N * N;
  for (int e = threadIdx.x; e < N * VPW; e += blockDim.x) {
    const int r = e / VPW, w = e % VPW;
    if (c0 + w < N) lds[w * Fft2<N>::STRIDE + pad(r)] = img[(size_t)r * N + c0 + w];
  }
  __syncthreads();
  if (c0 + wave < N) wave_fft<N, SIGN>(lds + wave * Fft2<N>::STRIDE, lane, TwTable<N>::stages());
  __syncthreads();
  for (int e = threadIdx.x; e < N * VPW; e += blockDim.x) {
    const int r = e / VPW, w = e % VPW;
    if (c0 + w < N) img[(size_t)r * N + c0 + w] = lds[w * Fft2<N>::STRIDE + pad(r)];
  }
}

// ============================================================== adjoint
// Weight sums alone (the adjoint needs 1/W before anything else): counts of
// kept entries (natural) or occupied cells (uniform) per half-spectrum column.
template <int N, bool UNI>
__global__ void __launch_bounds__(Cols<N>::THREADS) k_weights(ImgArgs a) {
  extern __shared__ int lw_raw[];
  __shared__ int red[Cols<N>::CPW];
  constexpr int H = N / 2;
  constexpr int CPW = Cols<N>::CPW;
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int li = blockIdx.y;
  const int img = a.img0 + li;
  const int t = img / a.C, ch = img - t * a.C;
  const int cs = blockIdx.x * CPW + wave;
  int w = 0;
  if (cs < min(H, a.ncz[img])) {
    int* cnt = lw_raw + wave * N;
    const double s = cells_per_metre(a.freq[ch], a.ndx);
    if (UNI) {
      for (int r = lane; r < N; r += WAVE) cnt[r] = 0;
      wave_sync();
    }
    const int* bnd = a.bnd + (size_t)img * (N + 2);
    const size_t tb = (size_t)t * a.B;
    int kept = 0;
    for (int pass = 0; pass < 2; ++pass) {
      const int c = pass == 0 ? cs : -cs;
      const int lo = bnd[c + H], hi = bnd[c + 1 + H];
      for (int j = lo + lane; j < hi; j += WAVE) {
        const double iv = rint(a.sv[tb + j] * s);
        if (fabs(iv) < (double)H) {
          ++kept;
          if (UNI) {
            int r = (int)iv;
            if (pass) r = -r;
            atomicAdd(&cnt[r < 0 ? r + N : r], 1);
          }
        }
      }
    }
    w = kept;
    if (UNI) {
      wave_sync();
      int occ = 0;
      for (int r = lane; r < N; r += WAVE) occ += cnt[r] > 0;
      w = occ;
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) w += __shfl_xor(w, o);
    w *= (cs > 0 ? 2 : 1);
  }
  if (lane == 0) red[wave] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ws = 0;
    for (int i = 0; i < CPW; ++i) ws += red[i];
    a.wpart[(size_t)img * a.wstride + blockIdx.x] = ws;
  }
}

// Adjoint of k_rows: image-gradient rows m, m+1 (zero outside the cutout,
// times 1/W, shift undone) packed as z = a + i b, forward transform, then the
// half-spectrum gradients c_k A[k], c_k B[k] (c_0 = 1, c_k = 2) with
// A[k] = (Z[k] + conj Z[N-k]) / 2 and B[k] = (Z[k] - conj Z[N-k]) / (2i).
// Only the columns that can hold baselines (k < ncz) are stored.
template <int N>
__global__ void __launch_bounds__(Rows<N>::THREADS) k_rows_adj(ImgArgs a) {
  extern __shared__ float4 lds_raw[];
  constexpr int H = N / 2;
  constexpr int PPW = Rows<N>::PPW;
  constexpr int ST = Rows<N>::STRIDE;
  float2* lds = reinterpret_cast<float2*>(lds_raw);
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int li = blockIdx.y;
  const int img = a.img0 + li;
  const int M = a.M;
  const int npair = M / 2;
  const int p0 = blockIdx.x * PPW;
  const int nz = min(H, a.ncz[img]);
  const float W = a.wsum_in ? a.wsum_in[img]
                  : a.kw > 0 ? sum_partials_f(a.wpart, img, a.wstride, a.wtiles, lane)
                             : (float)sum_partials(a.wpart, img, a.wstride, a.wtiles, lane);
  const float scale = a.norm ? (W > 0 ? 1.0f / W : 0.0f) : 1.0f;
  const float2* tw = stage_twiddles<N>(lds + PPW * ST);
  __syncthreads();
  const int pair = p0 + wave;
  if (pair < npair) {
    float2* z = lds + wave * ST;
    for (int r = lane; r < ST; r += WAVE) z[r] = make_float2(0.f, 0.f);
    wave_sync();
    const float* g0 = a.image_grad + ((size_t)img * M + 2 * pair) * M;
    const float* g1 = g0 + M;
    // with a gridding kernel the forward pass divided pixel (m, l) by
    // c(q_m / N) c(q_l / N); that diagonal scaling is its own adjoint
    float s0 = scale, s1 = scale;
    if (a.kw > 0) {
      s0 *= kb_inv_taper((double)(2 * pair - M / 2) / N, a);
      s1 *= kb_inv_taper((double)(2 * pair + 1 - M / 2) / N, a);
    }
    for (int l = lane; l < M; l += WAVE) {
      int q = l - M / 2;
      q = q < 0 ? q + N : q;
      const float cl = a.kw > 0 ? kb_inv_taper((double)(l - M / 2) / N, a) : 1.0f;
      z[pad(q)] = make_float2(g0[l] * s0 * cl, g1[l] * s1 * cl);
    }
    wave_sync();
    wave_fft<N, -1>(z, lane, tw);
  }
  __syncthreads();
  float4* dst = reinterpret_cast<float4*>(a.half + (size_t)li * H * M);
  for (int e = threadIdx.x; e < nz * PPW; e += blockDim.x) {
    const int k = e / PPW, p = e % PPW;
    if (p0 + p < npair) {
      const float2* z = lds + p * ST;
      const float2 zk = z[pad(k)];
      const float2 zm = z[pad(k == 0 ? 0 : N - k)];
      float4 o;
      if (k == 0) {
        o = make_float4(zk.x, 0.f, zk.y, 0.f);
      } else {  // 2 A[k] = Z[k] + conj Z[N-k]; 2 B[k] = -i (Z[k] - conj Z[N-k])
        o = make_float4(zk.x + zm.x, zk.y - zm.y, zk.y + zm.y, -(zk.x - zm.x));
      }
      dst[((size_t)k * M + 2 * (p0 + p)) / 2] = o;
    }
  }
}

// Adjoint of k_grid_cols (MODE_IMAGE): column gradient at the cutout rows,
// forward transform along v, cell weight, then gather (degrid) at every
// entry of the column: gamma'_b = w G[i_v] (direct) or conj(w G[-i_v])
// (mirror column), both for i_u = 0. Writes vis_grad = conj(g1 conj g2) gamma'
// and, with gains, gq = gamma' conj(V) for the gain gradient. Same XCD-grouped
// 1D layout and empty-column skip as the forward kernel.
// KBW (adjoint with a gridding kernel): the transformed column is written
// to a.gfull instead, for k_degrid_kb.
template <int N, bool UNI, bool KBW = false>
__global__ void __launch_bounds__(Cols<N>::THREADS) k_cols_adj(ImgArgs a) {
  extern __shared__ float4 lds_raw[];
  constexpr int H = N / 2;
  constexpr int CPW = Cols<N>::CPW;
  const int L = blockIdx.x;
  const int r8 = L >> 3;
  const int li = (r8 / a.ntiles) * 8 + (L & 7);
  const int tile = r8 % a.ntiles;
  if (li >= a.nimg) return;
  const int img = a.img0 + li;
  const int nz = min(H, a.ncz[img]);
  const int c0 = tile * CPW;
  if (c0 >= nz) return;                               // no baseline lives in this tile
  float2* lds = reinterpret_cast<float2*>(lds_raw);
  float2* ltw = lds + CPW * Cols<N>::STRIDE;
  int* lcnt = reinterpret_cast<int*>(ltw + Cols<N>::TW);
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int t = img / a.C, ch = img - t * a.C;
  const int cs = c0 + wave;
  const bool active = cs < nz;
  float2* buf = lds + wave * Cols<N>::STRIDE;
  int* cnt = UNI ? lcnt + wave * N : nullptr;
  const double s = cells_per_metre(a.freq[ch], a.ndx);
  const int M = a.M;
  const float2* tw = stage_twiddles<N>(ltw);
  __syncthreads();
  if (!active) return;
  for (int r = lane; r < Cols<N>::STRIDE; r += WAVE) buf[r] = make_float2(0.f, 0.f);
  if (UNI)
    for (int r = lane; r < N; r += WAVE) cnt[r] = 0;
  wave_sync();
  const float2* srcc = a.half + ((size_t)li * H + cs) * M;
  for (int m = lane; m < M; m += WAVE) {
    int q = m - M / 2;
    q = q < 0 ? q + N : q;
    buf[pad(q)] = srcc[m];
  }
  const int* bnd = a.bnd + (size_t)img * (N + 2);
  const int dlo = bnd[cs + H], dhi = bnd[cs + 1 + H];
  const int clo = bnd[-cs + H], chi = bnd[-cs + 1 + H];
  const size_t tb = (size_t)t * a.B;
  if (UNI) {
    for (int pass = 0; pass < 2; ++pass) {
      const int lo = pass ? clo : dlo, hi = pass ? chi : dhi;
      for (int j = lo + lane; j < hi; j += WAVE) {
        const double iv = rint(a.sv[tb + j] * s);
        if (fabs(iv) < (double)H) {
          int r = (int)iv;
          if (pass) r = -r;
          atomicAdd(&cnt[r < 0 ? r + N : r], 1);
        }
      }
    }
  }
  wave_sync();
  wave_fft<N, -1>(buf, lane, tw);
  if constexpr (KBW) {
    float2* g = a.gfull + ((size_t)li * H + cs) * N;
    for (int r = lane; r < N; r += WAVE) g[r] = buf[pad(r)];
    return;
  }
  const size_t vb = (size_t)img * a.B;
  // direct entries (and, for column 0, the conjugate entry of the same baseline)
  for (int pass = 0; pass < (cs == 0 ? 1 : 2); ++pass) {
    const int lo = pass ? clo : dlo, hi = pass ? chi : dhi;
    for (int j = lo + lane; j < hi; j += WAVE) {
      const double iv = rint(a.sv[tb + j] * s);
      if (fabs(iv) < (double)H) {
        const int r = (int)iv;
        const int rp = r < 0 ? r + N : r;
        const int rm = -r < 0 ? -r + N : -r;
        float2 g;
        if (pass == 0) {
          float2 v = buf[pad(rp)];
          if (UNI) v = cscale(v, 1.0f / (float)cnt[rp]);
          g = v;
          if (cs == 0) {
            float2 w = buf[pad(rm)];
            if (UNI) w = cscale(w, 1.0f / (float)cnt[rm]);
            g = cadd(g, cconj(w));
          }
        } else {
          float2 w = buf[pad(rm)];
          if (UNI) w = cscale(w, 1.0f / (float)cnt[rm]);
          g = cconj(w);
        }
        const int b = a.perm[tb + j];
        // gradient with respect to V' = g1 conj(g2) V: the load multiplied V' by
        // exp(+2 pi i d nu / c) (rotation, cables), so its gradient carries the conjugate
        if (a.sd != nullptr) g = rotate_phase(g, -a.sd[tb + j], a.freq[ch]);
        if (a.gains) {
          a.vis_grad[vb + b] = cmul(cconj(baseline_gain(a, b)), g);
          const float2 v = load_vis_raw(a, vb + b, ch);
          a.gamma[(size_t)li * a.B + b] = cmul(g, cconj(v));
        } else {
          a.vis_grad[vb + b] = g;
        }
      }
    }
  }
}

// Adjoint of kernel gridding: gamma'_b = sum over b's footprint cells (j, i)
// of C(i - x_u) C(j - x_v) G2[j][i], G2 = 2 Gh over the whole plane, taken
// from the transformed half-spectrum columns B in a.gfull: G2[j][i] = B[j][i]
// for i > 0 (the row pass packed both Hermitian halves there), B[j][0] +
// conj(B[-j][0]) for i = 0, conj(G2[-j][-i]) for i < 0. This is the
// direct-cell sum plus the conjugate of the mirror-cell sum (the gradient
// image is real, so its transform is Hermitian). One thread per sorted entry
// of each image of the chunk, summing in a fixed order; then the rotation and
// gain factors as in k_cols_adj. Uniform weighting divides by the entry's
// cell occupancy (a.kdens).
template <int N, int KMAX>
__global__ void __launch_bounds__(256) k_degrid_kb(ImgArgs a) {
  constexpr int H = N / 2;
  const int li = blockIdx.y;
  const int img = a.img0 + li;
  const int t = img / a.C, ch = img - t * a.C;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_valid[t]) return;
  const size_t tb = (size_t)t * a.B;
  const double s = cells_per_metre(a.freq[ch], a.ndx);
  const double hw = 0.5 * a.kw;
  const double xu = a.su[tb + j] * s, xv = a.sv[tb + j] * s;
  if (!(ceil(xu - hw) > (double)-H && floor(xu + hw) < (double)H && ceil(xv - hw) > (double)-H &&
        floor(xv + hw) < (double)H))
    return;                                          // not kept: its gradient stays zero
  const int i0 = (int)ceil(xu - hw), ni = (int)floor(xu + hw) - i0 + 1;
  const int j0 = (int)ceil(xv - hw), nj = (int)floor(xv + hw) - j0 + 1;
  float wv[KMAX + 1];
#pragma unroll
  for (int k = 0; k <= KMAX; ++k) {
    wv[k] = 0.f;
    if (k > a.kw) break;
    if (k < nj) wv[k] = kb_weight((float)((double)(j0 + k) - xv), a);
  }
  const float2* G = a.gfull + (size_t)li * H * N;
  auto at = [&](int r, int c) -> float2 {          // B[r][c], c >= 0
    return G[(size_t)c * N + (r < 0 ? r + N : r)];
  };
  float2 sum = make_float2(0.f, 0.f);
  for (int ii = 0; ii < ni; ++ii) {
    const int c = i0 + ii;
    const float wu = kb_weight((float)((double)c - xu), a);
    float2 col = make_float2(0.f, 0.f);
#pragma unroll
    for (int k = 0; k <= KMAX; ++k) {
      if (k >= nj) break;
      const int r = j0 + k;
      float2 g;
      if (c > 0) g = at(r, c);
      else if (c < 0) g = cconj(at(-r, -c));
      else g = cadd(at(r, 0), cconj(at(-r, 0)));
      col = make_float2(col.x + wv[k] * g.x, col.y + wv[k] * g.y);
    }
    sum = make_float2(sum.x + wu * col.x, sum.y + wu * col.y);
  }
  if (a.kdens != nullptr) sum = cscale(sum, 1.0f / (float)a.kdens[(size_t)li * a.B + j]);
  float2 g = sum;
  const int b = a.perm[tb + j];
  if (a.sd != nullptr) g = rotate_phase(g, -a.sd[tb + j], a.freq[ch]);
  const size_t vb = (size_t)img * a.B;
  if (a.gains) {
    a.vis_grad[vb + b] = cmul(cconj(baseline_gain(a, b)), g);
    const float2 v = load_vis_raw(a, vb + b, ch);
    a.gamma[(size_t)li * a.B + b] = cmul(g, cconj(v));
  } else {
    a.vis_grad[vb + b] = g;
  }
}

__global__ void k_fill2(float2* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_float2(0.f, 0.f);
}

// pacc[b] += sum over this chunk's images of gq[li][b]: 64 baselines per
// workgroup, 4 image slices per baseline, slices combined in a fixed order.
__global__ void __launch_bounds__(256) k_gq_reduce(ImgArgs a) {
  __shared__ float2 part[4][64];
  const int bl = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int b = blockIdx.x * 64 + bl;
  float2 acc = make_float2(0.f, 0.f);
  if (b < a.B)
    for (int li = sl; li < a.nimg; li += 4) acc = cadd(acc, a.gamma[(size_t)li * a.B + b]);
  part[sl][bl] = acc;
  __syncthreads();
  if (sl == 0 && b < a.B)
    a.pacc[b] = cadd(a.pacc[b], cadd(cadd(part[0][bl], part[1][bl]), cadd(part[2][bl], part[3][bl])));
}

// gain_grad[a] = sum_{b: a1 = a} g2 p_b + sum_{b: a2 = a} g1 conj(p_b)
__global__ void __launch_bounds__(256) k_gain_grad(ImgArgs a) {
  __shared__ float2 part[256];
  const int ant = blockIdx.x;
  float2 acc = make_float2(0.f, 0.f);
  for (int b = threadIdx.x; b < a.B; b += blockDim.x) {
    const int a1 = a.ant1[b], a2 = a.ant2[b];
    const float2 p = a.pacc[b];
    if (a1 == ant) acc = cadd(acc, cmul(antenna_gain(a.gains, a2, a.n_ant), p));
    if (a2 == ant) acc = cadd(acc, cmul(antenna_gain(a.gains, a1, a.n_ant), cconj(p)));
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] = cadd(part[threadIdx.x], part[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) a.gain_grad[ant] = part[0];
}

}  // namespace blink
