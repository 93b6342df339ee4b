// Probe: 1024-point column transforms of the image path (half-length
// exchange, radix 16 x 16 x 4, 512 cutout rows kept) with the first radix-16
// stage on the vector ALUs, as the library does, against the same stage as a
// matrix product on the FP32 matrix cores (v_mfma_f32_32x32x2_f32: the
// 16-point DFT in real 32 x 32 block form times the 32 x 64 real stage
// input, in two 32-column blocks). Inputs come from a small L2-resident set
// of columns so that the transform, not HBM, sets the time; prints ns per
// column and the difference between the two forms and against a direct DFT.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "blink_fft.hpp"
#include "twiddles.inc"

using namespace blink;

namespace {

constexpr int N = 1024, M = 512, CPW = 4;
constexpr int STRIDE = padded_len(N / 2);
constexpr int NTW = tw_entries(N);
constexpr int NSRC = 4096, NCOLS = 152064;   // ~ 297 columns x 512 images
typedef float v16f __attribute__((ext_vector_type(16)));

__global__ void __launch_bounds__(CPW * 64) k_valu(const float2* __restrict__ x, float2* __restrict__ out) {
  extern __shared__ float4 lds_raw[];
  float2* lds = reinterpret_cast<float2*>(lds_raw);
  float2* ltw = lds + CPW * STRIDE;
  for (int i = threadIdx.x; i < NTW; i += blockDim.x) ltw[i] = TwTable<N>::stages()[i];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  const int col = blockIdx.x * CPW + wave;
  if (col >= NCOLS) return;
  const float2* src = x + (size_t)(col % NSRC) * N;
  HalfIn<N> in;
#pragma unroll
  for (int r = 0; r < 16; ++r) in.v[0][r] = src[lane + 64 * r];
  float2* dst = out + (size_t)col * M;
  wave_fft_half_emit<N, +1>(lds + wave * STRIDE, lane, ltw, in, [&](auto qb, float2 v) {
    cutout_block_aligned<N, decltype(qb)::value>(lane, M / 2, [&](unsigned m) { store_at(dst, m, v); });
  });
}

// A operand of K step s for this lane: entry G[m][k] of the real block form
// of the 16-point DFT, m = lane % 32 (rows 0-15: real parts of the outputs,
// 16-31: imaginary parts), k = the real or imaginary part (s % 2) of input
// r = 2 (s / 2) + lane / 32.
__device__ float amat(int s, int lane) {
  const int m = lane % 32, part = s % 2, r = 2 * (s / 2) + lane / 32;
  float sn, cs;
  sincospif(2.0f * (float)(((m % 16) * r) % 16) / 16.0f, &sn, &cs);
  if (m < 16) return part == 0 ? cs : -sn;
  return part == 0 ? sn : cs;
}

__global__ void __launch_bounds__(CPW * 64) k_mfma(const float2* __restrict__ x, float2* __restrict__ out) {
  extern __shared__ float4 lds_raw[];
  float2* lds = reinterpret_cast<float2*>(lds_raw);
  float2* ltw = lds + CPW * STRIDE;
  for (int i = threadIdx.x; i < NTW; i += blockDim.x) ltw[i] = TwTable<N>::stages()[i];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  float a[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) a[s] = amat(s, lane);
  __syncthreads();
  const int col = blockIdx.x * CPW + wave;
  if (col >= NCOLS) return;
  float2* hbuf = lds + wave * STRIDE;
  const float2* src = x + (size_t)(col % NSRC) * N;
  const int h = lane / 32, c = lane % 32;
  float2 v2[1][16];
  static_for<0, 2>([&](auto cbc) {
    constexpr int cb = decltype(cbc)::value;     // butterflies j = 32 cb + c
    float2 xb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xb[q] = src[cb * 32 + c + 64 * (2 * q + h)];
    v16f d = {};
#pragma unroll
    for (int s = 0; s < 16; ++s)
      d = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], (s % 2) ? xb[s / 2].y : xb[s / 2].x, d, 0, 0, 0);
    // accumulator i holds row (i % 4) + 8 (i / 4) + 4 h of column c: output
    // k = that row (i < 8: real part, i + 8: imaginary part) of butterfly j,
    // written to y[16 j + k] of this half of the exchange buffer
#pragma unroll
    for (int i = 0; i < 8; ++i) hbuf[pad(16 * c + (i % 4) + 8 * (i / 4) + 4 * h)] = make_float2(d[i], d[i + 8]);
    wave_sync();
    half_read<N, 16, cb>(hbuf, lane, v2);
    wave_sync();
  });
  float2* dst = out + (size_t)col * M;
  half_chain<N, +1, 16>(hbuf, lane, ltw, v2, [&](auto qb, float2 v) {
    cutout_block_aligned<N, decltype(qb)::value>(lane, M / 2, [&](unsigned m) { store_at(dst, m, v); });
  });
}

template <class K>
float time_ms(K k, const float2* x, float2* out, int reps) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
  const size_t lds = (CPW * STRIDE + NTW) * sizeof(float2);
  (void)hipEventRecord(e0);
  for (int i = 0; i < reps; ++i) hipLaunchKernelGGL(k, dim3(NCOLS / CPW), dim3(CPW * 64), lds, 0, x, out);
  (void)hipEventRecord(e1);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  return ms / reps;
}

}  // namespace

int main() {
  static_assert(NCOLS % CPW == 0, "whole workgroups");
  std::vector<float2> hx((size_t)NSRC * N);
  srand(1);
  for (auto& v : hx) v = make_float2(rand() / (float)RAND_MAX - 0.5f, rand() / (float)RAND_MAX - 0.5f);
  float2 *x = nullptr, *o1 = nullptr, *o2 = nullptr;
  if (hipMalloc(&x, hx.size() * 8) != hipSuccess || hipMalloc(&o1, (size_t)NCOLS * M * 8) != hipSuccess ||
      hipMalloc(&o2, (size_t)NCOLS * M * 8) != hipSuccess)
    return 1;
  if (hipMemcpy(x, hx.data(), hx.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return 1;
  for (int i = 0; i < 200; ++i) time_ms(k_valu, x, o1, 1);          // warm the clocks
  float tv = 1e30f, tm = 1e30f;
  for (int round = 0; round < 5; ++round) {
    tv = fminf(tv, time_ms(k_valu, x, o1, 20));
    tm = fminf(tm, time_ms(k_mfma, x, o2, 20));
  }
  std::vector<float2> h1((size_t)NSRC * M), h2((size_t)NSRC * M);
  if (hipMemcpy(h1.data(), o1, h1.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(h2.data(), o2, h2.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return 1;
  double num = 0, den = 0;
  for (size_t i = 0; i < h1.size(); ++i) {
    num += (double)(h1[i].x - h2[i].x) * (h1[i].x - h2[i].x) + (double)(h1[i].y - h2[i].y) * (h1[i].y - h2[i].y);
    den += (double)h1[i].x * h1[i].x + (double)h1[i].y * h1[i].y;
  }
  double ev = 0, em = 0, ed = 0;   // column 0 against a direct DFT; output m holds frequency (m - M/2) mod N
  for (int m = 0; m < M; ++m) {
    const int q = m < M / 2 ? m + (N - M / 2) : m - M / 2;
    double sr = 0, si = 0;
    for (int n = 0; n < N; ++n) {
      const double th = 2 * M_PI * (double)((long long)q * n % N) / N;
      sr += hx[n].x * cos(th) - hx[n].y * sin(th);
      si += hx[n].x * sin(th) + hx[n].y * cos(th);
    }
    ev += (h1[m].x - sr) * (h1[m].x - sr) + (h1[m].y - si) * (h1[m].y - si);
    em += (h2[m].x - sr) * (h2[m].x - sr) + (h2[m].y - si) * (h2[m].y - si);
    ed += sr * sr + si * si;
  }
  printf("first stage on VALU: %.4f ms per %d columns (%.3f ns per column)\n", tv, NCOLS, tv * 1e6 / NCOLS);
  printf("first stage on MFMA: %.4f ms per %d columns (%.3f ns per column)\n", tm, NCOLS, tm * 1e6 / NCOLS);
  printf("MFMA / VALU time %.3f; rel-L2 MFMA vs VALU %.2e; column 0 vs direct DFT: VALU %.2e, MFMA %.2e\n",
         tm / tv, sqrt(num / den), sqrt(ev / ed), sqrt(em / ed));
  return 0;
}
