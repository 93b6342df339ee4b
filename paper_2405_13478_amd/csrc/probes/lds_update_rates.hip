// Probe: cost of one wave64 update of 64 LDS words on gfx950, by the form of
// the update. Each of 8 wavefronts per workgroup updates two words per lane
// per iteration in its own 4 KiB LDS region (consecutive addresses), 4
// workgroups per CU; prints CU cycles (at 2.4 GHz) per wave-level update.
// Used to choose how the column kernels accumulate gridded visibilities.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int WAVES = 8, WORDS = 1024, ITERS = 2000, BLOCKS = 256 * 4;

template <int MODE>
__global__ void __launch_bounds__(WAVES * 64) k_update(float* out, int iters) {
  __shared__ unsigned long long buf64[WAVES][WORDS / 2];
  __shared__ float buf[WAVES][WORDS];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (int i = threadIdx.x; i < WAVES * WORDS; i += blockDim.x) (&buf[0][0])[i] = 0.f;
  for (int i = threadIdx.x; i < WAVES * WORDS / 2; i += blockDim.x) (&buf64[0][0])[i] = 0;
  __syncthreads();
  for (int it = 0; it < iters; ++it) {
    if (MODE == 0) {            // LDS float atomic add (ds_add_f32)
      atomicAdd(&buf[w][lane], 1.0f);
      atomicAdd(&buf[w][lane + 512], 2.0f);
    } else if (MODE == 1) {     // LDS integer atomic add (ds_add_u32)
      atomicAdd(reinterpret_cast<unsigned*>(&buf[w][lane]), 1u);
      atomicAdd(reinterpret_cast<unsigned*>(&buf[w][lane + 512]), 2u);
    } else if (MODE == 2) {     // LDS integer atomic max (ds_max_u32)
      atomicMax(reinterpret_cast<unsigned*>(&buf[w][lane]), (unsigned)it);
      atomicMax(reinterpret_cast<unsigned*>(&buf[w][lane + 512]), (unsigned)it);
    } else if (MODE == 3) {     // 64-bit integer atomic add (ds_add_u64)
      atomicAdd(&buf64[w][lane], 1ull);
      atomicAdd(&buf64[w][lane + 256], 2ull);
    } else {                    // plain read-modify-write of wavefront-private words
      const float x = buf[w][lane], y = buf[w][lane + 512];
      buf[w][lane] = x + 1.0f;
      buf[w][lane + 512] = y + 2.0f;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
  out[blockIdx.x * blockDim.x + threadIdx.x] = buf[w][lane] + (float)buf64[w][lane % (WORDS / 2)];
}

template <int MODE>
int run(float* out, const char* name) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  hipLaunchKernelGGL(k_update<MODE>, dim3(BLOCKS), dim3(WAVES * 64), 0, 0, out, 10);
  if (hipEventRecord(e0) != hipSuccess) return 1;
  hipLaunchKernelGGL(k_update<MODE>, dim3(BLOCKS), dim3(WAVES * 64), 0, 0, out, ITERS);
  if (hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1;
  const double updates = (double)BLOCKS * WAVES * ITERS * 2;
  printf("%-34s %8.3f ms  %7.2f CU cycles per wave64 update\n", name, ms, ms * 1e-3 * 2.4e9 * 256 / updates);
  return 0;
}

}  // namespace

int main() {
  float* out = nullptr;
  if (hipMalloc(&out, (size_t)BLOCKS * WAVES * 64 * sizeof(float)) != hipSuccess) return 1;
  int e = run<0>(out, "(warm-up)");
  e |= run<0>(out, "ds_add_f32 (float atomic add)");
  e |= run<1>(out, "ds_add_u32 (integer atomic add)");
  e |= run<2>(out, "ds_max_u32 (integer atomic max)");
  e |= run<3>(out, "ds_add_u64 (64-bit atomic add)");
  e |= run<4>(out, "ds_read + add + ds_write (private)");
  return e;
}
