/*
 * Device bulk generator over synth/randomwalk.h: the same series as
 * synth_host_randomwalk, bit for bit, written straight into device memory
 * so that collections of 10^8 series need no host round trip.
 *
 * One thread per series; a block of 64 series is staged in LDS (row stride
 * len+1 floats, so the 64 lanes writing point t hit distinct banks) and then
 * written out row-major with consecutive lanes on consecutive addresses.
 * Series longer than 512 points are written row by row from registers.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "randomwalk.h"

#define SYNTH_BLOCK 64
#define SYNTH_MAX_LEN 512

__global__ __launch_bounds__(SYNTH_BLOCK) void synth_randomwalk_kernel(uint64_t seed, uint64_t id0,
                                                                       int64_t count, int len,
                                                                       float* __restrict__ out) {
  __shared__ float tile[SYNTH_BLOCK * (SYNTH_MAX_LEN + 1)];
  const int stride = len + 1;
  const int64_t first = (int64_t)blockIdx.x * SYNTH_BLOCK;
  const int64_t mine = first + threadIdx.x;
  if (mine < count) synth_randomwalk_one_strided(seed, id0 + (uint64_t)mine, len, tile + threadIdx.x * stride, 1);
  __syncthreads();
  const int64_t rows = (count - first) < SYNTH_BLOCK ? (count - first) : SYNTH_BLOCK;
  const int64_t total = rows * len;
  float* base = out + first * (int64_t)len;
  for (int64_t e = threadIdx.x; e < total; e += SYNTH_BLOCK) {
    int r = (int)(e / len);
    int c = (int)(e - (int64_t)r * len);
    base[e] = tile[r * stride + c];
  }
}

/* Longer series: one thread per series writing its own row directly (the
 * writes are strided, which only costs generation speed). */
__global__ __launch_bounds__(SYNTH_BLOCK) void synth_randomwalk_rows_kernel(uint64_t seed, uint64_t id0,
                                                                            int64_t count, int len,
                                                                            float* __restrict__ out) {
  const int64_t mine = (int64_t)blockIdx.x * SYNTH_BLOCK + threadIdx.x;
  if (mine < count) synth_randomwalk_one(seed, id0 + (uint64_t)mine, len, out + mine * (int64_t)len);
}

/* Returns 0 on success, -1 on bad arguments, -3 on a launch error. */
extern "C" int synth_dev_randomwalk(uint64_t seed, uint64_t id0, int64_t count, int32_t len,
                                    float* dev_out, void* stream) {
  if (count < 0 || len < 1 || (count > 0 && dev_out == nullptr)) return -1;
  if (count == 0) return 0;
  const int64_t blocks = (count + SYNTH_BLOCK - 1) / SYNTH_BLOCK;
  if (len <= SYNTH_MAX_LEN)
    hipLaunchKernelGGL(synth_randomwalk_kernel, dim3((unsigned)blocks), dim3(SYNTH_BLOCK), 0,
                       (hipStream_t)stream, seed, id0, count, (int)len, dev_out);
  else
    hipLaunchKernelGGL(synth_randomwalk_rows_kernel, dim3((unsigned)blocks), dim3(SYNTH_BLOCK), 0,
                       (hipStream_t)stream, seed, id0, count, (int)len, dev_out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

__global__ void synth_trend_labels_kernel(const float* __restrict__ raw, int64_t n, int len,
                                          int* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = synth_trend_class(raw + i * len, len);
}

/* Trend classes of raw device series into a device int32 array [n]. */
extern "C" int synth_dev_trend_labels(const float* dev_raw, int64_t n, int32_t len, int32_t* dev_out,
                                      void* stream) {
  if (n < 0 || len < 1 || (n > 0 && (dev_raw == nullptr || dev_out == nullptr))) return -1;
  if (n == 0) return 0;
  hipLaunchKernelGGL(synth_trend_labels_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, dev_raw, n, (int)len, dev_out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
