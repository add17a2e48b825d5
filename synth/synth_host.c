/*
 * Host (CPU) bulk generator over synth/randomwalk.h.  Serves the oracle side
 * of every test and the CPU baseline; the GPU side may use the device
 * generator in synth_device.hip, which produces the same bits.
 */
#include <stdint.h>
#include <stdlib.h>

#include "randomwalk.h"

/* Series id0 .. id0+count-1 of the collection keyed by seed, row-major. */
void synth_host_randomwalk(uint64_t seed, uint64_t id0, int64_t count, int32_t len, float* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i)
    synth_randomwalk_one(seed, id0 + (uint64_t)i, len, out + i * (int64_t)len);
}

/* Noisy queries j0 .. j0+count-1 over a collection of n series keyed by
 * data_seed: each copies a uniformly drawn collection series and adds noise
 * of level sigma (round robin over 0.01, 0.1, 1.0, relative to the series'
 * own standard deviation).  Writes the source ids and sigmas if non-NULL. */
void synth_host_noisy_queries(uint64_t data_seed, uint64_t n, int32_t len, uint64_t j0,
                              int64_t count, float* out, int64_t* src_ids, double* sigmas) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) {
    uint64_t j = j0 + (uint64_t)i;
    uint64_t src = synth_noisy_source_id(j, n);
    double sigma = synth_noise_sigma(j);
    float* row = out + i * (int64_t)len;
    float* tmp = (float*)malloc(sizeof(float) * (size_t)len);
    synth_randomwalk_one(data_seed, src, len, tmp);
    synth_noisy_query(tmp, len, sigma, j, row);
    free(tmp);
    if (src_ids) src_ids[i] = (int64_t)src;
    if (sigmas) sigmas[i] = sigma;
  }
}

/* Raw draws, for tests of the generator itself. */
void synth_host_normals(uint64_t seed, uint64_t id, int64_t count, double* out) {
  synth_stream s = synth_stream_init(seed, id);
  for (int64_t i = 0; i < count; ++i) out[i] = synth_normal(&s);
}

void synth_host_uniforms(uint64_t seed, uint64_t id, int64_t count, double* out) {
  synth_stream s = synth_stream_init(seed, id);
  for (int64_t i = 0; i < count; ++i) out[i] = synth_uniform(&s);
}

double synth_host_log(double x) { return synth_log(x); }
double synth_host_sqrt(double x) { return synth_sqrt(x); }

/* Trend classes of raw series (synth_trend_class), one per row. */
void synth_host_trend_labels(const float* raw, int64_t n, int32_t len, int32_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = synth_trend_class(raw + i * len, len);
}
