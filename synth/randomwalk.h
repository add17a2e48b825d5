/*
 * Seeded synthetic inputs for the index: random-walk series and the query
 * workloads built from them (Section 5.1: a first value drawn from N(0,1),
 * then a fresh N(0,1) step added at every time point; noisy-copy queries of
 * Section 5.3: a collection series plus Gaussian noise).
 *
 * This header holds no arithmetic of the indexing method itself: no
 * z-normalisation, summarisation or distance.  It is compiled both by a C
 * host compiler and by hipcc for a bulk device generator, and both must
 * produce the same bits.  To make that hold, every step uses only IEEE
 * add, subtract, multiply and divide in a fixed order (callers compile with
 * FP contraction off); the logarithm and square root it needs are written
 * out here from their series / Newton definitions instead of calling a libm
 * whose last bit may differ between host and device.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) run as a counter-based
 * stream keyed by (seed, stream id), so any id range can be regenerated on
 * its own.  Normals: Marsaglia's polar method (Marsaglia and Bray, 1964).
 */
#ifndef SYNTH_RANDOMWALK_H
#define SYNTH_RANDOMWALK_H

#include <stdint.h>

#if defined(__HIPCC__)
#define SYNTH_FN __host__ __device__ static inline
#else
#define SYNTH_FN static inline
#endif

/* Seeds of the workloads. */
#define SYNTH_SEED_DATA 1u
#define SYNTH_SEED_QUERY 2u
#define SYNTH_SEED_NOISE 3u
#define SYNTH_SEED_MIX 4u
#define SYNTH_SEED_ARRIVAL 5u

SYNTH_FN uint64_t synth_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

typedef struct synth_stream {
  uint64_t state;
  double spare;
  int has_spare;
} synth_stream;

/* Stream keyed by (seed, id): the starting state is a hash of both. */
SYNTH_FN synth_stream synth_stream_init(uint64_t seed, uint64_t id) {
  synth_stream s;
  s.state = synth_mix64(seed * 0x9e3779b97f4a7c15ULL + 0x632be59bd9b4e019ULL) ^
            synth_mix64(id + 0xd1b54a32d192ed03ULL);
  s.spare = 0.0;
  s.has_spare = 0;
  return s;
}

SYNTH_FN uint64_t synth_next_u64(synth_stream* s) {
  s->state += 0x9e3779b97f4a7c15ULL;
  return synth_mix64(s->state);
}

/* Uniform double in (0, 1): 53 random bits, offset by half a step. */
SYNTH_FN double synth_uniform(synth_stream* s) {
  return ((double)(synth_next_u64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* Natural logarithm of x > 0 (finite, normal): x = f * 2^e with f in
 * [sqrt(1/2), sqrt(2)), ln f = 2 atanh(t), t = (f-1)/(f+1), |t| < 0.1716,
 * atanh by its odd power series to t^25 (truncation < 1e-20). */
SYNTH_FN double synth_log(double x) {
  union {
    double d;
    uint64_t u;
  } v;
  v.d = x;
  int e = (int)((v.u >> 52) & 0x7ff) - 1023;
  v.u = (v.u & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL; /* f in [1,2) */
  double f = v.d;
  if (f > 1.4142135623730951) {
    f = f * 0.5;
    e = e + 1;
  }
  double t = (f - 1.0) / (f + 1.0);
  double t2 = t * t;
  /* Horner form of 1 + t2/3 + t2^2/5 + ... + t2^12/25 */
  double p = 1.0 / 25.0;
  p = p * t2 + 1.0 / 23.0;
  p = p * t2 + 1.0 / 21.0;
  p = p * t2 + 1.0 / 19.0;
  p = p * t2 + 1.0 / 17.0;
  p = p * t2 + 1.0 / 15.0;
  p = p * t2 + 1.0 / 13.0;
  p = p * t2 + 1.0 / 11.0;
  p = p * t2 + 1.0 / 9.0;
  p = p * t2 + 1.0 / 7.0;
  p = p * t2 + 1.0 / 5.0;
  p = p * t2 + 1.0 / 3.0;
  p = p * t2 + 1.0;
  return (double)e * 0.6931471805599453 + 2.0 * t * p;
}

/* Square root of y >= 0 by Newton's iteration from an exponent-halving
 * first guess; a fixed number of steps so both compilers do the same work. */
SYNTH_FN double synth_sqrt(double y) {
  if (y <= 0.0) return 0.0;
  union {
    double d;
    uint64_t u;
  } v;
  v.d = y;
  v.u = (v.u >> 1) + 0x1ff8000000000000ULL; /* ~sqrt(y), within ~6% */
  double g = v.d;
  for (int i = 0; i < 5; ++i) g = 0.5 * (g + y / g);
  return g;
}

/* One N(0,1) draw (polar method: keeps the second value of each pair). */
SYNTH_FN double synth_normal(synth_stream* s) {
  if (s->has_spare) {
    s->has_spare = 0;
    return s->spare;
  }
  double u, v, r2;
  do {
    u = 2.0 * synth_uniform(s) - 1.0;
    v = 2.0 * synth_uniform(s) - 1.0;
    r2 = u * u + v * v;
  } while (r2 >= 1.0 || r2 == 0.0);
  double f = synth_sqrt(-2.0 * synth_log(r2) / r2);
  s->spare = v * f;
  s->has_spare = 1;
  return u * f;
}

/* Random-walk series number `id` of the collection keyed by `seed`:
 * cumulative sum in FP64 of N(0,1) draws, each point rounded to FP32. */
SYNTH_FN void synth_randomwalk_one(uint64_t seed, uint64_t id, int len, float* out) {
  synth_stream s = synth_stream_init(seed, id);
  double acc = 0.0;
  for (int t = 0; t < len; ++t) {
    acc = acc + synth_normal(&s);
    out[t] = (float)acc;
  }
}

/* Same walk, writing point t to out[t * stride] (for transposed staging). */
SYNTH_FN void synth_randomwalk_one_strided(uint64_t seed, uint64_t id, int len, float* out,
                                           int stride) {
  synth_stream s = synth_stream_init(seed, id);
  double acc = 0.0;
  for (int t = 0; t < len; ++t) {
    acc = acc + synth_normal(&s);
    out[(int64_t)t * stride] = (float)acc;
  }
}

/* Noise level of noisy query number j: round robin over {0.01, 0.1, 1.0}. */
SYNTH_FN double synth_noise_sigma(uint64_t j) {
  uint64_t r = j % 3u;
  return r == 0 ? 0.01 : (r == 1 ? 0.1 : 1.0);
}

/* Collection id that noisy query number j copies: uniform in [0, n). */
SYNTH_FN uint64_t synth_noisy_source_id(uint64_t j, uint64_t n) {
  synth_stream s = synth_stream_init(SYNTH_SEED_MIX, j);
  double u = synth_uniform(&s);
  uint64_t id = (uint64_t)(u * (double)n);
  return id < n ? id : n - 1;
}

/* Noisy query number j: the collection series `src` (length len, as
 * generated) plus N(0, (sigma * s)^2) per point, where s is the population
 * standard deviation of that series computed here in FP64.  Scaling by s
 * makes sigma the noise level relative to the series' own spread, that is,
 * on the series after it is brought to unit variance. */
SYNTH_FN void synth_noisy_query(const float* src, int len, double sigma, uint64_t j, float* out) {
  double m = 0.0;
  for (int t = 0; t < len; ++t) m = m + (double)src[t];
  m = m / (double)len;
  double v = 0.0;
  for (int t = 0; t < len; ++t) {
    double d = (double)src[t] - m;
    v = v + d * d;
  }
  double sd = synth_sqrt(v / (double)len);
  synth_stream s = synth_stream_init(SYNTH_SEED_NOISE, j);
  for (int t = 0; t < len; ++t) out[t] = (float)((double)src[t] + sigma * sd * synth_normal(&s));
}

/* Class of a series for the k-NN classification workload (the paper's
 * collections carry no classes): its trend shape, 2 [x_end > x_0] +
 * [x_mid > x_0], four classes, read off the raw generated values. */
SYNTH_FN int synth_trend_class(const float* x, int len) {
  return 2 * (x[len - 1] > x[0] ? 1 : 0) + (x[len / 2] > x[0] ? 1 : 0);
}

#endif /* SYNTH_RANDOMWALK_H */
