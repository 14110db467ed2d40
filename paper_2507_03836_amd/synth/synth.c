/*
 * Seeded synthetic inputs for F-Hash: time-varying scalar volumes shaped like
 * the paper's workloads (sparse moving features in a [0,1]-normalised 4D
 * field), the gradient-magnitude attribute that the production feature is
 * defined on, and the order statistic that sets its threshold value.  This
 * module holds none of the method's arithmetic (feature masks, dilation and
 * coresets are computed from these inputs by the method's own code); it only
 * produces inputs that both the HIP path and the CPU oracle consume.  Host
 * code, FP64 evaluation, FP32 storage.
 *
 * Volume layout: [T][Sz][Sy][Sx], x fastest.  Voxel (i,j,k) of any timestep
 * sits at p = (i/(Sx-1), j/(Sy-1), k/(Sz-1)); timestep n at n/(T-1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014). */
static uint64_t sm64_next(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double sm64_u01(uint64_t* s) { return (double)(sm64_next(s) >> 11) * (1.0 / 9007199254740992.0); }

uint64_t sy_splitmix64(uint64_t state) { return sm64_next(&state); }

/* Blob parameters, 8 per blob: cx, cy, cz, sigma, amplitude, vx, vy, vz. */
void sy_blob_params(uint64_t seed, int n_blobs, double sig_lo, double sig_hi, double amp_lo,
                    double amp_hi, double vmax, double* out) {
  uint64_t s = seed;
  for (int b = 0; b < n_blobs; ++b) {
    double* o = out + 8 * b;
    o[0] = sm64_u01(&s);
    o[1] = sm64_u01(&s);
    o[2] = sm64_u01(&s);
    o[3] = sig_lo + (sig_hi - sig_lo) * sm64_u01(&s);
    o[4] = amp_lo + (amp_hi - amp_lo) * sm64_u01(&s);
    o[5] = -vmax + 2.0 * vmax * sm64_u01(&s);
    o[6] = -vmax + 2.0 * vmax * sm64_u01(&s);
    o[7] = -vmax + 2.0 * vmax * sm64_u01(&s);
  }
}

/* Lattice value of 4D value noise at integer point (X,Y,Z,T), in [0,1). */
static double vn_lattice(uint64_t seed, int64_t X, int64_t Y, int64_t Z, int64_t T) {
  uint64_t h = seed;
  h ^= sy_splitmix64((uint64_t)X * 0x8CB92BA72F3D8DD7ull);
  h = sy_splitmix64(h ^ ((uint64_t)Y * 0xD6E8FEB86659FD93ull));
  h = sy_splitmix64(h ^ ((uint64_t)Z * 0xA0761D6478BD642Full));
  h = sy_splitmix64(h ^ ((uint64_t)T * 0xE7037ED1A0B428DBull));
  return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

static double smooth(double u) { return u * u * (3.0 - 2.0 * u); }

/* 4D value noise: smoothstep-weighted quadrilinear blend of lattice values. */
double sy_value_noise4(uint64_t seed, double x, double y, double z, double t) {
  double q[4] = {x, y, z, t};
  int64_t b[4];
  double w[4];
  for (int d = 0; d < 4; ++d) {
    double fl = floor(q[d]);
    b[d] = (int64_t)fl;
    w[d] = smooth(q[d] - fl);
  }
  double acc = 0.0;
  for (int c = 0; c < 16; ++c) {
    double wc = 1.0;
    for (int d = 0; d < 4; ++d) wc *= ((c >> d) & 1) ? w[d] : 1.0 - w[d];
    acc += wc * vn_lattice(seed, b[0] + (c & 1), b[1] + ((c >> 1) & 1), b[2] + ((c >> 2) & 1),
                           b[3] + ((c >> 3) & 1));
  }
  return acc;
}

/* Field: sum of advected Gaussian blobs (centre c + n v at timestep n) plus an
 * optional 3-octave turbulence term 0.25 * sum_o 2^-o VN(2^o (8x, 8y, 8z, 4t)).
 * clip01 != 0 clips to [0,1]; normalise != 0 min-max normalises the whole 4D
 * volume to [0,1] afterwards. */
void sy_field(const int64_t S[4], const double* blobs, int n_blobs, double turb_amp,
              uint64_t noise_seed, int clip01, int normalise, float* out) {
  const int64_t Sx = S[0], Sy = S[1], Sz = S[2], T = S[3];
  for (int64_t n = 0; n < T; ++n)
    for (int64_t k = 0; k < Sz; ++k)
      for (int64_t j = 0; j < Sy; ++j)
        for (int64_t i = 0; i < Sx; ++i) {
          double x = (double)i / (double)(Sx - 1), y = (double)j / (double)(Sy - 1);
          double z = (double)k / (double)(Sz - 1);
          double t = T > 1 ? (double)n / (double)(T - 1) : 0.0;
          double f = 0.0;
          for (int b = 0; b < n_blobs; ++b) {
            const double* o = blobs + 8 * b;
            double dx = x - (o[0] + n * o[5]), dy = y - (o[1] + n * o[6]);
            double dz = z - (o[2] + n * o[7]);
            f += o[4] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * o[3] * o[3]));
          }
          if (turb_amp != 0.0) {
            double s = 1.0;
            for (int oc = 0; oc < 3; ++oc) {
              f += turb_amp * s * sy_value_noise4(noise_seed + (uint64_t)oc, 8.0 * x * (1 << oc),
                                                  8.0 * y * (1 << oc), 8.0 * z * (1 << oc),
                                                  4.0 * t * (1 << oc));
              s *= 0.5;
            }
          }
          if (clip01) f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
          out[((n * Sz + k) * Sy + j) * Sx + i] = (float)f;
        }
  if (normalise) {
    int64_t N = Sx * Sy * Sz * T;
    float lo = out[0], hi = out[0];
    for (int64_t q = 1; q < N; ++q) {
      if (out[q] < lo) lo = out[q];
      if (out[q] > hi) hi = out[q];
    }
    double inv = hi > lo ? 1.0 / ((double)hi - (double)lo) : 0.0;
    for (int64_t q = 0; q < N; ++q) out[q] = (float)(((double)out[q] - lo) * inv);
  }
}

/* Gradient magnitude in voxel units: central differences inside, one-sided
 * differences on the border, per timestep. */
void sy_grad_mag(const int64_t S[4], const float* f, float* out) {
  const int64_t Sx = S[0], Sy = S[1], Sz = S[2], T = S[3];
  for (int64_t n = 0; n < T; ++n)
    for (int64_t k = 0; k < Sz; ++k)
      for (int64_t j = 0; j < Sy; ++j)
        for (int64_t i = 0; i < Sx; ++i) {
          int64_t idx[3] = {i, j, k}, ext[3] = {Sx, Sy, Sz};
          int64_t stride[3] = {1, Sx, Sx * Sy};
          int64_t base = ((n * Sz + k) * Sy + j) * Sx + i;
          double g2 = 0.0;
          for (int d = 0; d < 3; ++d) {
            double g;
            if (ext[d] < 2) g = 0.0;
            else if (idx[d] == 0) g = (double)f[base + stride[d]] - f[base];
            else if (idx[d] == ext[d] - 1) g = (double)f[base] - f[base - stride[d]];
            else g = 0.5 * ((double)f[base + stride[d]] - f[base - stride[d]]);
            g2 += g * g;
          }
          out[base] = (float)sqrt(g2);
        }
}

static int cmp_float(const void* a, const void* b) {
  float x = *(const float*)a, y = *(const float*)b;
  return (x > y) - (x < y);
}

/* q-th quantile as an order statistic: the element of rank floor(q * N) of the
 * ascending sort (0-based). */
float sy_quantile(const float* v, int64_t N, double q) {
  float* c = (float*)malloc(sizeof(float) * (size_t)N);
  memcpy(c, v, sizeof(float) * (size_t)N);
  qsort(c, (size_t)N, sizeof(float), cmp_float);
  int64_t r = (int64_t)floor(q * (double)N);
  if (r >= N) r = N - 1;
  float out = c[r];
  free(c);
  return out;
}
