// Spreading of a jet from its time-averaged velocity, on every cross-section
// normal to the jet axis (Section 3: the width of Eq. (23) and the profile
// of Eq. (24)). The streamwise mean u is interpolated bilinearly in the
// section's two coordinates (a, b), increasing axis order; u_m is its value
// at the jet centre. Rays leave the centre at the angles 2 pi j / ndir (from
// a towards b) and are sampled at r_k = k dr, k < nr, while the sample lies
// within the section's nodes. A ray's radius r_e is the first point where u
// falls to 0.368 u_m (half the spreading width; the paper's fraction),
// interpolated linearly between the samples around it.
//
// One workgroup per section: its threads first walk the rays (one ray per
// thread and pass), then the radii (one sample radius per thread, averaged
// over all rays). The mean field is read in place; a section is a few
// hundred KB, so the repeated bilinear reads hit the caches.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace lbm {

constexpr double kSpreadFraction = 0.368;

// A cross-section family of the [3][nz][ny][nx] mean field: element strides
// of the section index p and of the in-section coordinates a and b, their
// extents and the offset of the streamwise component.
struct JetSections {
  long long sp, sa, sb, comp;
  int np, na, nb;
};

template <typename T>
__device__ __forceinline__ double jet_bilinear(const T* sec, const JetSections& s, double a,
                                               double b) {
  int i = (int)floor(a), j = (int)floor(b);
  i = i > s.na - 2 ? s.na - 2 : i;
  j = j > s.nb - 2 ? s.nb - 2 : j;
  const double fa = a - i, fb = b - j;
  const T* q = sec + i * s.sa + j * s.sb;
  return (1 - fa) * (1 - fb) * double(q[0]) + fa * (1 - fb) * double(q[s.sa]) +
         (1 - fa) * fb * double(q[s.sb]) + fa * fb * double(q[s.sa + s.sb]);
}

__device__ __forceinline__ bool jet_inside(const JetSections& s, double a, double b) {
  return a >= 0.0 && a <= s.na - 1 && b >= 0.0 && b <= s.nb - 1;
}

// um [np]; re [3][np]: minimum, maximum and mean of r_e over the rays that
// reach it (NaN if none); prof [np][nr] (or null): the mean of u(r_k) / u_m
// over the rays whose sample k lies within the section (NaN if none).
template <typename T>
__global__ __launch_bounds__(256) void jet_profile_kernel(const T* mean, const JetSections s,
                                                          double c0, double c1, int ndir,
                                                          double dr, int nr, double* um,
                                                          double* re, double* prof) {
  __shared__ double smin[256], smax[256], ssum[256];
  __shared__ int scnt[256];
  const int p = blockIdx.x, tid = threadIdx.x;
  const T* sec = mean + s.comp + p * s.sp;
  const double u0 = jet_bilinear(sec, s, c0, c1);
  const double thr = kSpreadFraction * u0;
  double lo = INFINITY, hi = -INFINITY, sum = 0.0;
  int cnt = 0;
  for (int j = tid; j < ndir; j += blockDim.x) {
    const double th = 2.0 * M_PI * j / ndir;
    const double ca = cos(th), sa = sin(th);
    double prev = u0;
    for (int k = 0; k < nr; ++k) {
      const double a = c0 + k * dr * ca, b = c1 + k * dr * sa;
      if (!jet_inside(s, a, b)) break;
      const double v = jet_bilinear(sec, s, a, b);
      if (k > 0 && v <= thr) {
        const double r = (k - 1) * dr + dr * (prev - thr) / (prev - v);
        lo = fmin(lo, r);
        hi = fmax(hi, r);
        sum += r;
        ++cnt;
        break;
      }
      prev = v;
    }
  }
  smin[tid] = lo;
  smax[tid] = hi;
  ssum[tid] = sum;
  scnt[tid] = cnt;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) {
      smin[tid] = fmin(smin[tid], smin[tid + w]);
      smax[tid] = fmax(smax[tid], smax[tid + w]);
      ssum[tid] += ssum[tid + w];
      scnt[tid] += scnt[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    um[p] = u0;
    const bool any = scnt[0] > 0;
    re[p] = any ? smin[0] : NAN;
    re[s.np + p] = any ? smax[0] : NAN;
    re[2 * s.np + p] = any ? ssum[0] / scnt[0] : NAN;
  }
  if (!prof) return;
  for (int k = tid; k < nr; k += blockDim.x) {
    double acc = 0.0;
    int n = 0;
    for (int j = 0; j < ndir; ++j) {
      const double th = 2.0 * M_PI * j / ndir;
      const double a = c0 + k * dr * cos(th), b = c1 + k * dr * sin(th);
      if (!jet_inside(s, a, b)) continue;
      acc += jet_bilinear(sec, s, a, b) / u0;
      ++n;
    }
    prof[(size_t)p * nr + k] = n ? acc / n : NAN;
  }
}

// The jet laws of Section 3 fitted to a jet_profile_kernel result over the
// sections p0 <= p < p1 downstream of the nozzle exit x0 (x = p - x0 > 0;
// NaN inputs skipped): k_par by least squares of u_m = u0 k_par d / x
// (Eq. (22)), k_perp of b_g = k_perp x with b_g the mean r_e (Eq. (23)), and
// the root mean square of prof - 0.938 exp(-0.944 (r / r_e)^2) over the
// samples r = k dr <= 2 r_e (Eq. (24)). out: k_par, k_perp, residual, the
// number of profile samples. One workgroup of 256 threads.
__global__ __launch_bounds__(256) void jet_fit_kernel(const double* um, const double* re,
                                                      const double* prof, int np, int nr,
                                                      double dr, double x0, double u0, double d,
                                                      int p0, int p1, double* out) {
  __shared__ double sh[5][256];
  __shared__ int sn[256];
  const int tid = threadIdx.x;
  double s[5] = {0, 0, 0, 0, 0};
  int n = 0;
  for (int p = p0 + tid; p < p1; p += blockDim.x) {
    const double x = p - x0;
    if (!(x > 0.0)) continue;
    if (!isnan(um[p])) {
      const double a = u0 * d / x;
      s[0] += um[p] * a;
      s[1] += a * a;
    }
    const double r_e = re[2 * np + p];
    if (isnan(r_e)) continue;
    s[2] += r_e * x;
    s[3] += x * x;
    for (int k = 0; k < nr; ++k) {
      const double r = k * dr, v = prof[(size_t)p * nr + k];
      if (r > 2.0 * r_e || isnan(v)) continue;
      const double t = r / r_e;
      const double e = v - 0.938 * exp(-0.944 * (t * t));
      s[4] += e * e;
      ++n;
    }
  }
  for (int i = 0; i < 5; ++i) sh[i][tid] = s[i];
  sn[tid] = n;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) {
      for (int i = 0; i < 5; ++i) sh[i][tid] += sh[i][tid + w];
      sn[tid] += sn[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = sh[1][0] > 0.0 ? sh[0][0] / sh[1][0] : NAN;
    out[1] = sh[3][0] > 0.0 ? sh[2][0] / sh[3][0] : NAN;
    out[2] = sn[0] > 0 ? sqrt(sh[4][0] / sn[0]) : NAN;
    out[3] = (double)sn[0];
  }
}

}  // namespace lbm
