// C ABI of the CBS solver: plans, setup kernels, the iteration loop,
// adjoint source, gradient and the Green's-operator entry point.
//
// The operation each entry point performs is specified in include/cbs.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <chrono>
#include <climits>
#include <complex>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/cbs.h"
#include "kernels.hpp"
#include "scpml.hpp"

namespace cbs {

const SizeOps* sizes_small(int* count);
const SizeOps* sizes_mid(int* count);
const SizeOps* sizes_large(int* count);

const SizeOps* find_size(int n) {
  const SizeOps* (*tables[])(int*) = {sizes_small, sizes_mid, sizes_large};
  for (auto tab : tables) {
    int cnt = 0;
    const SizeOps* t = tab(&cnt);
    for (int i = 0; i < cnt; ++i)
      if (t[i].n == n) return &t[i];
  }
  return nullptr;
}

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(call)                                                               \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) return fail(CBS_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define HIP_LAUNCHED()                                                              \
  do {                                                                              \
    hipError_t e_ = hipGetLastError();                                              \
    if (e_ != hipSuccess) return fail(CBS_E_HIP, "kernel launch: %s", hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// setup and small kernels
// ---------------------------------------------------------------------------
constexpr int kSetupBlocks = 1024;
constexpr int kSetupThreads = 256;

struct SetupArgs {
  int nx, ny, nz, px, py, pz, order, dtype;
  double sigma_max, k0d2, kbd2, nb2;
  float nb2f;
  const void* eps;
  float2* V0;
  double* part;  // 2 per block: max|V0|, flags
};

__device__ __forceinline__ double layer_depth(int i, int n, int p) {
  if (p <= 0) return 0.0;
  if (i < p) return double(p - i) / double(p);
  if (i >= n - p) return double(i - (n - p - 1)) / double(p);
  return 0.0;
}

__device__ __forceinline__ double ipow(double u, int m) {
  double r = 1.0;
  for (int k = 0; k < m; ++k) r *= u;
  return r;
}

// sigma, V0 = k0^2 (eps_r - n_bg^2) + i kb^2 sigma (times d^2), max|V0| in
// FP64 and input validation flags (1 non-finite, 2 gain, 4 layer != n_bg^2)
__global__ void __launch_bounds__(kSetupThreads) k_setup(SetupArgs a) {
  __shared__ double smx[kSetupThreads / 64];
  __shared__ unsigned sfl[kSetupThreads / 64];
  const long long N = (long long)a.nx * a.ny * a.nz;
  double mx = 0.0;
  unsigned fl = 0;
  for (long long i = (long long)blockIdx.x * kSetupThreads + threadIdx.x; i < N;
       i += (long long)gridDim.x * kSetupThreads) {
    const int x = (int)(i % a.nx);
    const long long r = i / a.nx;
    const int y = (int)(r % a.ny);
    const int z = (int)(r / a.ny);
    float er, ei;
    if (a.dtype == CBS_F32) {
      er = static_cast<const float*>(a.eps)[i];
      ei = 0.f;
    } else {
      const float2 e = static_cast<const float2*>(a.eps)[i];
      er = e.x;
      ei = e.y;
    }
    if (!isfinite(er) || !isfinite(ei)) fl |= 1u;
    if (ei < 0.f) fl |= 2u;
    const bool layer = x < a.px || x >= a.nx - a.px || y < a.py || y >= a.ny - a.py ||
                       z < a.pz || z >= a.nz - a.pz;
    if (layer && (er != a.nb2f || ei != 0.f)) fl |= 4u;
    const double su = ipow(layer_depth(x, a.nx, a.px), a.order) +
                      ipow(layer_depth(y, a.ny, a.py), a.order) +
                      ipow(layer_depth(z, a.nz, a.pz), a.order);
    const double sigma = a.sigma_max * (su < 1.0 ? su : 1.0);
    const double vr = a.k0d2 * ((double)er - a.nb2);
    const double vi = a.k0d2 * (double)ei + a.kbd2 * sigma;
    const double m = sqrt(vr * vr + vi * vi);
    mx = m > mx ? m : mx;
    a.V0[i] = make_float2((float)vr, (float)vi);
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double om = __shfl_xor(mx, o, 64);
    mx = om > mx ? om : mx;
    fl |= (unsigned)__shfl_xor((int)fl, o, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    smx[wv] = mx;
    sfl[wv] = fl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kSetupThreads / 64; ++w) {
      mx = smx[w] > smx[0] ? smx[w] : smx[0];
      smx[0] = mx;
      sfl[0] |= sfl[w];
    }
    a.part[2 * blockIdx.x] = smx[0];
    a.part[2 * blockIdx.x + 1] = (double)sfl[0];
  }
}

__global__ void k_state_init(DevState* st, double tol, int max_iter, int record) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->done = 0;
    st->iter = 0;
    st->status = 0;
    st->max_iter = max_iter;
    st->tol = tol;
    st->eta = INFINITY;
    st->record = record;
    st->pending = 0;
  }
}

// point-source amplitude: conj(E(r0)) * scale (from_field) or given * scale
__global__ void k_point_amp(DevState* st, const float2* E, long long idx, long long sE,
                            int from_field, float scale, float2 g0, float2 g1, float2 g2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (from_field) {
      for (int c = 0; c < 3; ++c) {
        const float2 e = E[c * sE + idx];
        st->amp[c] = make_float2(e.x * scale, -e.y * scale);
      }
    } else {
      st->amp[0] = make_float2(g0.x * scale, g0.y * scale);
      st->amp[1] = make_float2(g1.x * scale, g1.y * scale);
      st->amp[2] = make_float2(g2.x * scale, g2.y * scale);
    }
  }
}

// eta = sqrt(sum |dE|^2 / sum |E|^2) over the K1 block partials (fixed order);
// a separate launch when the x-pass does not fold it in
constexpr int kResThreads = 256;
__global__ void __launch_bounds__(kResThreads)
k_residual(const double* part, int per_b, int nb, DevState* st, double* hist) {
  __shared__ double red[2 * kResStreams];
  if (st->done || !st->pending) return;
  residual_finish<kResThreads>(part, per_b, nb, st, hist, red);
  if (threadIdx.x == 0) st->pending = 0;
}

// E_b += sign * pol_b exp(i k_b . r) for every illumination b of a solve
// (the incident plane waves; normal incidence: pol exp(i kb z))
__global__ void k_incident(CbsArgs a, float sign) {
  const long long N = (long long)a.nx * a.ny * a.nz;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx);
    const int y = (int)((i / a.nx) % a.ny);
    const int z = (int)(i / ((long long)a.nx * a.ny));
    for (int b = 0; b < a.nb; ++b) {
      const float2 pxy = a.oblique ? cmul(a.phy[b * a.ny + y], a.phx[b * a.nx + x])
                                   : make_float2(1.f, 0.f);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float2 pz = a.phase[(b * 3 + c) * a.nz + z];
        const float2 inc = a.oblique ? cmul(pz, pxy) : pz;
        float2* ep = a.E + b * a.sEb + c * a.sE + i;
        float2 e = *ep;
        e.x += sign * inc.x;
        e.y += sign * inc.y;
        *ep = e;
      }
    }
  }
}

// Plane-wave tables of the illuminations of a solve, in FP64 rounded to FP32:
// phx[b][x] = exp(i kx_b d x), phy[b][y] = exp(i ky_b d y) and
// phz[b][c][z] = pol_{b,c} exp(i kz_b d z); phase zero at the voxel (0, 0, 0).
struct Kvec {
  int nb;
  double kd[kMaxIllum][3];       // (kx, ky, kz) d of each illumination
  double pol[kMaxIllum][3][2];   // polarisation (re, im)
};
__global__ void k_phase_tables(float2* phx, float2* phy, float2* phz, int nx, int ny, int nz,
                               Kvec kv) {
  const int per = nx + ny + 3 * nz;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kv.nb * per; i += gridDim.x * blockDim.x) {
    const int b = i / per, j = i - b * per;
    double sn, cs;
    if (j < nx) {
      sincos(kv.kd[b][0] * (double)j, &sn, &cs);
      phx[b * nx + j] = make_float2((float)cs, (float)sn);
    } else if (j < nx + ny) {
      const int k = j - nx;
      sincos(kv.kd[b][1] * (double)k, &sn, &cs);
      phy[b * ny + k] = make_float2((float)cs, (float)sn);
    } else {
      const int m = j - nx - ny, c = m / nz, k = m - c * nz;
      sincos(kv.kd[b][2] * (double)k, &sn, &cs);
      const double pr = kv.pol[b][c][0], pi = kv.pol[b][c][1];
      phz[(b * 3 + c) * nz + k] = make_float2((float)(pr * cs - pi * sn), (float)(pr * sn + pi * cs));
    }
  }
}

// grad[z][y][x] = scale * Re(sum_c Ea_c E_c) over the box (FP64 accumulate)
__global__ void k_gradient(const float2* E, const float2* Ea, long long sE, int nx, int ny,
                           int x0, int y0, int z0, int bx, int by, int bz, double scale,
                           float* grad) {
  const long long NB = (long long)bx * by * bz;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < NB;
       i += (long long)gridDim.x * blockDim.x) {
    const int xi = (int)(i % bx);
    const long long r = i / bx;
    const int yi = (int)(r % by);
    const int zi = (int)(r / by);
    const long long idx = ((long long)(z0 + zi) * ny + (y0 + yi)) * nx + (x0 + xi);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float2 e = E[c * sE + idx], ea = Ea[c * sE + idx];
      s += (double)ea.x * (double)e.x - (double)ea.y * (double)e.y;
    }
    grad[i] = (float)(scale * s);
  }
}

// ---------------------------------------------------------------------------
// lens metrics: focus search, line profiles, disc power (FP64 reductions)
// ---------------------------------------------------------------------------
constexpr int kMetricBlocks = 256;
constexpr int kMetricThreads = 256;

__device__ __forceinline__ double intensity(const float2* E, long long sE, long long idx) {
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float2 e = E[c * sE + idx];
    s += (double)e.x * (double)e.x + (double)e.y * (double)e.y;
  }
  return s;
}

// Per-block maximum of |E|^2 over a box with its linear voxel index; ties go
// to the smaller index, so the result does not depend on the launch shape.
__global__ void __launch_bounds__(kMetricThreads)
k_argmax_intensity(const float2* E, long long sE, int nx, int ny, int x0, int y0, int z0, int bx,
                   int by, int bz, double* part) {
  __shared__ double sv[kMetricThreads];
  __shared__ long long si[kMetricThreads];
  double best = -1.0;
  long long bi = 0x7fffffffffffffffLL;
  const long long NB = (long long)bx * by * bz;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < NB;
       i += (long long)gridDim.x * blockDim.x) {
    const int xi = (int)(i % bx);
    const long long r = i / bx;
    const int yi = (int)(r % by);
    const int zi = (int)(r / by);
    const long long idx = ((long long)(z0 + zi) * ny + (y0 + yi)) * nx + (x0 + xi);
    const double s = intensity(E, sE, idx);
    if (s > best || (s == best && idx < bi)) {
      best = s;
      bi = idx;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = kMetricThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const double v = sv[threadIdx.x + o];
      const long long j = si[threadIdx.x + o];
      if (v > sv[threadIdx.x] || (v == sv[threadIdx.x] && j < si[threadIdx.x])) {
        sv[threadIdx.x] = v;
        si[threadIdx.x] = j;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sv[0];
    part[2 * blockIdx.x + 1] = (double)si[0];
  }
}

// |E|^2 along the x, y and z lines through (fx, fy, fz): out[0, nx) then
// out[nx, nx + ny) then out[nx + ny, nx + ny + nz).
__global__ void k_line_intensity(const float2* E, long long sE, int nx, int ny, int nz, int fx,
                                 int fy, int fz, double* out) {
  const int n = nx + ny + nz;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int x = fx, y = fy, z = fz;
    if (i < nx) x = i;
    else if (i < nx + ny) y = i - nx;
    else z = i - nx - ny;
    out[i] = intensity(E, sE, ((long long)z * ny + y) * nx + x);
  }
}

// The transverse field of plane fz in FP64: ex, ey [ny][nx].
__global__ void k_plane_extract(const float2* E, long long sE, int nx, int ny, int fz,
                                double2* ex, double2* ey) {
  const long long NP = (long long)nx * ny;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < NP;
       i += (long long)gridDim.x * blockDim.x) {
    const float2 a = E[(long long)fz * NP + i], b = E[sE + (long long)fz * NP + i];
    ex[i] = make_double2(a.x, a.y);
    ey[i] = make_double2(b.x, b.y);
  }
}

// One pass of a plane DFT in FP64, out-of-place: along x (axis 0) or y
// (axis 1) of an [ny][nx] plane, out[k] = sum_j in[j] w^(sign j k), with
// w = tw[m] = exp(-2 pi i m / n) (sign -1: forward, +1: inverse, unscaled).
// Direct sums: the planes are small and this runs once per measurement.
__global__ void k_plane_dft(const double2* in, double2* out, int nx, int ny, int axis, int sign,
                            const double2* tw) {
  const long long NP = (long long)nx * ny;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < NP;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % nx), y = (int)(i / nx);
    const int n = axis == 0 ? nx : ny;
    const int k = axis == 0 ? x : y;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < n; ++j) {
      const double2 v = axis == 0 ? in[(long long)y * nx + j] : in[(long long)j * nx + x];
      const double2 w = tw[(int)(((long long)j * k) % n)];
      const double wi = sign < 0 ? w.y : -w.y;
      re += v.x * w.x - v.y * wi;
      im += v.x * wi + v.y * w.x;
    }
    out[i] = make_double2(re, im);
  }
}

// Angular spectrum of the transverse field -> propagating part of E and the
// magnetic field in units where a plane wave has H = z x E:
//   kz = sqrt(k^2 - kx^2 - ky^2) (evanescent components dropped),
//   Ez = -(kx Ex + ky Ey) / kz,  H = k_vec x E / k.
__global__ void k_angular_h(double2* ax, double2* ay, double2* hx, double2* hy, int nx, int ny,
                            double dkx, double dky, double k) {
  const long long NP = (long long)nx * ny;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < NP;
       i += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(i % nx), iy = (int)(i / nx);
    const double kx = dkx * (ix < (nx + 1) / 2 ? ix : ix - nx);
    const double ky = dky * (iy < (ny + 1) / 2 ? iy : iy - ny);
    const double kz2 = k * k - kx * kx - ky * ky;
    if (kz2 <= 0.0) {
      ax[i] = ay[i] = hx[i] = hy[i] = make_double2(0.0, 0.0);
      continue;
    }
    const double kz = sqrt(kz2);
    const double2 ex = ax[i], ey = ay[i];
    const double2 ez = make_double2(-(kx * ex.x + ky * ey.x) / kz, -(kx * ex.y + ky * ey.y) / kz);
    hx[i] = make_double2((ky * ez.x - kz * ey.x) / k, (ky * ez.y - kz * ey.y) / k);
    hy[i] = make_double2((kz * ex.x - kx * ez.x) / k, (kz * ex.y - kx * ez.y) / k);
  }
}

// Per-block sums of S_z = Re(Ex conj(Hy) - Ey conj(Hx)) (times scale) over the
// voxels of the plane whose centres lie within sqrt(r2) voxels of (cx, cy).
__global__ void __launch_bounds__(kMetricThreads)
k_disc_flux(const double2* ex, const double2* ey, const double2* hx, const double2* hy, int nx,
            int ny, double cx, double cy, double r2, double scale, double* part) {
  __shared__ double sh[kMetricThreads];
  double acc = 0.0;
  const long long NP = (long long)nx * ny;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < NP;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % nx), y = (int)(i / nx);
    const double dx = x - cx, dy = y - cy;
    if (dx * dx + dy * dy <= r2) {
      const double2 a = ex[i], b = ey[i], u = hx[i], v = hy[i];
      acc += (a.x * v.x + a.y * v.y) - (b.x * u.x + b.y * u.y);
    }
  }
  sh[threadIdx.x] = acc * scale;
  __syncthreads();
  for (int o = kMetricThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// ---------------------------------------------------------------------------
// total-field / scattered-field source: S = (L - K_bg)(chi E_inc)
// ---------------------------------------------------------------------------
// chi is the indicator of a box and E_inc = q exp(i k.r), so chi E_inc = q u
// with u = fx(x) fy(y) fz(z), f_a(i) = chi_a(i) exp(i k_a d i), and every term
// of L (q u) = F^-1 [ |p|^2 q u^ - pt (pt . q) u^ ] is a product of 1D
// transforms of the f_a.  Per axis the tables hold (FP64, n_a entries each,
// axes one after the other):
//   tab[0] = f,  tab[1] = F f (spectrum),  tab[2] = F^-1[p^2 F f],
//   tab[3] = F^-1[pt F f],  tab[4] = F^-1[pt^2 F f]   (p in 1/m; pt = p except
// 0 at the Nyquist bin of an even axis), by direct O(n^2) sums.
struct TfsfArgs {
  int n[3], lo[3], hi[3], off[3];   // axis lengths, box, table offsets
  int ntot;                         // n[0] + n[1] + n[2]
  double kd[3];                     // (kx, ky, kz) d of the plane wave
  double pitch;
  double2* tab;                     // 5 ntot entries
};

__device__ __forceinline__ int tfsf_axis(const TfsfArgs& t, int j, int& i) {
  const int a = j < t.n[0] ? 0 : (j < t.n[0] + t.n[1] ? 1 : 2);
  i = j - t.off[a];
  return a;
}

// f and its DFT (one thread per axis entry)
__global__ void k_tfsf_forward(TfsfArgs t) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < t.ntot; j += gridDim.x * blockDim.x) {
    int m;
    const int a = tfsf_axis(t, j, m);
    const int n = t.n[a];
    double re = 0.0, im = 0.0;
    for (int i = t.lo[a]; i < t.hi[a]; ++i) {   // f vanishes outside the box
      double sf, cf, sw, cw;
      sincos(t.kd[a] * (double)i, &sf, &cf);
      sincos(-2.0 * M_PI * (double)(((long long)m * i) % n) / (double)n, &sw, &cw);
      re += cf * cw - sf * sw;
      im += cf * sw + sf * cw;
    }
    t.tab[t.ntot + j] = make_double2(re, im);
    double sf = 0.0, cf = 0.0;
    if (m >= t.lo[a] && m < t.hi[a]) sincos(t.kd[a] * (double)m, &sf, &cf);
    t.tab[j] = make_double2(cf, sf);
  }
}

// the three filtered inverse transforms (one thread per axis entry)
__global__ void k_tfsf_inverse(TfsfArgs t) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < t.ntot; j += gridDim.x * blockDim.x) {
    int i;
    const int a = tfsf_axis(t, j, i);
    const int n = t.n[a];
    double r2 = 0.0, i2 = 0.0, r1 = 0.0, i1 = 0.0, rt = 0.0, it = 0.0;
    for (int m = 0; m < n; ++m) {
      const double2 F = t.tab[t.ntot + t.off[a] + m];
      const int mm = (m < (n + 1) / 2) ? m : m - n;
      const double pm = 2.0 * M_PI * (double)mm / ((double)n * t.pitch);
      const double ptm = ((n & 1) == 0 && 2 * m == n) ? 0.0 : pm;
      double sw, cw;
      sincos(2.0 * M_PI * (double)(((long long)m * i) % n) / (double)n, &sw, &cw);
      const double gr = F.x * cw - F.y * sw, gi = F.x * sw + F.y * cw;   // F(m) e^{+2 pi i m i/n}
      r2 += pm * pm * gr;
      i2 += pm * pm * gi;
      r1 += ptm * gr;
      i1 += ptm * gi;
      rt += ptm * ptm * gr;
      it += ptm * ptm * gi;
    }
    const double inv = 1.0 / (double)n;
    t.tab[2 * t.ntot + j] = make_double2(r2 * inv, i2 * inv);
    t.tab[3 * t.ntot + j] = make_double2(r1 * inv, i1 * inv);
    t.tab[4 * t.ntot + j] = make_double2(rt * inv, it * inv);
  }
}

// zmul: complex FP64 product (scpml.hpp)
__device__ __forceinline__ double2 zmul3(double2 a, double2 b, double2 c) {
  return zmul(zmul(a, b), c);
}

struct TfsfAssemble {
  TfsfArgs t;
  int nx, ny, nz, px, py, pz, order;
  double sigma_max, kb2;
  double2 q[3];          // polarisation
  float2* S;             // [3][nz][ny][nx]
};

// S_c = q_c (D2x fy fz + fx D2y fz + fx fy D2z - kb^2 (1 + i sigma) u)
//       - sum_b q_b T_c T_b u   (T_c T_b u = (T1 f)(T1 f)(f) for c != b, (T2 f)(f)(f) for c = b)
__global__ void k_tfsf_assemble(TfsfAssemble A) {
  const TfsfArgs& t = A.t;
  const long long N = (long long)A.nx * A.ny * A.nz;
  const double2* f = t.tab;
  const double2* d2 = t.tab + 2 * t.ntot;
  const double2* t1 = t.tab + 3 * t.ntot;
  const double2* t2 = t.tab + 4 * t.ntot;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % A.nx);
    const int y = (int)((i / A.nx) % A.ny);
    const int z = (int)(i / ((long long)A.nx * A.ny));
    const int ix = t.off[0] + x, iy = t.off[1] + y, iz = t.off[2] + z;
    const double2 u = zmul3(f[ix], f[iy], f[iz]);
    const double su = ipow(layer_depth(x, A.nx, A.px), A.order) +
                      ipow(layer_depth(y, A.ny, A.py), A.order) +
                      ipow(layer_depth(z, A.nz, A.pz), A.order);
    const double sigma = A.sigma_max * (su < 1.0 ? su : 1.0);
    const double2 kbg = make_double2(A.kb2, A.kb2 * sigma);
    const double2 lap = make_double2(
        zmul3(d2[ix], f[iy], f[iz]).x + zmul3(f[ix], d2[iy], f[iz]).x + zmul3(f[ix], f[iy], d2[iz]).x,
        zmul3(d2[ix], f[iy], f[iz]).y + zmul3(f[ix], d2[iy], f[iz]).y + zmul3(f[ix], f[iy], d2[iz]).y);
    const double2 diag = make_double2(lap.x - zmul(kbg, u).x, lap.y - zmul(kbg, u).y);
    // T_c T_b u for the 3 x 3 pairs
    const int idx[3] = {ix, iy, iz};
    double2 tt[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        double2 v;
        if (c == b) {
          v = t2[idx[c]];
        } else {
          v = zmul(t1[idx[c]], t1[idx[b]]);
        }
        const int o = 3 - c - b;   // the remaining axis when c != b
        if (c == b) {
          const int o1 = (c + 1) % 3, o2 = (c + 2) % 3;
          v = zmul3(v, f[idx[o1]], f[idx[o2]]);
        } else {
          v = zmul(v, f[idx[o]]);
        }
        tt[c][b] = v;
      }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double2 sc = zmul(A.q[c], diag);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double2 w = zmul(A.q[b], tt[c][b]);
        sc.x -= w.x;
        sc.y -= w.y;
      }
      A.S[c * N + i] = make_float2((float)sc.x, (float)sc.y);
    }
  }
}

// streaming copy: one float4 per thread over a grid that covers the buffer
// (the fastest plain copy form measured on this part)
constexpr int kCopyThreads = 256;
__global__ void __launch_bounds__(kCopyThreads)
k_copy(const float4* __restrict__ src, float4* __restrict__ dst, long long n4) {
  const long long i = (long long)blockIdx.x * kCopyThreads + threadIdx.x;
  if (i < n4) dst[i] = src[i];
}

}  // namespace cbs

using namespace cbs;

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct cbs_plan_s {
  int nx, ny, nz, nxp;
  int pml[3];
  double pitch, lambda0, n_bg, k0, kb;
  int order;
  double sigma_max;
  double shift_factor;
  const SizeOps *ox, *oy, *oz;
  int k1_blocks;
  hipStream_t stream;
  // workspace carve-up
  float2 *W, *V0, *twx, *twy, *twz, *phase, *phx, *phy;
  double *partials, *setup_part, *hist, *metrics;
  DevState* state;
  bool have_eps;
  double eps;  // 1/m^2
  int hist_len;
  hipEvent_t ev0, ev1;
  hipEvent_t evp[6];
  // asynchronous solve in progress (cbs_solve_begin .. cbs_solve_end)
  struct Active {
    bool on;        // begun and not ended
    bool stopped;   // device reported the stop; later launches are no-ops
    bool plane;     // plane-wave source: E_inc is added at the end
    unsigned flags;
    int max_iter;
    int enqueued;   // iterations enqueued so far
    int head, count;  // ring of outstanding quanta
    float ms;       // device time from begin to the quantum that stopped
    CbsArgs args;
  } act;
  static constexpr int kRing = 4;
  hipEvent_t evq[kRing];
  DevState* mirror;  // pinned host copies of the device state, one per quantum slot
  DevState last;     // state read at the last completed quantum
};

// The workspace of cbs_solve_static: one plan's scratch in a static device
// array, held by each GPU the library runs on until the process ends.  In host
// code cbs_scratch names a host-side stand-in; its device address comes from
// hipGetSymbolAddress, once per device (static_scratch below), and only that
// address is ever passed to a kernel or a copy.
static __device__ __align__(256) unsigned char cbs_scratch[CBS_STATIC_SCRATCH_BYTES];

namespace {

struct Layout {
  size_t W, V0, twx, twy, twz, phase, phx, phy, partials, setup, hist, metrics, state, total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int padded_pitch(int nx) { return (nx + kBrick - 1) / kBrick * kBrick; }

bool layout_of(int nx, int ny, int nz, Layout& L) {
  const SizeOps* ox = find_size(nx);
  if (!ox) return false;
  const long long N = (long long)nx * ny * nz;
  const long long k1b = 3LL * ((ny + ox->k1_rows - 1) / ox->k1_rows) * nz;   // x-pass blocks
  const size_t c8 = sizeof(float2);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.W = take((size_t)3 * nz * ny * padded_pitch(nx) * c8);
  L.V0 = take((size_t)N * c8);
  L.twx = take((size_t)nx * c8);
  L.twy = take((size_t)ny * c8);
  L.twz = take((size_t)nz * c8);
  L.phase = take((size_t)3 * nz * c8);
  L.phx = take((size_t)nx * c8);
  L.phy = take((size_t)ny * c8);
  L.partials = take((size_t)2 * k1b * sizeof(double));
  L.setup = take((size_t)2 * kSetupBlocks * sizeof(double));
  L.hist = take((size_t)kHistCap * sizeof(double));
  L.metrics = take((size_t)(2 * kMetricBlocks + nx + ny + nz + 1) * sizeof(double) +
                   (size_t)(nx + ny + 5 * N / nz) * sizeof(double2));
  L.state = take(sizeof(DevState));
  L.total = off;
  return true;
}

// Twiddles of a two-level split n = n1 n2: t[j2 n1 + k1] = exp(-2 pi i j2 k1 / n),
// j2 < n2, k1 < n1 (FP64 on the host, rounded to FP32).  j2 k1 < n, so the
// angle needs no reduction, and the same table read at [k][t] serves the
// transposed split.  t holds n entries.
void fill_twiddles(float2* t, int n1, int n2) {
  const int n = n1 * n2;
  for (int j2 = 0; j2 < n2; ++j2)
    for (int k1 = 0; k1 < n1; ++k1) {
      const double ang = -2.0 * M_PI * double(j2 * k1) / double(n);
      t[j2 * n1 + k1] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
}

// Longest registered axis: the host staging arrays of the tables are this long.
constexpr int kMaxAxis = 1024;

// Argument checks of a grid and its optics (cbs_plan_create's contract).
int check_grid(int nx, int ny, int nz, double pitch_m, double lambda0_m, double n_bg,
               const int pml[3], int pm[3]) {
  if (nx < 2 || ny < 2 || nz < 2) return fail(CBS_E_INVALID, "grid %dx%dx%d: each axis must be >= 2", nx, ny, nz);
  const int dims[3] = {nx, ny, nz};
  for (int a = 0; a < 3; ++a)
    if (!cbs_axis_supported(a, dims[a]) || dims[a] > kMaxAxis)
      return fail(CBS_E_INVALID, "axis %d length %d has no FFT specialisation", a, dims[a]);
  if (!(pitch_m > 0) || !std::isfinite(pitch_m)) return fail(CBS_E_INVALID, "pitch must be > 0");
  if (!(lambda0_m > 0) || !std::isfinite(lambda0_m)) return fail(CBS_E_INVALID, "lambda0 must be > 0");
  if (!(n_bg > 0) || !std::isfinite(n_bg)) return fail(CBS_E_INVALID, "n_bg must be > 0");
  pm[0] = pm[1] = pm[2] = 0;
  if (pml)
    for (int a = 0; a < 3; ++a) {
      pm[a] = pml[a];
      if (pm[a] < 0 || 2 * pm[a] >= dims[a])
        return fail(CBS_E_INVALID, "pml[%d]=%d must satisfy 0 <= 2 pml < %d", a, pm[a], dims[a]);
    }
  return CBS_OK;
}

// Fill a plan's grid, optics and workspace carve-up (no HIP calls).
void init_plan(cbs_plan_s* p, int nx, int ny, int nz, double pitch_m, double lambda0_m,
               double n_bg, const int pm[3], void* workspace, hipStream_t stream) {
  Layout L;
  layout_of(nx, ny, nz, L);
  p->nx = nx;
  p->ny = ny;
  p->nz = nz;
  p->nxp = padded_pitch(nx);
  for (int a = 0; a < 3; ++a) p->pml[a] = pm[a];
  p->pitch = pitch_m;
  p->lambda0 = lambda0_m;
  p->n_bg = n_bg;
  p->k0 = 2.0 * M_PI / lambda0_m;
  p->kb = p->k0 * n_bg;
  p->order = 2;
  p->sigma_max = 1.0;
  p->shift_factor = 1.1;
  p->ox = find_size(nx);
  p->oy = find_size(ny);
  p->oz = find_size(nz);
  p->k1_blocks = (int)(3LL * ((ny + p->ox->k1_rows - 1) / p->ox->k1_rows) * nz);
  p->stream = stream;
  char* base = static_cast<char*>(workspace);
  p->W = reinterpret_cast<float2*>(base + L.W);
  p->V0 = reinterpret_cast<float2*>(base + L.V0);
  p->twx = reinterpret_cast<float2*>(base + L.twx);
  p->twy = reinterpret_cast<float2*>(base + L.twy);
  p->twz = reinterpret_cast<float2*>(base + L.twz);
  p->phase = reinterpret_cast<float2*>(base + L.phase);
  p->phx = reinterpret_cast<float2*>(base + L.phx);
  p->phy = reinterpret_cast<float2*>(base + L.phy);
  p->partials = reinterpret_cast<double*>(base + L.partials);
  p->setup_part = reinterpret_cast<double*>(base + L.setup);
  p->hist = reinterpret_cast<double*>(base + L.hist);
  p->metrics = reinterpret_cast<double*>(base + L.metrics);
  p->state = reinterpret_cast<DevState*>(base + L.state);
  p->have_eps = false;
  p->eps = -1.0;
  p->hist_len = 0;
}

// Enqueue the twiddle tables (FP64 on the host, rounded to FP32) from host
// staging arrays that live until the stream has consumed them (the caller
// synchronises before they go out of scope).  The plane-wave phase tables are
// built on the device when a solve starts (k_phase_tables).
struct Tables {
  float2 tx[kMaxAxis], ty[kMaxAxis], tz[kMaxAxis];
};
hipError_t upload_tables(cbs_plan_s* p, Tables& t) {
  fill_twiddles(t.tx, p->ox->n1, p->ox->n2);
  fill_twiddles(t.ty, p->oy->n1, p->oy->n2);
  fill_twiddles(t.tz, p->oz->z1, p->oz->z2);
  hipError_t e = hipMemcpyAsync(p->twx, t.tx, p->nx * sizeof(float2), hipMemcpyHostToDevice, p->stream);
  e = e == hipSuccess ? hipMemcpyAsync(p->twy, t.ty, p->ny * sizeof(float2), hipMemcpyHostToDevice, p->stream) : e;
  e = e == hipSuccess ? hipMemcpyAsync(p->twz, t.tz, p->nz * sizeof(float2), hipMemcpyHostToDevice, p->stream) : e;
  return e;
}

// The potential V0, the shift eps and the validity checks of a medium
// (cbs_set_permittivity's contract).  Synchronises the plan's stream.
int set_permittivity_impl(cbs_plan_s* p, const void* eps_r, int dtype) {
  if (!eps_r) return fail(CBS_E_INVALID, "eps_r is NULL");
  if (dtype != CBS_F32 && dtype != CBS_C64) return fail(CBS_E_INVALID, "dtype must be CBS_F32 or CBS_C64");
  p->have_eps = false;
  SetupArgs s;
  s.nx = p->nx;
  s.ny = p->ny;
  s.nz = p->nz;
  s.px = p->pml[0];
  s.py = p->pml[1];
  s.pz = p->pml[2];
  s.order = p->order;
  s.dtype = dtype;
  s.sigma_max = p->sigma_max;
  const double d2 = p->pitch * p->pitch;
  s.k0d2 = p->k0 * p->k0 * d2;
  s.kbd2 = p->kb * p->kb * d2;
  s.nb2 = p->n_bg * p->n_bg;
  s.nb2f = (float)(p->n_bg * p->n_bg);
  s.eps = eps_r;
  s.V0 = p->V0;
  s.part = p->setup_part;
  hipLaunchKernelGGL(k_setup, dim3(kSetupBlocks), dim3(kSetupThreads), 0, p->stream, s);
  HIP_LAUNCHED();
  double part[2 * kSetupBlocks];
  HIP_TRY(hipMemcpyAsync(part, p->setup_part, sizeof(part), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  double mx = 0.0;
  unsigned fl = 0;
  for (int b = 0; b < kSetupBlocks; ++b) {
    mx = part[2 * b] > mx ? part[2 * b] : mx;
    fl |= (unsigned)part[2 * b + 1];
  }
  if (fl & 1u) return fail(CBS_E_INVALID, "eps_r has non-finite values");
  if (fl & 2u) return fail(CBS_E_INVALID, "gain medium (Im eps_r < 0) is not admissible");
  if (fl & 4u) return fail(CBS_E_INVALID, "eps_r must equal n_bg^2 inside the absorbing layer");
  const double floor_ = 1e-3 * p->kb * p->kb * d2;
  const double eps_d2 = p->shift_factor * (mx > floor_ ? mx : floor_);
  // the iteration forms (V0 - i eps) E in FP32: keep the shift far inside its range
  if (!(eps_d2 < 1e30))
    return fail(CBS_E_INVALID, "eps_r contrast too large for the FP32 iteration (shift %g)", eps_d2);
  p->eps = eps_d2 / d2;
  p->have_eps = true;
  return CBS_OK;
}

CbsArgs base_args(cbs_plan_s* p) {
  CbsArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nx = p->nx;
  a.ny = p->ny;
  a.nz = p->nz;
  a.nxp = p->nxp;
  a.gx = p->nxp / kBrick;
  a.gy = (p->ny + p->ox->k1_rows - 1) / p->ox->k1_rows;
  a.px = p->pml[0];
  a.py = p->pml[1];
  a.pz = p->pml[2];
  a.sW = (long long)p->nz * p->ny * p->nxp;
  a.sE = (long long)p->nz * p->ny * p->nx;
  a.W = p->W;
  a.V0 = p->V0;
  a.twx = p->twx;
  a.twy = p->twy;
  a.twz = p->twz;
  a.phase = p->phase;
  a.partials = p->partials;
  a.k1_blocks = p->k1_blocks;
  a.nb = 1;
  a.sWb = 3 * a.sW;
  a.sEb = 3 * a.sE;
  a.phx = p->phx;
  a.phy = p->phy;
  a.oblique = 0;
  a.hist = p->hist;
  a.st = p->state;
  const double d2 = p->pitch * p->pitch;
  a.eps = (float)(p->eps * d2);
  a.inv_eps = (float)(1.0 / (p->eps * d2));
  a.kb2 = (float)(p->kb * p->kb * d2);
  a.pfx = (float)(2.0 * M_PI / p->nx);
  a.pfy = (float)(2.0 * M_PI / p->ny);
  a.pfz = (float)(2.0 * M_PI / p->nz);
  a.invN = (float)(1.0 / ((double)p->nx * p->ny * p->nz));
  a.src_scale = (float)d2;
  return a;
}

int check_plan(cbs_plan_t p, bool need_eps) {
  if (!p) return fail(CBS_E_INVALID, "null plan");
  if (need_eps && !p->have_eps)
    return fail(CBS_E_STATE, "cbs_set_permittivity must be called before solving");
  return CBS_OK;
}

int check_opts(const cbs_opts* o) {
  if (!o) return fail(CBS_E_INVALID, "opts is NULL");
  if (o->max_iter < 1) return fail(CBS_E_INVALID, "max_iter must be >= 1 (got %d)", o->max_iter);
  if (o->check_every < 1) return fail(CBS_E_INVALID, "check_every must be >= 1");
  if (!(o->tol >= 0.0)) return fail(CBS_E_INVALID, "tol must be >= 0");
  return CBS_OK;
}

// one CBS iteration: y forward, z forward + Green + z inverse, y inverse,
// x inverse + update + next forward x, residual
int enqueue_iteration(cbs_plan_s* p, const CbsArgs& a) {
  p->oy->ky(a, -1, p->stream);
  p->oz->kz(a, p->stream);
  p->oy->ky(a, +1, p->stream);
  p->ox->k1(a, K1_ITER, p->stream);   // its residual is reduced by the next y pass
  HIP_LAUNCHED();
  return CBS_OK;
}

// reduce the residual of the last enqueued iteration (a no-op when nothing is
// pending), so the state copied to the host is current
int enqueue_residual(cbs_plan_s* p, const CbsArgs& a) {
  hipLaunchKernelGGL(k_residual, dim3(1), dim3(kResThreads), 0, p->stream, a.partials,
                     a.k1_blocks, a.nb, p->state, p->hist);
  HIP_LAUNCHED();
  return CBS_OK;
}

// Start a solve: device state, point-source amplitude, optional warm-start
// conversion to the scattered field, and the prologue (W = V E + S, forward x).
// Device state, point-source amplitude and warm-start conversion of a solve.
int enqueue_solve_start(cbs_plan_s* p, CbsArgs& a, const cbs_opts* o, const cbs_source* src,
                        const void* E_fwd, const Kvec& kv) {
  if (a.src == SRC_PLANE) {
    // the incident plane waves' phase tables (built before anything reads them)
    const int n = kv.nb * (p->nx + p->ny + 3 * p->nz);
    hipLaunchKernelGGL(k_phase_tables, dim3((n + 255) / 256), dim3(256), 0, p->stream,
                       const_cast<float2*>(a.phx), const_cast<float2*>(a.phy),
                       const_cast<float2*>(a.phase), p->nx, p->ny, p->nz, kv);
    HIP_LAUNCHED();
  }
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, p->stream, p->state, o->tol,
                     o->max_iter, (o->flags & CBS_RECORD_HISTORY) ? 1 : 0);
  HIP_LAUNCHED();
  if (a.src == SRC_POINT) {
    const long long idx = ((long long)src->r0[2] * p->ny + src->r0[1]) * p->nx + src->r0[0];
    hipLaunchKernelGGL(k_point_amp, dim3(1), dim3(64), 0, p->stream, p->state,
                       static_cast<const float2*>(E_fwd), idx, a.sE, E_fwd ? 1 : 0,
                       (float)(p->pitch * p->pitch),
                       make_float2((float)src->amp[0][0], (float)src->amp[0][1]),
                       make_float2((float)src->amp[1][0], (float)src->amp[1][1]),
                       make_float2((float)src->amp[2][0], (float)src->amp[2][1]));
    HIP_LAUNCHED();
  }
  a.warm = (o->flags & CBS_WARM_START) ? 1 : 0;
  if (a.warm && a.src == SRC_PLANE) {
    hipLaunchKernelGGL(k_incident, dim3(2048), dim3(256), 0, p->stream, a, -1.0f);
    HIP_LAUNCHED();
  }
  return CBS_OK;
}

int begin_solve(cbs_plan_s* p, CbsArgs& a, const cbs_opts* o, const cbs_source* src,
                const void* E_fwd, const Kvec& kv) {
  auto& A = p->act;
  if (A.on) return fail(CBS_E_STATE, "a solve is already in progress on this plan");
  if (int rc = enqueue_solve_start(p, a, o, src, E_fwd, kv)) return rc;
  const bool plane = a.src == SRC_PLANE;
  HIP_TRY(hipEventRecord(p->ev0, p->stream));
  p->ox->k1(a, K1_FWD, p->stream);
  HIP_LAUNCHED();
  A.on = true;
  A.stopped = false;
  A.plane = plane;
  A.flags = o->flags;
  A.max_iter = o->max_iter;
  A.enqueued = 0;
  A.head = A.count = 0;
  A.ms = 0.f;
  A.args = a;
  std::memset(&p->last, 0, sizeof(DevState));
  return CBS_OK;
}

// Enqueue up to `iters` iterations and an asynchronous copy of the device
// state into the next pinned slot; never blocks.
int advance_solve(cbs_plan_s* p, int iters) {
  auto& A = p->act;
  if (!A.on) return fail(CBS_E_STATE, "no solve in progress (cbs_solve_begin first)");
  if (iters < 1) return fail(CBS_E_INVALID, "iters must be >= 1");
  if (A.stopped || A.enqueued >= A.max_iter) return CBS_OK;
  if (A.count == cbs_plan_s::kRing)
    return fail(CBS_E_STATE, "%d quanta already outstanding; poll before advancing", A.count);
  const int q = std::min(iters, A.max_iter - A.enqueued);
  for (int i = 0; i < q; ++i) {
    int rc = enqueue_iteration(p, A.args);
    if (rc != CBS_OK) return rc;
  }
  A.enqueued += q;
  if (int rc = enqueue_residual(p, A.args)) return rc;
  const int slot = (A.head + A.count) % cbs_plan_s::kRing;
  HIP_TRY(hipMemcpyAsync(&p->mirror[slot], p->state, sizeof(DevState), hipMemcpyDeviceToHost,
                         p->stream));
  HIP_TRY(hipEventRecord(p->evq[slot], p->stream));
  A.count++;
  return CBS_OK;
}

// Retire completed quanta in order; never blocks.
int poll_solve(cbs_plan_s* p, int* done) {
  auto& A = p->act;
  if (!A.on) return fail(CBS_E_STATE, "no solve in progress");
  while (A.count > 0) {
    const hipError_t e = hipEventQuery(p->evq[A.head]);
    if (e == hipErrorNotReady) break;
    if (e != hipSuccess) return fail(CBS_E_HIP, "hipEventQuery: %s", hipGetErrorString(e));
    p->last = p->mirror[A.head];
    if (p->last.done && !A.stopped) {
      A.stopped = true;
      HIP_TRY(hipEventElapsedTime(&A.ms, p->ev0, p->evq[A.head]));
    }
    A.head = (A.head + 1) % cbs_plan_s::kRing;
    A.count--;
  }
  if (done) *done = A.stopped ? 1 : 0;
  return CBS_OK;
}

int wait_solve(cbs_plan_s* p) {
  auto& A = p->act;
  if (A.count > 0) {
    const int tail = (A.head + A.count - 1) % cbs_plan_s::kRing;
    HIP_TRY(hipEventSynchronize(p->evq[tail]));
  }
  return poll_solve(p, nullptr);
}

// Finish: add E_inc for plane-wave solves (enqueued), report stats and status.
int end_solve(cbs_plan_s* p, cbs_stats* stats) {
  auto& A = p->act;
  if (!A.on) return fail(CBS_E_STATE, "no solve in progress");
  int rc = wait_solve(p);
  if (rc) return rc;
  if (!A.stopped) return fail(CBS_E_STATE, "solve has not stopped yet (advance further)");
  A.on = false;
  if (A.plane && !(A.flags & CBS_RETURN_SCATTERED)) {
    hipLaunchKernelGGL(k_incident, dim3(2048), dim3(256), 0, p->stream, A.args, 1.0f);
    HIP_LAUNCHED();
  }
  const DevState& hs = p->last;
  p->hist_len = (A.flags & CBS_RECORD_HISTORY) ? std::min(hs.iter, kHistCap) : 0;
  if (stats) {
    stats->iterations = hs.iter;
    stats->converged = hs.status == 1;
    stats->residual = hs.eta;
    stats->eps_shift = p->eps;
    stats->ms = A.ms;
  }
  if (hs.status == 3) return fail(CBS_E_DIVERGED, "non-finite residual after %d iterations", hs.iter);
  if (hs.status == 1) return CBS_OK;
  g_err = "max_iter reached before the residual met tol";
  return CBS_NOT_CONVERGED;
}

// Blocking solve on top of the primitives: host polls every check_every.
int run_blocking(cbs_plan_s* p, int check_every, cbs_stats* stats) {
  int done = 0, rc = CBS_OK;
  while (!done) {
    if ((rc = advance_solve(p, check_every))) break;
    if ((rc = wait_solve(p))) break;
    if ((rc = poll_solve(p, &done))) break;
  }
  if (rc) {
    p->act.on = false;
    (void)hipStreamSynchronize(p->stream);
    return rc;
  }
  rc = end_solve(p, stats);
  const hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return fail(CBS_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
  return rc;
}

// Argument checks and source set-up shared by the blocking and the
// asynchronous entry points.
int prepare(cbs_plan_s* p, int adjoint, const cbs_source* src, void* E, const cbs_opts* o,
            CbsArgs& a, Kvec& kv);

// Illumination b of a plane-wave source: polarisation (x if all zero) and the
// wave vector from the transverse direction cosines (normal incidence if zero).
int set_plane_wave(cbs_plan_s* p, CbsArgs& a, Kvec& kv, int b, const cbs_source* src) {
  for (int c = 0; c < 3; ++c) kv.pol[b][c][0] = kv.pol[b][c][1] = 0.0;
  kv.pol[b][0][0] = 1.0;
  double sx = 0.0, sy = 0.0;
  if (src) {
    bool any = false;
    for (int c = 0; c < 3; ++c) any |= (src->pol[c][0] != 0.0 || src->pol[c][1] != 0.0);
    if (any)
      for (int c = 0; c < 3; ++c) {
        kv.pol[b][c][0] = src->pol[c][0];
        kv.pol[b][c][1] = src->pol[c][1];
      }
    sx = src->dir[0];
    sy = src->dir[1];
  }
  if (!std::isfinite(sx) || !std::isfinite(sy) || !(sx * sx + sy * sy < 1.0))
    return fail(CBS_E_INVALID, "plane-wave direction (%g, %g): need sx^2 + sy^2 < 1", sx, sy);
  const double kbd = p->kb * p->pitch;
  kv.kd[b][0] = kbd * sx;
  kv.kd[b][1] = kbd * sy;
  kv.kd[b][2] = kbd * std::sqrt(1.0 - sx * sx - sy * sy);
  if (sx != 0.0 || sy != 0.0) a.oblique = 1;
  return CBS_OK;
}

int set_source(cbs_plan_s* p, CbsArgs& a, const cbs_source* src, bool adjoint, Kvec& kv) {
  const int kind = src ? src->kind : CBS_SRC_PLANE_WAVE;
  kv.nb = 1;
  for (int c = 0; c < 3; ++c) kv.kd[0][c] = kv.pol[0][c][0] = kv.pol[0][c][1] = 0.0;
  kv.pol[0][0][0] = 1.0;
  switch (kind) {
    case CBS_SRC_NONE:
      a.src = SRC_NONE;
      break;
    case CBS_SRC_PLANE_WAVE: {
      if (adjoint) return fail(CBS_E_INVALID, "adjoint source cannot be a plane wave");
      a.src = SRC_PLANE;
      if (int rc = set_plane_wave(p, a, kv, 0, src)) return rc;
      break;
    }
    case CBS_SRC_FIELD:
    case CBS_SRC_FIELD_CONJ:
      if (!src->field) return fail(CBS_E_INVALID, "FIELD source without a field pointer");
      a.src = kind == CBS_SRC_FIELD ? SRC_FIELD : SRC_FIELD_CONJ;
      a.fin = static_cast<const float2*>(src->field);
      break;
    case CBS_SRC_POINT:
      for (int c = 0; c < 3; ++c) {
        const int n = c == 0 ? p->nx : (c == 1 ? p->ny : p->nz);
        if (src->r0[c] < 0 || src->r0[c] >= n)
          return fail(CBS_E_INVALID, "point source r0[%d]=%d outside [0,%d)", c, src->r0[c], n);
      }
      a.src = SRC_POINT;
      a.r0x = src->r0[0];
      a.r0y = src->r0[1];
      a.r0z = src->r0[2];
      break;
    default:
      return fail(CBS_E_INVALID, "unknown source kind %d", kind);
  }
  return CBS_OK;
}

int prepare(cbs_plan_s* p, int adjoint, const cbs_source* src, void* E, const cbs_opts* o,
            CbsArgs& a, Kvec& kv) {
  int rc = check_plan(p, true);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if (!E) return fail(CBS_E_INVALID, "output field is NULL");
  if (adjoint) {
    if (!src) return fail(CBS_E_INVALID, "adjoint source is NULL");
    if (src->kind != CBS_SRC_POINT && src->kind != CBS_SRC_FIELD &&
        src->kind != CBS_SRC_FIELD_CONJ)
      return fail(CBS_E_INVALID, "adjoint source must be POINT, FIELD or FIELD_CONJ");
  }
  a = base_args(p);
  if ((rc = set_source(p, a, src, adjoint != 0, kv))) return rc;
  a.E = static_cast<float2*>(E);
  return CBS_OK;
}

// ---------------------------------------------------------------------------
// allocation-free solve: the workspace of one plan in a static device array
// ---------------------------------------------------------------------------
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];   // device address of cbs_scratch, per device

int static_scratch(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CBS_E_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(cbs_scratch)));
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256 != 0)
      return fail(CBS_E_HIP, "static scratch of device %d has no usable address", dev);
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CBS_OK;
}

__global__ void k_clear_words(unsigned* w, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) w[i] = 0u;
}

// The blocking solve loop without events or a pinned ring: enqueue
// check_every iterations and the residual, read the device state back
// synchronously, repeat until the device has stopped.
int run_static(cbs_plan_s* p, CbsArgs& a, const cbs_opts* o, const cbs_source* src,
               const Kvec& kv, cbs_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (int rc = enqueue_solve_start(p, a, o, src, nullptr, kv)) return rc;
  p->ox->k1(a, K1_FWD, p->stream);
  HIP_LAUNCHED();
  DevState hs;
  std::memset(&hs, 0, sizeof(hs));
  int enqueued = 0;
  for (;;) {
    const int q = std::min(o->check_every, o->max_iter - enqueued);
    for (int i = 0; i < q; ++i)
      if (int rc = enqueue_iteration(p, a)) return rc;
    enqueued += q;
    if (int rc = enqueue_residual(p, a)) return rc;
    HIP_TRY(hipMemcpyAsync(&hs, p->state, sizeof(DevState), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    if (hs.done || enqueued >= o->max_iter) break;
  }
  if (a.src == SRC_PLANE && !(o->flags & CBS_RETURN_SCATTERED)) {
    hipLaunchKernelGGL(k_incident, dim3(2048), dim3(256), 0, p->stream, a, 1.0f);
    HIP_LAUNCHED();
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) {
    stats->iterations = hs.iter;
    stats->converged = hs.status == 1;
    stats->residual = hs.eta;
    stats->eps_shift = p->eps;
    stats->ms = (float)ms;
  }
  if (hs.status == 3) return fail(CBS_E_DIVERGED, "non-finite residual after %d iterations", hs.iter);
  if (hs.status == 1) return CBS_OK;
  g_err = "max_iter reached before the residual met tol";
  return CBS_NOT_CONVERGED;
}

}  // namespace

extern "C" {

int cbs_solve_static(int nx, int ny, int nz, double pitch_m, double lambda0_m, double n_bg,
                     const int pml[3], const void* eps_r_dev, int dtype, const cbs_source* src,
                     void* E_dev, const cbs_opts* opts, cbs_stats* stats, void* stream) {
  int pm[3];
  if (int rc = check_grid(nx, ny, nz, pitch_m, lambda0_m, n_bg, pml, pm)) return rc;
  Layout L;
  layout_of(nx, ny, nz, L);
  if (L.total > CBS_STATIC_SCRATCH_BYTES)
    return fail(CBS_E_WORKSPACE,
                "grid %dx%dx%d needs %zu bytes of scratch; the static scratch holds %zu "
                "(use cbs_plan_create with a workspace)",
                nx, ny, nz, L.total, (size_t)CBS_STATIC_SCRATCH_BYTES);
  if (int rc = check_opts(opts)) return rc;
  if (!eps_r_dev || !E_dev) return fail(CBS_E_INVALID, "eps_r or the output field is NULL");
  void* base = nullptr;
  if (int rc = static_scratch(&base)) return rc;
  cbs_plan_s p{};   // on the stack: no events, no pinned memory
  init_plan(&p, nx, ny, nz, pitch_m, lambda0_m, n_bg, pm, base, static_cast<hipStream_t>(stream));
  Tables t;         // host staging of the tables, consumed before set-up returns
  HIP_TRY(upload_tables(&p, t));
  hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, p.stream,
                     reinterpret_cast<unsigned*>(p.state), (int)(sizeof(DevState) / 4));
  HIP_LAUNCHED();
  if (int rc = set_permittivity_impl(&p, eps_r_dev, dtype)) return rc;   // synchronises
  CbsArgs a;
  Kvec kv;
  if (int rc = prepare(&p, 0, src, E_dev, opts, a, kv)) return rc;
  return run_static(&p, a, opts, src, kv, stats);
}


size_t cbs_plan_workspace_bytes(int nx, int ny, int nz) {
  if (nx < 2 || ny < 2 || nz < 2) return 0;
  if (!cbs_axis_supported(0, nx) || !cbs_axis_supported(1, ny) || !cbs_axis_supported(2, nz))
    return 0;
  Layout L;
  if (!layout_of(nx, ny, nz, L)) return 0;
  return L.total;
}

int cbs_axis_supported(int axis, int n) {
  const SizeOps* o = find_size(n);
  if (!o) return 0;
  if (axis == 2) return o->kz != nullptr;
  return (axis == 0 || axis == 1) ? 1 : 0;
}

int cbs_plan_create(cbs_plan_t* out, int nx, int ny, int nz, double pitch_m, double lambda0_m,
                    double n_bg, const int pml[3], void* workspace, size_t workspace_bytes,
                    void* stream) {
  if (!out) return fail(CBS_E_INVALID, "out is NULL");
  *out = nullptr;
  int pm[3];
  if (int rc = check_grid(nx, ny, nz, pitch_m, lambda0_m, n_bg, pml, pm)) return rc;
  Layout L;
  layout_of(nx, ny, nz, L);
  if (!workspace) return fail(CBS_E_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(CBS_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (workspace_bytes < L.total)
    return fail(CBS_E_WORKSPACE, "workspace %zu bytes < required %zu", workspace_bytes, L.total);

  cbs_plan_s* p = new (std::nothrow) cbs_plan_s();
  if (!p) return fail(CBS_E_INVALID, "out of host memory");
  init_plan(p, nx, ny, nz, pitch_m, lambda0_m, n_bg, pm, workspace,
            static_cast<hipStream_t>(stream));
  // events are created null and destroyed by cleanup whatever succeeded
  auto cleanup = [&](int rc) {
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    for (int i = 0; i < 6; ++i)
      if (p->evp[i]) (void)hipEventDestroy(p->evp[i]);
    for (int i = 0; i < cbs_plan_s::kRing; ++i)
      if (p->evq[i]) (void)hipEventDestroy(p->evq[i]);
    if (p->mirror) (void)hipHostFree(p->mirror);
    delete p;
    return rc;
  };
  if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess)
    return cleanup(fail(CBS_E_HIP, "hipEventCreate failed"));
  for (int i = 0; i < 6; ++i)
    if (hipEventCreate(&p->evp[i]) != hipSuccess) return cleanup(fail(CBS_E_HIP, "hipEventCreate failed"));
  for (int i = 0; i < cbs_plan_s::kRing; ++i)
    if (hipEventCreate(&p->evq[i]) != hipSuccess) return cleanup(fail(CBS_E_HIP, "hipEventCreate failed"));
  if (hipHostMalloc((void**)&p->mirror, cbs_plan_s::kRing * sizeof(DevState), hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(CBS_E_HIP, "hipHostMalloc of the state mirror failed"));
  Tables* t = new (std::nothrow) Tables;
  if (!t) return cleanup(fail(CBS_E_INVALID, "out of host memory"));
  hipError_t e = upload_tables(p, *t);
  e = e == hipSuccess ? hipMemsetAsync(p->W, 0, L.V0 - L.W, p->stream) : e;
  e = e == hipSuccess ? hipMemsetAsync(p->state, 0, sizeof(DevState), p->stream) : e;
  const hipError_t es = hipStreamSynchronize(p->stream);
  delete t;
  e = e == hipSuccess ? es : e;
  if (e != hipSuccess) return cleanup(fail(CBS_E_HIP, "plan upload: %s", hipGetErrorString(e)));
  *out = p;
  return CBS_OK;
}

int cbs_plan_set_pml_profile(cbs_plan_t p, int order, double sigma_max) {
  int rc = check_plan(p, false);
  if (rc) return rc;
  if (order < 1 || order > 8) return fail(CBS_E_INVALID, "order must be in [1, 8]");
  if (!(sigma_max >= 0) || !std::isfinite(sigma_max)) return fail(CBS_E_INVALID, "sigma_max must be >= 0");
  p->order = order;
  p->sigma_max = sigma_max;
  p->have_eps = false;
  p->eps = -1.0;
  return CBS_OK;
}

int cbs_plan_set_shift_factor(cbs_plan_t p, double kappa) {
  int rc = check_plan(p, false);
  if (rc) return rc;
  if (!(kappa >= 1.0) || !std::isfinite(kappa)) return fail(CBS_E_INVALID, "shift factor must be >= 1 (got %g)", kappa);
  p->shift_factor = kappa;
  p->have_eps = false;
  p->eps = -1.0;
  return CBS_OK;
}

int cbs_set_permittivity(cbs_plan_t p, const void* eps_r, int dtype) {
  int rc = check_plan(p, false);
  if (rc) return rc;
  return set_permittivity_impl(p, eps_r, dtype);
}

double cbs_eps_shift(cbs_plan_t p) { return (p && p->have_eps) ? p->eps : -1.0; }

int cbs_solve(cbs_plan_t p, const cbs_source* src, void* E_dev, const cbs_opts* o,
              cbs_stats* stats) {
  CbsArgs a;
  Kvec kv;
  int rc = prepare(p, 0, src, E_dev, o, a, kv);
  if (rc) return rc;
  if ((rc = begin_solve(p, a, o, src, nullptr, kv))) return rc;
  return run_blocking(p, o->check_every, stats);
}

int cbs_adjoint_solve(cbs_plan_t p, const void* E_fwd, const cbs_source* adj, void* E_adj,
                      const cbs_opts* o, cbs_stats* stats) {
  CbsArgs a;
  Kvec kv;
  int rc = prepare(p, 1, adj, E_adj, o, a, kv);
  if (rc) return rc;
  if ((rc = begin_solve(p, a, o, adj, E_fwd, kv))) return rc;
  return run_blocking(p, o->check_every, stats);
}

int cbs_solve_begin(cbs_plan_t p, int adjoint, const void* E_fwd, const cbs_source* src,
                    void* E_dev, const cbs_opts* o) {
  CbsArgs a;
  Kvec kv;
  int rc = prepare(p, adjoint, src, E_dev, o, a, kv);
  if (rc) return rc;
  return begin_solve(p, a, o, src, adjoint ? E_fwd : nullptr, kv);
}

int cbs_solve_advance(cbs_plan_t p, int iters) {
  int rc = check_plan(p, true);
  if (rc) return rc;
  return advance_solve(p, iters);
}

int cbs_solve_poll(cbs_plan_t p, int* done, int* outstanding) {
  int rc = check_plan(p, true);
  if (rc) return rc;
  rc = poll_solve(p, done);
  if (outstanding) *outstanding = p->act.count;
  return rc;
}

int cbs_solve_end(cbs_plan_t p, cbs_stats* stats) {
  int rc = check_plan(p, true);
  if (rc) return rc;
  return end_solve(p, stats);
}

namespace {
struct BatchLayout {
  size_t W, partials, phx, phy, phz, total;
};
bool batch_layout(int nx, int ny, int nz, int count, BatchLayout& B) {
  const SizeOps* ox = find_size(nx);
  if (!ox || count < 1 || count > kMaxIllum) return false;
  const long long k1b = 3LL * ((ny + ox->k1_rows - 1) / ox->k1_rows) * nz;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  // the fields follow each other with no padding: W_b = W_0 + 3 b sW
  B.W = take((size_t)count * 3 * nz * ny * padded_pitch(nx) * sizeof(float2));
  B.partials = take((size_t)count * 2 * k1b * sizeof(double));
  B.phx = take((size_t)count * nx * sizeof(float2));
  B.phy = take((size_t)count * ny * sizeof(float2));
  B.phz = take((size_t)count * 3 * nz * sizeof(float2));
  B.total = off;
  return true;
}
}  // namespace

size_t cbs_batch_workspace_bytes(int nx, int ny, int nz, int count) {
  if (!cbs_plan_workspace_bytes(nx, ny, nz)) return 0;
  BatchLayout B;
  return batch_layout(nx, ny, nz, count, B) ? B.total : 0;
}

int cbs_solve_batch(cbs_plan_t p, int count, const cbs_source* srcs, void* E_dev,
                    const cbs_opts* o, cbs_stats* stats, void* work, size_t work_bytes) {
  int rc = check_plan(p, true);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if (count < 1 || count > kMaxIllum)
    return fail(CBS_E_INVALID, "count %d outside [1, %d]", count, kMaxIllum);
  if (!srcs || !E_dev) return fail(CBS_E_INVALID, "sources or the output field is NULL");
  BatchLayout B;
  batch_layout(p->nx, p->ny, p->nz, count, B);
  if (!work) return fail(CBS_E_WORKSPACE, "batch workspace is NULL");
  if (reinterpret_cast<uintptr_t>(work) % 256 != 0)
    return fail(CBS_E_WORKSPACE, "batch workspace must be 256-byte aligned");
  if (work_bytes < B.total)
    return fail(CBS_E_WORKSPACE, "batch workspace %zu bytes < required %zu", work_bytes, B.total);
  CbsArgs a = base_args(p);
  Kvec kv;
  kv.nb = count;
  a.src = SRC_PLANE;
  for (int b = 0; b < count; ++b) {
    if (srcs[b].kind != CBS_SRC_PLANE_WAVE)
      return fail(CBS_E_INVALID, "batched source %d is not a plane wave", b);
    if ((rc = set_plane_wave(p, a, kv, b, &srcs[b]))) return rc;
  }
  char* base = static_cast<char*>(work);
  a.nb = count;
  a.W = reinterpret_cast<float2*>(base + B.W);
  a.partials = reinterpret_cast<double*>(base + B.partials);
  a.phx = reinterpret_cast<float2*>(base + B.phx);
  a.phy = reinterpret_cast<float2*>(base + B.phy);
  a.phase = reinterpret_cast<float2*>(base + B.phz);
  a.E = static_cast<float2*>(E_dev);
  if ((rc = begin_solve(p, a, o, nullptr, nullptr, kv))) return rc;
  cbs_stats st;
  rc = run_blocking(p, o->check_every, &st);
  if (rc < 0 && rc != CBS_E_DIVERGED) return rc;
  if (stats)
    for (int b = 0; b < count; ++b) {
      stats[b] = st;
      stats[b].residual = p->last.eta_b[b];
      stats[b].converged = p->last.eta_b[b] <= o->tol ? 1 : 0;
    }
  return rc;
}

int cbs_batch_step(cbs_plan_t* plans, int count, int iters, int* done_out) {
  if (count < 0 || (count > 0 && (!plans || !done_out)))
    return fail(CBS_E_INVALID, "bad plan array");
  for (int i = 0; i < count; ++i) {
    int rc = check_plan(plans[i], true);
    if (rc) return rc;
    if (!plans[i]->act.on) return fail(CBS_E_STATE, "plan %d has no solve in progress", i);
  }
  // enqueue every plan's quantum first (each on its own stream), then wait
  for (int i = 0; i < count; ++i) {
    int rc = advance_solve(plans[i], iters);
    if (rc) return rc;
  }
  for (int i = 0; i < count; ++i) {
    int rc = wait_solve(plans[i]);
    if (rc) return rc;
    done_out[i] = plans[i]->act.stopped ? 1 : 0;
  }
  return CBS_OK;
}

int cbs_gradient(cbs_plan_t p, const void* E, const void* Ea, const int lo[3], const int hi[3],
                 double scale, float* grad) {
  int rc = check_plan(p, false);
  if (rc) return rc;
  if (!E || !Ea || !grad || !lo || !hi) return fail(CBS_E_INVALID, "NULL argument");
  const int dims[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a)
    if (lo[a] < 0 || hi[a] > dims[a] || lo[a] > hi[a])
      return fail(CBS_E_INVALID, "box axis %d [%d,%d) outside [0,%d)", a, lo[a], hi[a], dims[a]);
  const int bx = hi[0] - lo[0], by = hi[1] - lo[1], bz = hi[2] - lo[2];
  if ((long long)bx * by * bz == 0) return CBS_OK;
  hipLaunchKernelGGL(k_gradient, dim3(2048), dim3(256), 0, p->stream,
                     static_cast<const float2*>(E), static_cast<const float2*>(Ea),
                     (long long)p->nx * p->ny * p->nz, p->nx, p->ny, lo[0], lo[1], lo[2], bx, by,
                     bz, scale * p->k0 * p->k0, grad);
  HIP_LAUNCHED();
  return CBS_OK;
}

namespace {
// Full width at half maximum of the profile v[0, n) around its sample i0, with
// the half-maximum crossings interpolated linearly between samples; NaN when
// the profile does not fall below half on both sides inside [0, n).
double fwhm_of(const double* v, int n, int i0, double pitch) {
  const double half = 0.5 * v[i0];
  int l = i0;
  while (l > 0 && v[l - 1] >= half) --l;
  int r = i0;
  while (r < n - 1 && v[r + 1] >= half) ++r;
  if (l == 0 || r == n - 1) return std::nan("");
  const double xl = (l - 1) + (half - v[l - 1]) / (v[l] - v[l - 1]);
  const double xr = r + (v[r] - half) / (v[r] - v[r + 1]);
  return (xr - xl) * pitch;
}
}  // namespace

int cbs_lens_metrics(cbs_plan_t p, const void* E, const int lo[3], const int hi[3],
                     double disc_factor, double aperture_m, double e0, cbs_lens_figures* out) {
  int rc = check_plan(p, false);
  if (rc) return rc;
  if (!E || !lo || !hi || !out) return fail(CBS_E_INVALID, "NULL argument");
  if (!(disc_factor > 0) || !(aperture_m > 0) || !(e0 > 0))
    return fail(CBS_E_INVALID, "disc_factor, aperture and e0 must be > 0");
  const int dims[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a)
    if (lo[a] < 0 || hi[a] > dims[a] || lo[a] >= hi[a])
      return fail(CBS_E_INVALID, "search box axis %d [%d,%d) empty or outside [0,%d)", a, lo[a],
                  hi[a], dims[a]);
  const float2* F = static_cast<const float2*>(E);
  const long long sE = (long long)p->nx * p->ny * p->nz;
  const int bx = hi[0] - lo[0], by = hi[1] - lo[1], bz = hi[2] - lo[2];
  const long long NB = (long long)bx * by * bz;
  const int nb = (int)std::min<long long>(kMetricBlocks, (NB + kMetricThreads - 1) / kMetricThreads);
  // 1. focus: the maximum of |E|^2 in the box
  hipLaunchKernelGGL(k_argmax_intensity, dim3(nb), dim3(kMetricThreads), 0, p->stream, F, sE,
                     p->nx, p->ny, lo[0], lo[1], lo[2], bx, by, bz, p->metrics);
  HIP_LAUNCHED();
  std::vector<double> part(2 * kMetricBlocks);
  HIP_TRY(hipMemcpyAsync(part.data(), p->metrics, 2 * nb * sizeof(double), hipMemcpyDeviceToHost,
                         p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  double best = -1.0;
  long long bi = 0;
  for (int b = 0; b < nb; ++b)
    if (part[2 * b] > best || (part[2 * b] == best && (long long)part[2 * b + 1] < bi)) {
      best = part[2 * b];
      bi = (long long)part[2 * b + 1];
    }
  const int fx = (int)(bi % p->nx), fy = (int)((bi / p->nx) % p->ny), fz = (int)(bi / ((long long)p->nx * p->ny));
  // 2. profiles through the focus and their widths
  const int nl = p->nx + p->ny + p->nz;
  double* lines = p->metrics + 2 * kMetricBlocks;
  hipLaunchKernelGGL(k_line_intensity, dim3((nl + 255) / 256), dim3(256), 0, p->stream, F, sE,
                     p->nx, p->ny, p->nz, fx, fy, fz, lines);
  HIP_LAUNCHED();
  std::vector<double> prof(nl);
  HIP_TRY(hipMemcpyAsync(prof.data(), lines, nl * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  out->focus[0] = fx;
  out->focus[1] = fy;
  out->focus[2] = fz;
  out->peak = best;
  out->fwhm[0] = fwhm_of(prof.data(), p->nx, fx, p->pitch);
  out->fwhm[1] = fwhm_of(prof.data() + p->nx, p->ny, fy, p->pitch);
  out->fwhm[2] = fwhm_of(prof.data() + p->nx + p->ny, p->nz, fz, p->pitch);
  // 3. power through the disc of diameter disc_factor x lateral FWHM: the
  // Poynting flux of the plane's propagating angular spectrum
  out->disc_flux = std::nan("");
  out->eta_f = std::nan("");
  if (std::isfinite(out->fwhm[0]) && std::isfinite(out->fwhm[1])) {
    const int nx = p->nx, ny = p->ny;
    const long long NP = (long long)nx * ny;
    double2* twx = reinterpret_cast<double2*>(lines + ((nl + 1) & ~1));   // 16-byte aligned
    double2* twy = twx + nx;
    double2* pl[5];
    for (int k = 0; k < 5; ++k) pl[k] = twy + ny + k * NP;
    std::vector<double2> t(nx + ny);
    for (int m = 0; m < nx; ++m) t[m] = make_double2(std::cos(2 * M_PI * m / nx), -std::sin(2 * M_PI * m / nx));
    for (int m = 0; m < ny; ++m) t[nx + m] = make_double2(std::cos(2 * M_PI * m / ny), -std::sin(2 * M_PI * m / ny));
    HIP_TRY(hipMemcpyAsync(twx, t.data(), (nx + ny) * sizeof(double2), hipMemcpyHostToDevice, p->stream));
    const dim3 g((unsigned)std::min<long long>(4096, (NP + 255) / 256)), b(256);
    // pl[0] = Ex, pl[1] = Ey, pl[4] scratch; forward 2D DFTs in place via scratch
    hipLaunchKernelGGL(k_plane_extract, g, b, 0, p->stream, F, sE, nx, ny, fz, pl[0], pl[1]);
    HIP_LAUNCHED();
    auto dft2 = [&](double2* f, int sign) -> int {
      hipLaunchKernelGGL(k_plane_dft, g, b, 0, p->stream, f, pl[4], nx, ny, 0, sign, twx);
      HIP_LAUNCHED();
      hipLaunchKernelGGL(k_plane_dft, g, b, 0, p->stream, pl[4], f, nx, ny, 1, sign, twy);
      HIP_LAUNCHED();
      return CBS_OK;
    };
    if ((rc = dft2(pl[0], -1)) || (rc = dft2(pl[1], -1))) return rc;
    const double k = 2.0 * M_PI * p->n_bg / p->lambda0;
    hipLaunchKernelGGL(k_angular_h, g, b, 0, p->stream, pl[0], pl[1], pl[2], pl[3], nx, ny,
                       2.0 * M_PI / (nx * p->pitch), 2.0 * M_PI / (ny * p->pitch), k);
    HIP_LAUNCHED();
    for (int q = 0; q < 4; ++q)
      if ((rc = dft2(pl[q], +1))) return rc;
    const double radius = 0.5 * disc_factor * 0.5 * (out->fwhm[0] + out->fwhm[1]) / p->pitch;
    const int nd = (int)std::min<long long>(kMetricBlocks, (NP + kMetricThreads - 1) / kMetricThreads);
    const double scale = 1.0 / ((double)NP * (double)NP);   // two unscaled inverse transforms
    hipLaunchKernelGGL(k_disc_flux, dim3(nd), dim3(kMetricThreads), 0, p->stream, pl[0], pl[1],
                       pl[2], pl[3], nx, ny, (double)fx, (double)fy, radius * radius, scale,
                       p->metrics);
    HIP_LAUNCHED();
    HIP_TRY(hipMemcpyAsync(part.data(), p->metrics, nd * sizeof(double), hipMemcpyDeviceToHost,
                           p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    double sum = 0.0;
    for (int q = 0; q < nd; ++q) sum += part[q];
    out->disc_flux = sum * p->pitch * p->pitch;
    out->eta_f = out->disc_flux / (e0 * e0 * M_PI * 0.25 * aperture_m * aperture_m);
  }
  return CBS_OK;
}

int cbs_tfsf_source(cbs_plan_t p, const cbs_source* src, const int lo[3], const int hi[3],
                    void* S_dev) {
  int rc = check_plan(p, false);
  if (rc) return rc;
  if (!S_dev || !lo || !hi) return fail(CBS_E_INVALID, "NULL argument");
  if (src && src->kind != CBS_SRC_PLANE_WAVE)
    return fail(CBS_E_INVALID, "the TF/SF source injects a plane wave (kind PLANE_WAVE)");
  if (p->act.on) return fail(CBS_E_STATE, "a solve is in progress on this plan");
  const int dims[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a)
    if (lo[a] < 0 || hi[a] > dims[a] || lo[a] >= hi[a])
      return fail(CBS_E_INVALID, "box axis %d [%d,%d) empty or outside [0,%d)", a, lo[a], hi[a],
                  dims[a]);
  CbsArgs a = base_args(p);
  Kvec kv;
  kv.nb = 1;
  if ((rc = set_plane_wave(p, a, kv, 0, src))) return rc;
  TfsfAssemble A;
  TfsfArgs& t = A.t;
  t.ntot = p->nx + p->ny + p->nz;
  for (int ax = 0; ax < 3; ++ax) {
    t.n[ax] = dims[ax];
    t.lo[ax] = lo[ax];
    t.hi[ax] = hi[ax];
    t.kd[ax] = kv.kd[0][ax];
  }
  t.off[0] = 0;
  t.off[1] = p->nx;
  t.off[2] = p->nx + p->ny;
  t.pitch = p->pitch;
  t.tab = reinterpret_cast<double2*>(p->W);   // the spectral work field is free between solves
  A.nx = p->nx;
  A.ny = p->ny;
  A.nz = p->nz;
  A.px = p->pml[0];
  A.py = p->pml[1];
  A.pz = p->pml[2];
  A.order = p->order;
  A.sigma_max = p->sigma_max;
  A.kb2 = p->kb * p->kb;
  for (int c = 0; c < 3; ++c) {
    double re = c == 0 ? 1.0 : 0.0, im = 0.0;
    if (src) {
      bool any = false;
      for (int k = 0; k < 3; ++k) any |= (src->pol[k][0] != 0.0 || src->pol[k][1] != 0.0);
      if (any) {
        re = src->pol[c][0];
        im = src->pol[c][1];
      }
    }
    A.q[c] = make_double2(re, im);
  }
  A.S = static_cast<float2*>(S_dev);
  const dim3 g1((t.ntot + 127) / 128), b1(128);
  hipLaunchKernelGGL(k_tfsf_forward, g1, b1, 0, p->stream, t);
  HIP_LAUNCHED();
  hipLaunchKernelGGL(k_tfsf_inverse, g1, b1, 0, p->stream, t);
  HIP_LAUNCHED();
  hipLaunchKernelGGL(k_tfsf_assemble, dim3(2048), dim3(256), 0, p->stream, A);
  HIP_LAUNCHED();
  return CBS_OK;
}

int cbs_apply_green(cbs_plan_t p, const void* in, void* out) {
  int rc = check_plan(p, true);
  if (rc) return rc;
  if (!in || !out) return fail(CBS_E_INVALID, "NULL field");
  if (in == out) return fail(CBS_E_INVALID, "in and out must not alias");
  CbsArgs a = base_args(p);
  a.green_in = 1;
  a.fin = static_cast<const float2*>(in);
  a.fout = static_cast<float2*>(out);
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, p->stream, p->state, 0.0, 1, 0);
  HIP_LAUNCHED();
  p->ox->k1(a, K1_FWD, p->stream);
  p->oy->ky(a, -1, p->stream);
  p->oz->kz(a, p->stream);
  p->oy->ky(a, +1, p->stream);
  p->ox->k1(a, K1_INV, p->stream);
  HIP_LAUNCHED();
  return CBS_OK;
}

int cbs_time_passes(cbs_plan_t p, void* E_dev, int iters, float* ms_out) {
  int rc = check_plan(p, true);
  if (rc) return rc;
  if (!E_dev || !ms_out || iters < 1) return fail(CBS_E_INVALID, "bad arguments");
  CbsArgs a = base_args(p);
  Kvec kv;
  if ((rc = set_source(p, a, nullptr, false, kv))) return rc;
  a.E = static_cast<float2*>(E_dev);
  hipLaunchKernelGGL(k_phase_tables, dim3(8), dim3(256), 0, p->stream, p->phx, p->phy, p->phase,
                     p->nx, p->ny, p->nz, kv);
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, p->stream, p->state, 0.0, iters, 0);
  HIP_LAUNCHED();
  p->ox->k1(a, K1_FWD, p->stream);
  double acc[5] = {0, 0, 0, 0, 0};
  for (int it = 0; it < iters; ++it) {
    HIP_TRY(hipEventRecord(p->evp[0], p->stream));
    p->oy->ky(a, -1, p->stream);
    HIP_TRY(hipEventRecord(p->evp[1], p->stream));
    p->oz->kz(a, p->stream);
    HIP_TRY(hipEventRecord(p->evp[2], p->stream));
    p->oy->ky(a, +1, p->stream);
    HIP_TRY(hipEventRecord(p->evp[3], p->stream));
    p->ox->k1(a, K1_ITER, p->stream);
    HIP_TRY(hipEventRecord(p->evp[4], p->stream));
    HIP_LAUNCHED();   // the next y pass reduces the residual, as in a solve
    HIP_TRY(hipEventRecord(p->evp[5], p->stream));
    HIP_TRY(hipEventSynchronize(p->evp[5]));
    for (int k = 0; k < 5; ++k) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, p->evp[k], p->evp[k + 1]));
      acc[k] += ms;
    }
  }
  for (int k = 0; k < 5; ++k) ms_out[k] = (float)(acc[k] / iters);
  return CBS_OK;
}

int cbs_bandwidth_probe(const void* src, void* dst, size_t bytes, int reps, void* stream,
                        float* ms_out) {
  if (!src || !dst || !ms_out || reps < 1 || bytes == 0 || bytes % 16 != 0)
    return fail(CBS_E_INVALID, "bandwidth probe: bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long n4 = (long long)(bytes / 16);
  const long long nb = (n4 + kCopyThreads - 1) / kCopyThreads;
  if (nb > 0x7fffffffLL) return fail(CBS_E_INVALID, "bandwidth probe: buffer too large");
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int rc = CBS_OK;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)nb), dim3(kCopyThreads), 0, s,
                     static_cast<const float4*>(src), static_cast<float4*>(dst), n4);
  if (hipEventRecord(e0, s) != hipSuccess) rc = fail(CBS_E_HIP, "hipEventRecord failed");
  for (int r = 0; r < reps && rc == CBS_OK; ++r)
    hipLaunchKernelGGL(k_copy, dim3((unsigned)nb), dim3(kCopyThreads), 0, s,
                       static_cast<const float4*>(src), static_cast<float4*>(dst), n4);
  hipError_t e = hipGetLastError();
  if (rc == CBS_OK && e != hipSuccess) rc = fail(CBS_E_HIP, "kernel launch: %s", hipGetErrorString(e));
  if (rc == CBS_OK && hipEventRecord(e1, s) != hipSuccess) rc = fail(CBS_E_HIP, "hipEventRecord failed");
  if (rc == CBS_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(CBS_E_HIP, "hipEventSynchronize failed");
  float ms = 0.f;
  if (rc == CBS_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(CBS_E_HIP, "hipEventElapsedTime failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == CBS_OK) *ms_out = ms / reps;
  return rc;
}

// ---------------------------------------------------------------------------
// stretched-coordinate layer (reference [31]): per-axis operators, the
// operator of the preconditioned system and its GMRES solve
// ---------------------------------------------------------------------------
namespace {

struct ScpmlLayout {
  size_t basis, b, F, X, Z, mats[3], cols[3], part, h, y, total;
};

bool scpml_layout(int nx, int ny, int nz, int restart, ScpmlLayout& S) {
  if (restart < 1 || restart > kScpmlMaxRestart) return false;
  const int dims[3] = {nx, ny, nz};
  for (int a = 0; a < 3; ++a)
    if (dims[a] < 2 || dims[a] > kScpmlMaxAxis) return false;
  const size_t N = (size_t)nx * ny * nz;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  S.basis = take((size_t)(restart + 1) * 3 * N * sizeof(float2));
  S.b = take(3 * N * sizeof(float2));
  S.F = take(3 * N * sizeof(float2));
  S.X = take(N * sizeof(float2));
  S.Z = take(N * sizeof(float2));
  for (int a = 0; a < 3; ++a)
    S.mats[a] = take((3 * (size_t)dims[a] * dims[a] + dims[a]) * sizeof(float2));
  for (int a = 0; a < 3; ++a) S.cols[a] = take(5 * (size_t)dims[a] * sizeof(double2));
  S.part = take((size_t)(kScpmlMaxRestart + 1) * kGmBlocks * sizeof(double2));
  S.h = take((size_t)3 * (kScpmlMaxRestart + 1) * sizeof(double2));
  S.y = take((size_t)(kScpmlMaxRestart + 1) * sizeof(double2));
  S.total = off;
  return true;
}

struct Scpml {
  cbs_plan_s* p;
  int dims[3];
  long long N, n3;            // voxels; complex values of a vector field
  float2 *basis, *b, *F, *X, *Z;
  const float2 *A[3], *B[3], *T[3], *sinv[3];
  bool thin[3];               // 8p <= n: A and B in the two-launch form (RA|CA, RB|CB)
  double2 *part, *h, *y;
  float2* vec(int i) const { return basis + (long long)i * n3; }
};

int scpml_setup(cbs_plan_s* p, const cbs_scpml* layer, int restart, void* work, size_t bytes,
                Scpml& s) {
  if (!layer) return fail(CBS_E_INVALID, "layer parameters are NULL");
  if (!(layer->alpha_max >= 0.0) || !std::isfinite(layer->alpha_max))
    return fail(CBS_E_INVALID, "alpha_max must be finite and >= 0");
  if (layer->order < 1 || layer->order > 8) return fail(CBS_E_INVALID, "order must be in [1, 8]");
  ScpmlLayout S;
  if (!scpml_layout(p->nx, p->ny, p->nz, restart, S))
    return fail(CBS_E_INVALID, "restart must be in [1, %d] and every axis <= %d", kScpmlMaxRestart,
                kScpmlMaxAxis);
  if (!work) return fail(CBS_E_WORKSPACE, "stretched-layer workspace is NULL");
  if (reinterpret_cast<uintptr_t>(work) % 256 != 0)
    return fail(CBS_E_WORKSPACE, "stretched-layer workspace must be 256-byte aligned");
  if (bytes < S.total)
    return fail(CBS_E_WORKSPACE, "stretched-layer workspace %zu bytes < required %zu", bytes, S.total);
  char* base = static_cast<char*>(work);
  s.p = p;
  s.dims[0] = p->nx;
  s.dims[1] = p->ny;
  s.dims[2] = p->nz;
  s.N = (long long)p->nx * p->ny * p->nz;
  s.n3 = 3 * s.N;
  s.basis = reinterpret_cast<float2*>(base + S.basis);
  s.b = reinterpret_cast<float2*>(base + S.b);
  s.F = reinterpret_cast<float2*>(base + S.F);
  s.X = reinterpret_cast<float2*>(base + S.X);
  s.Z = reinterpret_cast<float2*>(base + S.Z);
  s.part = reinterpret_cast<double2*>(base + S.part);
  s.h = reinterpret_cast<double2*>(base + S.h);
  s.y = reinterpret_cast<double2*>(base + S.y);
  for (int a = 0; a < 3; ++a) {
    const int n = s.dims[a];
    float2* m = reinterpret_cast<float2*>(base + S.mats[a]);
    double2* col = reinterpret_cast<double2*>(base + S.cols[a]);
    s.A[a] = m;
    s.B[a] = m + (size_t)n * n;
    s.T[a] = m + 2 * (size_t)n * n;
    s.sinv[a] = m + 3 * (size_t)n * n;
    hipLaunchKernelGGL(k_scpml_columns, dim3((n + 127) / 128), dim3(128), 0, p->stream, n,
                       p->pml[a], layer->order, layer->alpha_max, col, col + n, col + 2 * n,
                       col + 3 * n, col + 4 * n);
    HIP_LAUNCHED();
    const long long nn = (long long)n * n;
    hipLaunchKernelGGL(k_scpml_matrices, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0,
                       p->stream, n, p->pml[a], col, col + n, col + 2 * n, col + 3 * n,
                       col + 4 * n, const_cast<float2*>(s.A[a]), const_cast<float2*>(s.B[a]),
                       const_cast<float2*>(s.T[a]), const_cast<float2*>(s.sinv[a]));
    HIP_LAUNCHED();
    const int pa = p->pml[a];
    s.thin[a] = pa > 0 && 8 * pa <= n;
    if (s.thin[a]) {
      const long long nt = 6LL * pa * n;
      hipLaunchKernelGGL(k_scpml_thin, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0,
                         p->stream, n, pa, col, col + n, col + 2 * n, col + 3 * n,
                         const_cast<float2*>(s.A[a]), const_cast<float2*>(s.B[a]));
      HIP_LAUNCHED();
    }
  }
  return CBS_OK;
}

// one axis product (kMm* epilogues, see scpml.hpp) over scalar [nz][ny][nx] fields;
// kMmCompact writes and kMmColFix reads the compact [lines][4p] buffer cbuf
int enqueue_axis_mm(const Scpml& s, int axis, const float2* M, const float2* in, float2* out,
                    float alpha, bool accumulate, int mode = kMmPlain, float2* out2 = nullptr,
                    const float2* cbuf = nullptr) {
  AxisMM a;
  a.M = M;
  a.in = in;
  a.out = out;
  a.out2 = out2;
  a.sinv = s.sinv[axis];
  a.aux = cbuf;
  a.n = s.dims[axis];
  a.Q = axis == 0 ? 1 : (axis == 1 ? s.dims[0] : s.dims[0] * s.dims[1]);
  a.p = s.p->pml[axis];
  a.rows = mode == kMmLayer ? 2 * a.p : (mode == kMmCompact ? 4 * a.p : a.n);
  a.K = mode == kMmColFix ? 2 * a.p : a.n;
  a.ldm = a.K;
  a.cld = 4LL * a.p;
  a.in_ld = mode == kMmColFix ? a.cld : 0;
  a.L = s.N / a.n;
  a.alpha = alpha;
  a.accumulate = accumulate ? 1 : 0;
  a.mode = mode;
  if (a.rows <= 0 || a.K <= 0) return CBS_OK;
  const unsigned tiles = (unsigned)((a.L + kMmTL - 1) / kMmTL) *
                         (unsigned)((a.rows + kMmTI - 1) / kMmTI);
  if (a.Q == 1 || a.in_ld > 0)
    hipLaunchKernelGGL(k_axis_mm<true>, dim3(tiles), dim3(256), 0, s.p->stream, a);
  else
    hipLaunchKernelGGL(k_axis_mm<false>, dim3(tiles), dim3(256), 0, s.p->stream, a);
  HIP_LAUNCHED();
  return CBS_OK;
}

// F_c += alpha M v_c along axis b for M = A_b (B) or B_b (!A): one dense product,
// or on a thin layer the two launches of the split form, with X as the compact
// buffer (X is no longer needed once every (S^-1 - I) T_c X term is formed)
int enqueue_ab(const Scpml& s, int b, bool A, const float2* vc, float2* Fc, float alpha) {
  const float2* M = A ? s.A[b] : s.B[b];
  if (!s.thin[b]) return enqueue_axis_mm(s, b, M, vc, Fc, alpha, true);
  const long long rows4 = 4LL * s.p->pml[b] * s.dims[b];   // RA (4p x n), then CA (n x 2p)
  if (int rc = enqueue_axis_mm(s, b, M, vc, s.X, 1.0f, false, kMmCompact)) return rc;
  return enqueue_axis_mm(s, b, M + rows4, s.X, Fc, alpha, true, kMmColFix, nullptr, s.X);
}

// F = alpha (L_s - L) v:  per component c, sum_{b != c} A_b v_c + B_c v_c +
// T_c Z + (S_c^-1 - I) T_c X, where one product u_b = T_b v_b per axis gives
// X = sum_b S_b^-1 u_b and Z = sum_b (S_b^-1 - I) u_b, and (S_c^-1 - I) T_c X is
// formed on the layer rows only (an axis without a layer has A = B = 0 and
// S^-1 = I exactly and skips those terms).  The X and Z terms of every component
// come first, so X can serve the thin-layer products as scratch.
int enqueue_delta(const Scpml& s, const float2* v, float2* F, float alpha) {
  const long long N = s.N;
  const int* pml = s.p->pml;
  int rc;
  for (int b = 0; b < 3; ++b)
    if ((rc = enqueue_axis_mm(s, b, s.T[b], v + b * N, s.X, 1.0f, b > 0, kMmSplit, s.Z)))
      return rc;
  for (int c = 0; c < 3; ++c) {
    float2* Fc = F + c * N;
    if ((rc = enqueue_axis_mm(s, c, s.T[c], s.Z, Fc, alpha, false))) return rc;
    if (pml[c] > 0 && (rc = enqueue_axis_mm(s, c, s.T[c], s.X, Fc, alpha, true, kMmLayer)))
      return rc;
  }
  for (int c = 0; c < 3; ++c) {
    float2* Fc = F + c * N;
    const float2* vc = v + c * N;
    if (pml[c] > 0 && (rc = enqueue_ab(s, c, false, vc, Fc, alpha))) return rc;
    for (int b = 0; b < 3; ++b)
      if (b != c && pml[b] > 0 && (rc = enqueue_ab(s, b, true, vc, Fc, alpha))) return rc;
  }
  return CBS_OK;
}

void gm_grid(long long n, dim3& g) {
  g = dim3((unsigned)std::min<long long>((n + kGmThreads - 1) / kGmThreads, 8192));
}

// w = B v = v - (the CBS step from v with the field source -(L_s - L) v):
// B = gamma [I - G (V - (L_s - L))], the CBS-preconditioned stretched operator
int enqueue_operator(const Scpml& s, const float2* v, float2* w) {
  cbs_plan_s* p = s.p;
  int rc = enqueue_delta(s, v, s.F, -1.0f);
  if (rc) return rc;
  dim3 g;
  gm_grid(s.n3, g);
  hipLaunchKernelGGL(k_gm_copy, g, dim3(kGmThreads), 0, p->stream, v, w, s.n3);
  HIP_LAUNCHED();
  CbsArgs a = base_args(p);
  a.E = w;
  a.src = SRC_FIELD;
  a.fin = s.F;
  a.src_scale = 1.0f;   // F is already in units of the pitch
  a.warm = 1;
  p->ox->k1(a, K1_FWD, p->stream);
  if ((rc = enqueue_iteration(p, a))) return rc;
  hipLaunchKernelGGL(k_gm_rsub, g, dim3(kGmThreads), 0, p->stream, v, w, s.n3);
  HIP_LAUNCHED();
  return CBS_OK;
}

// h[0..cnt) = V[0..cnt)^H w (vectors of n3 values, V_i = V + i n3)
int enqueue_dots(const Scpml& s, const float2* V, int cnt, const float2* w, double2* h) {
  hipLaunchKernelGGL(k_gm_dots, dim3(kGmBlocks, cnt), dim3(kGmThreads), 0, s.p->stream, V, s.n3,
                     w, s.n3, s.part);
  HIP_LAUNCHED();
  hipLaunchKernelGGL(k_gm_dots_finish, dim3(cnt), dim3(kGmThreads), 0, s.p->stream, s.part,
                     kGmBlocks, h);
  HIP_LAUNCHED();
  return CBS_OK;
}

// w += sign sum_i c_i V_i
int enqueue_update(const Scpml& s, int cnt, const double2* c, float sign, float2* w) {
  dim3 g;
  gm_grid(s.n3, g);
  hipLaunchKernelGGL(k_gm_update, g, dim3(kGmThreads), 0, s.p->stream, s.basis, s.n3, cnt, c,
                     sign, w, s.n3);
  HIP_LAUNCHED();
  return CBS_OK;
}

int enqueue_scale(const Scpml& s, float2* w, double f) {
  dim3 g;
  gm_grid(s.n3, g);
  hipLaunchKernelGGL(k_gm_scale, g, dim3(kGmThreads), 0, s.p->stream, w, s.n3, (float)f);
  HIP_LAUNCHED();
  return CBS_OK;
}

// copy n device double2 to the host and wait for the stream
int read_back(cbs_plan_s* p, const double2* dev, std::complex<double>* host, int n) {
  HIP_TRY(hipMemcpyAsync(host, dev, n * sizeof(double2), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return CBS_OK;
}

// Restarted GMRES(m) on B x = b from x = 0 (x in E_dev).  Arnoldi with
// classical Gram-Schmidt (fused dot and update passes over the basis),
// repeated for a step whose projection shortened w more than tenfold;
// Givens rotations on the host in FP64; at the end of each cycle the true
// residual b - B x gives the restart vector and the reported residual.
int scpml_gmres(const Scpml& s, float2* x, int m, const cbs_opts* o, double beta0, int* iters,
                double* rel_out, std::vector<double>& hist) {
  cbs_plan_s* p = s.p;
  using cd = std::complex<double>;
  std::vector<cd> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hv(3 * (m + 1)), y(m + 1);
  auto Hij = [&](int i, int j) -> cd& { return H[(size_t)j * (m + 1) + i]; };
  int total = 0, rc;
  double beta = beta0, rel = 1.0;
  // V_0 = b / beta0
  dim3 gg;
  gm_grid(s.n3, gg);
  hipLaunchKernelGGL(k_gm_copy, gg, dim3(kGmThreads), 0, p->stream, s.b, s.vec(0), s.n3);
  HIP_LAUNCHED();
  if ((rc = enqueue_scale(s, s.vec(0), 1.0 / beta0))) return rc;
  while (true) {
    std::fill(g.begin(), g.end(), cd(0));
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m && total < o->max_iter; ++j) {
      float2* w = s.vec(j + 1);
      if ((rc = enqueue_operator(s, s.vec(j), w))) return rc;
      double2* h0 = s.h;
      double2* h1 = s.h + (m + 1);
      double2* h2 = s.h + 2 * (m + 1);
      // classical Gram-Schmidt; w = V_{j+1}, so one sweep over V_0..V_{j+1}
      // also gives |w|^2 before the projection (h0[j+1])
      if ((rc = enqueue_dots(s, s.basis, j + 2, w, h0))) return rc;
      if ((rc = enqueue_update(s, j + 1, h0, -1.0f, w))) return rc;
      if ((rc = enqueue_dots(s, w, 1, w, h2))) return rc;
      if ((rc = read_back(p, s.h, hv.data(), 3 * (m + 1)))) return rc;
      for (int i = 0; i <= j; ++i) Hij(i, j) = hv[i];
      double nn = hv[2 * (m + 1)].real();
      // the projection shortened w more than tenfold: FP32 rounding of the
      // update may have left components along the basis of about 10 ulp of the
      // original length, so project once more (a DGKS-type test)
      if (nn < 1e-2 * hv[j + 1].real()) {
        if ((rc = enqueue_dots(s, s.basis, j + 1, w, h1))) return rc;
        if ((rc = enqueue_update(s, j + 1, h1, -1.0f, w))) return rc;
        if ((rc = enqueue_dots(s, w, 1, w, h2))) return rc;
        if ((rc = read_back(p, s.h, hv.data(), 3 * (m + 1)))) return rc;
        for (int i = 0; i <= j; ++i) Hij(i, j) += hv[(m + 1) + i];
        nn = hv[2 * (m + 1)].real();
      }
      const double hn = std::sqrt(std::max(0.0, nn));
      Hij(j + 1, j) = hn;
      for (int i = 0; i <= j; ++i)
        if (!std::isfinite(Hij(i, j).real()) || !std::isfinite(Hij(i, j).imag()))
          return fail(CBS_E_DIVERGED, "non-finite Arnoldi coefficient after %d steps", total);
      if (!std::isfinite(hn)) return fail(CBS_E_DIVERGED, "non-finite norm after %d steps", total);
      if (hn > 0.0 && (rc = enqueue_scale(s, w, 1.0 / hn))) return rc;
      // previous rotations, then the one that zeroes H(j+1, j)
      for (int i = 0; i < j; ++i) {
        const cd t = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
        Hij(i + 1, j) = -std::conj(sn[i]) * Hij(i, j) + cs[i] * Hij(i + 1, j);
        Hij(i, j) = t;
      }
      const cd a = Hij(j, j);
      const double r = std::hypot(std::abs(a), hn);
      cs[j] = r > 0 ? cd(std::abs(a) / r) : cd(1.0);
      sn[j] = r > 0 ? (std::abs(a) > 0 ? (a / std::abs(a)) * hn / r : cd(1.0)) : cd(0.0);
      Hij(j, j) = cs[j] * a + sn[j] * hn;
      Hij(j + 1, j) = 0.0;
      g[j + 1] = -std::conj(sn[j]) * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      ++k;
      const double est = std::abs(g[j + 1]) / beta0;
      hist.push_back(est);
      if (est <= o->tol || hn <= 1e-300) break;
    }
    // x += V y, H(0..k, 0..k) y = g
    for (int i = k - 1; i >= 0; --i) {
      cd t = g[i];
      for (int l = i + 1; l < k; ++l) t -= Hij(i, l) * y[l];
      y[i] = t / Hij(i, i);
    }
    if (k > 0) {
      HIP_TRY(hipMemcpyAsync(s.y, y.data(), k * sizeof(double2), hipMemcpyHostToDevice, p->stream));
      if ((rc = enqueue_update(s, k, s.y, 1.0f, x))) return rc;
    }
    // true residual r = b - B x into V_0
    if ((rc = enqueue_operator(s, x, s.vec(0)))) return rc;
    hipLaunchKernelGGL(k_gm_rsub, gg, dim3(kGmThreads), 0, p->stream, s.b, s.vec(0), s.n3);
    HIP_LAUNCHED();
    if ((rc = enqueue_dots(s, s.vec(0), 1, s.vec(0), s.h))) return rc;
    if ((rc = read_back(p, s.h, hv.data(), 1))) return rc;   // also retires the y upload
    beta = std::sqrt(std::max(0.0, hv[0].real()));
    if (!std::isfinite(beta)) return fail(CBS_E_DIVERGED, "non-finite residual after %d steps", total);
    rel = beta / beta0;
    if (rel <= o->tol || total >= o->max_iter || k == 0) break;
    if ((rc = enqueue_scale(s, s.vec(0), 1.0 / beta))) return rc;
  }
  *iters = total;
  *rel_out = rel;
  return CBS_OK;
}

}  // namespace

size_t cbs_scpml_workspace_bytes(int nx, int ny, int nz, int restart) {
  ScpmlLayout S;
  if (!find_size(nx) || !find_size(ny) || !find_size(nz)) return 0;
  return scpml_layout(nx, ny, nz, restart, S) ? S.total : 0;
}

int cbs_scpml_operator(cbs_plan_t p, const cbs_scpml* layer, const void* in, void* out,
                       void* work, size_t work_bytes) {
  int rc = check_plan(p, false);
  if (rc) return rc;
  if (!in || !out) return fail(CBS_E_INVALID, "NULL field");
  if (in == out) return fail(CBS_E_INVALID, "in and out must not alias");
  if (p->act.on) return fail(CBS_E_STATE, "a solve is in progress on this plan");
  Scpml s;
  if ((rc = scpml_setup(p, layer, 1, work, work_bytes, s))) return rc;
  // the operators are in units of the pitch: 1/d^2 gives 1/m^2
  return enqueue_delta(s, static_cast<const float2*>(in), static_cast<float2*>(out),
                       (float)(1.0 / (p->pitch * p->pitch)));
}

int cbs_solve_scpml(cbs_plan_t p, const cbs_source* src, void* E_dev, const cbs_opts* o,
                    const cbs_scpml* layer, cbs_stats* stats, void* work, size_t work_bytes) {
  int rc = check_plan(p, true);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if (!E_dev) return fail(CBS_E_INVALID, "output field is NULL");
  if (p->act.on) return fail(CBS_E_STATE, "a solve is in progress on this plan");
  if (p->sigma_max != 0.0)
    return fail(CBS_E_STATE, "the stretched layer replaces the graded potential: set the "
                             "plan's sigma_max to 0 (cbs_plan_set_pml_profile) first");
  if (o->flags & CBS_WARM_START)
    return fail(CBS_E_INVALID, "the stretched-layer solve starts from zero (no CBS_WARM_START)");
  if (!layer) return fail(CBS_E_INVALID, "layer parameters are NULL");
  Scpml s;
  if ((rc = scpml_setup(p, layer, layer->restart, work, work_bytes, s))) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  // b = gamma G S: one CBS step from zero with the solve's source
  CbsArgs a = base_args(p);
  Kvec kv;
  if ((rc = set_source(p, a, src, false, kv))) return rc;
  cbs_opts so = *o;
  so.flags = 0;
  so.tol = -1.0;            // the step count never stops the passes
  so.max_iter = INT_MAX;
  if ((rc = enqueue_solve_start(p, a, &so, src, nullptr, kv))) return rc;
  a.E = s.b;
  a.warm = 0;
  p->ox->k1(a, K1_FWD, p->stream);
  if ((rc = enqueue_iteration(p, a))) return rc;
  float2* x = static_cast<float2*>(E_dev);
  dim3 gg;
  gm_grid(s.n3, gg);
  hipLaunchKernelGGL(k_gm_copy, gg, dim3(kGmThreads), 0, p->stream, nullptr, x, s.n3);
  HIP_LAUNCHED();
  std::complex<double> bb;
  if ((rc = enqueue_dots(s, s.b, 1, s.b, s.h))) return rc;
  if ((rc = read_back(p, s.h, &bb, 1))) return rc;
  const double beta0 = std::sqrt(std::max(0.0, bb.real()));
  if (!std::isfinite(beta0)) return fail(CBS_E_DIVERGED, "non-finite source");
  std::vector<double> hist;
  int iters = 0;
  double rel = 0.0;
  if (beta0 > 0.0 && (rc = scpml_gmres(s, x, layer->restart, o, beta0, &iters, &rel, hist)))
    return rc;
  if (a.src == SRC_PLANE && !(o->flags & CBS_RETURN_SCATTERED)) {
    CbsArgs ai = a;
    ai.E = x;
    hipLaunchKernelGGL(k_incident, dim3(2048), dim3(256), 0, p->stream, ai, 1.0f);
    HIP_LAUNCHED();
  }
  DevState ds;
  HIP_TRY(hipMemcpyAsync(&ds, p->state, sizeof(DevState), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (ds.status == 3) return fail(CBS_E_DIVERGED, "non-finite field in a CBS step");
  p->hist_len = 0;
  if ((o->flags & CBS_RECORD_HISTORY) && !hist.empty()) {
    const int n = std::min<int>((int)hist.size(), kHistCap);
    HIP_TRY(hipMemcpy(p->hist, hist.data(), n * sizeof(double), hipMemcpyHostToDevice));
    p->hist_len = n;
  }
  const bool ok = rel <= o->tol;
  if (stats) {
    stats->iterations = iters;
    stats->converged = ok ? 1 : 0;
    stats->residual = rel;
    stats->eps_shift = p->eps;
    stats->ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (ok) return CBS_OK;
  g_err = "max_iter reached before the residual met tol";
  return CBS_NOT_CONVERGED;
}

int cbs_history(cbs_plan_t p, double* out, int max) {
  int rc = check_plan(p, false);
  if (rc) return rc;
  const int n = std::min(max, p->hist_len);
  if (n > 0 && out)
    HIP_TRY(hipMemcpy(out, p->hist, n * sizeof(double), hipMemcpyDeviceToHost));
  return p->hist_len;
}

int cbs_plan_destroy(cbs_plan_t p) {
  if (!p) return CBS_OK;
  // outstanding asynchronous copies target the pinned mirror: drain first
  if (p->act.on || p->act.count > 0) (void)hipStreamSynchronize(p->stream);
  (void)hipEventDestroy(p->ev0);
  (void)hipEventDestroy(p->ev1);
  for (int i = 0; i < 6; ++i) (void)hipEventDestroy(p->evp[i]);
  for (int i = 0; i < cbs_plan_s::kRing; ++i) (void)hipEventDestroy(p->evq[i]);
  (void)hipHostFree(p->mirror);
  delete p;
  return CBS_OK;
}

const char* cbs_last_error(void) { return g_err.c_str(); }

}  // extern "C"
