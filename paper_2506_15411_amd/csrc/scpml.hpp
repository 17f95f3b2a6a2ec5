// Stretched-coordinate absorbing layer (reference [31] of arXiv 2506.15411,
// named in its simulation-setup paragraph) for the spectral vector operator,
// and the vector kernels of the GMRES solve that uses it.
//
// In a stretched layer every derivative d/da becomes (1/s_a) d/da with
// s_a = 1 + i alpha_max u_a^m (u_a the depth into the layer of axis a, the
// graded potential's u).  With the solver's spectral derivatives D_a (symbol
// i p), T_a (symbol i pt, pt = p except 0 at the Nyquist bin of an even axis)
// and S_a = diag(s_a), the stretched operator differs from L = F^-1 (|p|^2 I -
// pt pt^T) F by
//
//   ((L_s - L) E)_c = sum_{b != c} A_b E_c + B_c E_c + C_c X - T_c Y,
//   X = sum_b C_b E_b,   Y = sum_b T_b E_b,
//   A_a = D_a^2 - S_a^-1 D_a S_a^-1 D_a,  B_a = T_a^2 - S_a^-1 T_a S_a^-1 T_a,
//   C_a = S_a^-1 T_a,
//
// every term a 1D operator along one axis.  Each is stored as a dense n x n
// matrix (built in FP64 on the device from the circulant columns of D, T, D^2,
// T^2) and applied to all lines of a field by a tiled complex GEMM; on a thin
// layer A and B are applied in a two-launch form over the layer's rows and
// columns instead (see kMmCompact below).  Since
// S^-1 - I vanishes outside the layer, C_c X - T_c Y is evaluated as
// T_c Z + (S_c^-1 - I) T_c X with Z = X - Y = sum_b (S_b^-1 - I) T_b E_b: one
// product T_b E_b per axis gives both X and Z, and T_c X is needed on the 2p
// layer rows only.  Work is in units of the pitch (p d in [-pi, pi]).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cbs {

constexpr int kScpmlMaxRestart = 64;   // GMRES basis <= 65 vectors
constexpr int kScpmlMaxAxis = 1024;
constexpr int kGmBlocks = 512;         // fixed grid of the FP64 dot products
constexpr int kGmThreads = 256;

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 zsub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}

// depth u in (0, 1] into a layer of p voxels on each side of an axis of n
// voxels (outermost voxel 1, first layer voxel next to the interior 1/p), else 0
__device__ __forceinline__ double stretch_depth(int i, int n, int p) {
  if (p <= 0) return 0.0;
  if (i < p) return double(p - i) / double(p);
  if (i >= n - p) return double(i - (n - p - 1)) / double(p);
  return 0.0;
}

// Circulant columns (pitch 1) of D (i p), T (i pt), D^2 (-p^2), T^2 (-pt^2)
// along one axis: col[m] = (1/n) sum_k sym_k exp(2 pi i k m / n), p_k = 2 pi
// f_k / n with f_k the FFT-order frequency (the Nyquist bin of an even axis
// negative); and 1/s over the axis.  One thread per m, FP64.
__global__ void k_scpml_columns(int n, int pml, int order, double alpha, double2* d,
                                double2* t, double2* dd, double2* tt, double2* sinv) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  double dx = 0, dy = 0, tx = 0, ty = 0, ddx = 0, ddy = 0, ttx = 0, tty = 0;
  for (int k = 0; k < n; ++k) {
    const int f = 2 * k < n ? k : k - n;
    const double p = 2.0 * M_PI * f / n;
    const double pt = (2 * k == n) ? 0.0 : p;
    const long long km = ((long long)k * m) % n;
    double s, c;
    sincospi(2.0 * (double)km / n, &s, &c);
    // (i q) (c + i s) = -q s + i q c
    dx -= p * s;
    dy += p * c;
    tx -= pt * s;
    ty += pt * c;
    ddx -= p * p * c;
    ddy -= p * p * s;
    ttx -= pt * pt * c;
    tty -= pt * pt * s;
  }
  const double inv = 1.0 / n;
  d[m] = make_double2(dx * inv, dy * inv);
  t[m] = make_double2(tx * inv, ty * inv);
  dd[m] = make_double2(ddx * inv, ddy * inv);
  tt[m] = make_double2(ttx * inv, tty * inv);
  double u = stretch_depth(m, n, pml), um = 1.0;
  for (int k = 0; k < order; ++k) um *= u;
  const double a = alpha * um;   // s = 1 + i a, 1/s = (1 - i a) / (1 + a^2)
  sinv[m] = make_double2(1.0 / (1.0 + a * a), -a / (1.0 + a * a));
}

// The three n x n operators of one axis, row-major FP32:
//   A = D^2 - S^-1 D S^-1 D,  B = T^2 - S^-1 T S^-1 T,  T,
// and 1/s in FP32 (C = S^-1 T is applied as 1/s times the T product).
// (S^-1 D S^-1 D)_ij = s_i^-1 (D^2_ij + sum_{k in layer} D_ik (s_k^-1 - 1) D_kj):
// only layer voxels have s_k != 1.  One thread per entry, FP64.
__global__ void k_scpml_matrices(int n, int pml, const double2* d, const double2* t,
                                 const double2* dd, const double2* tt, const double2* sinv,
                                 float2* A, float2* B, float2* T, float2* sinv32) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  if (j == 0) sinv32[i] = make_float2((float)sinv[i].x, (float)sinv[i].y);
  const int ij = ((i - j) % n + n) % n;
  double2 sd = make_double2(0, 0), st = make_double2(0, 0);
  auto layer_term = [&](int k) {
    const double2 w = make_double2(sinv[k].x - 1.0, sinv[k].y);
    const int ik = ((i - k) % n + n) % n, kj = ((k - j) % n + n) % n;
    sd = zadd(sd, zmul(zmul(d[ik], w), d[kj]));
    st = zadd(st, zmul(zmul(t[ik], w), t[kj]));
  };
  const int p = pml < 0 ? 0 : pml;
  for (int k = 0; k < p; ++k) layer_term(k);
  for (int k = n - p; k < n; ++k)
    if (k >= p) layer_term(k);
  const double2 si = sinv[i];
  const double2 a = zsub(dd[ij], zmul(si, zadd(dd[ij], sd)));
  const double2 b = zsub(tt[ij], zmul(si, zadd(tt[ij], st)));
  A[e] = make_float2((float)a.x, (float)a.y);
  B[e] = make_float2((float)b.x, (float)b.y);
  T[e] = make_float2((float)t[ij].x, (float)t[ij].y);
}

// Tables of a thin layer (8p <= n) for the two-launch form of A and B, written
// over the dense A and B (6pn <= n^2 entries each): RA = [D[L, :]; D^2[L, :]]
// (4p x n) then CA = D[:, L] (n x 2p), and RB, CB the same with T and T^2.
// Layer voxel q < 2p is axis voxel q (q < p) or q + n - 2p.  One thread per
// entry, FP64 columns rounded to FP32.
__global__ void k_scpml_thin(int n, int p, const double2* d, const double2* t,
                             const double2* dd, const double2* tt, float2* RA, float2* RB) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long rows = 4LL * p * n, total = 6LL * p * n;
  if (e >= total) return;
  auto lrow = [&](int q) { return q < p ? q : q + (n - 2 * p); };
  double2 va, vb;
  if (e < rows) {
    const int r = (int)(e / n), j = (int)(e % n);
    const bool sq = r >= 2 * p;
    const int i = lrow(sq ? r - 2 * p : r);
    const int ij = ((i - j) % n + n) % n;
    va = sq ? dd[ij] : d[ij];
    vb = sq ? tt[ij] : t[ij];
  } else {
    const long long e2 = e - rows;
    const int i = (int)(e2 / (2 * p)), q = (int)(e2 % (2 * p));
    const int ij = ((i - lrow(q)) % n + n) % n;
    va = d[ij];
    vb = t[ij];
  }
  RA[e] = make_float2((float)va.x, (float)va.y);
  RB[e] = make_float2((float)vb.x, (float)vb.y);
}

// Products of one n x n matrix M with every line of a scalar [nz][ny][nx] field
// along one axis of length n: element i of line l sits at (l / Q) n Q + l % Q
// + i Q (Q = 1 along x, nx along y, nx ny along z).  With acc(l, i) = sum_j
// M[i][j] in(l, j), the epilogue is one of
//   kMmPlain:  out = alpha acc               (+ out if accumulate)
//   kMmSplit:  out = alpha s_i acc,  out2 = alpha (s_i - 1) acc   (+= each if accumulate)
//   kMmLayer:  out += alpha (s_i - 1) acc, for the 2p layer rows i only
// where s_i is 1/s at voxel i of the axis (FP32).  Tiles of 64 lines x 64
// outputs, j staged through LDS 32 at a time.
//
// An axis whose layer is thin (8p <= n) applies A and B in two narrow products
// instead of one dense one.  With lambda = 1 - 1/s (non-zero on the 2p layer
// voxels L only), A = D^2 - S^-1 D S^-1 D is
//   A v = lambda (D^2 v) + S^-1 D[:, L] (lambda_L (D v)_L)
// (B the same with T): the layer rows of D and D^2 times v (4p rows, K = n),
// then D's layer columns times 2p values per line (n rows, K = 2p).  The two
// launches use
//   kMmCompact: out[l][r] = alpha lambda acc for the 4p stacked layer rows r
//               (D rows, then D^2 rows), a compact [lines][4p] buffer;
//   kMmColFix:  out += alpha (s_i acc + [i in L] aux[l][2p + q(i)]), the input
//               the first 2p values of each compact line and aux that buffer.
enum : int { kMmPlain = 0, kMmSplit = 1, kMmLayer = 2, kMmCompact = 3, kMmColFix = 4 };

struct AxisMM {
  const float2* M;
  const float2* in;
  float2* out;
  float2* out2;         // kMmSplit
  const float2* sinv;   // 1/s along the axis
  const float2* aux;    // kMmColFix: the compact buffer of kMmCompact
  int n, Q;
  int rows;             // output rows computed: n, 2p (kMmLayer) or 4p (kMmCompact)
  int K;                // reduction length: n, or 2p (kMmColFix)
  int ldm;              // row stride of M
  int p;                // layer voxels per side
  long long in_ld;      // > 0: compact input, line l at in + l in_ld (j contiguous)
  long long cld;        // line stride of the compact buffers (4p)
  long long L;          // lines
  float alpha;
  int accumulate;
  int mode;
};

constexpr int kMmTL = 64, kMmTI = 64, kMmTJ = 32;

__device__ __forceinline__ long long axis_addr(long long l, int i, int n, int Q) {
  return (l / Q) * (long long)n * Q + l % Q + (long long)i * Q;
}

// output row r of the launch -> row i of the matrix (the layer rows for kMmLayer)
__device__ __forceinline__ int mm_row(const AxisMM& a, int r) {
  return (a.mode == kMmLayer && r >= a.p) ? r + (a.n - 2 * a.p) : r;
}

typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// The complex products run on the FP32 matrix cores: v_mfma_f32_16x16x4_f32
// multiplies a 16 x 4 block A (lane l holds A[l % 16][l / 16]) by a 4 x 16 block
// B (lane l holds B[l / 16][l % 16]) into a 16 x 16 block D (lane l holds
// D[4 (l / 16) + r][l % 16] in register r).  A complex block product takes three
// (Gauss's form): P1 += Mr Xr, P2 += Mi Xi, P3 += (Mr + Mi)(Xr + Xi), and then
// Re = P1 - P2, Im = P3 - P1 - P2.  Each of the four waves of a work-group owns
// a 32 x 32 part of the 64 x 64 output tile (2 x 2 blocks).  ROWWISE (Q = 1,
// the x axis): a line's elements j are contiguous in memory; otherwise
// consecutive lines are, and the loads run along the lines.
template <bool ROWWISE>
__global__ void __launch_bounds__(256) k_axis_mm(AxisMM a) {
  __shared__ float2 sIn[kMmTJ][kMmTL + 1];
  __shared__ float2 sM[kMmTJ][kMmTI + 1];
  const int tid = threadIdx.x;
  // block -> (line tile, row tile) with the row tiles of one line tile adjacent
  // in the XCD-remapped order, so the line tile they all read stays in one L2
  const unsigned rtiles = (unsigned)((a.rows + kMmTI - 1) / kMmTI);
  const unsigned Lb = xcd_remap(blockIdx.x, gridDim.x);
  const long long l0 = (long long)(Lb / rtiles) * kMmTL;
  const int r0 = (int)(Lb % rtiles) * kMmTI;
  const int lane = tid & 63, wave = tid >> 6;
  const int wi = (wave & 1) * 32, wl = (wave >> 1) * 32;   // this wave's rows i, lines l
  const int lr = lane & 15, lk = lane >> 4;
  mfma_f4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int lb = 0; lb < 2; ++lb) {
      p1[ib][lb] = mfma_f4{0.f, 0.f, 0.f, 0.f};
      p2[ib][lb] = mfma_f4{0.f, 0.f, 0.f, 0.f};
      p3[ib][lb] = mfma_f4{0.f, 0.f, 0.f, 0.f};
    }

  // the next stage's tiles are fetched into registers while the matrix cores
  // work on the current one
  constexpr int kIn = (kMmTL * kMmTJ) / 256, kMt = (kMmTI * kMmTJ) / 256;
  float2 pin[kIn], pm[kMt];
  // input element e of this thread (idx = tid + 256 e): along x, line
  // tl + 8 e at j0 + tj; otherwise line tl (the same for every e) at
  // j0 + tj + 4 e.  The line's base address is formed once, outside the loop.
  // Loads are unconditional: an element outside the field or the matrix reads
  // element 0 instead and is replaced by zero.
  constexpr int kLineStep = 256 / kMmTJ, kJStep = 256 / kMmTL, kRowStep = 256 / kMmTJ;
  const int tj = ROWWISE ? tid % kMmTJ : tid / kMmTL;
  const long long tl = l0 + (ROWWISE ? tid / kMmTJ : tid % kMmTL);
  const long long lstride = a.in_ld > 0 ? a.in_ld : (long long)a.n;   // ROWWISE line stride
  const long long lbase = ROWWISE ? tl * lstride : axis_addr(tl, 0, a.n, a.Q);
  unsigned lok = 0;   // bit e: the line of input element e exists
#pragma unroll
  for (int e = 0; e < kIn; ++e)
    if ((ROWWISE ? tl + kLineStep * e : tl) < a.L) lok |= 1u << e;
  const int ti = tid / kMmTJ, tjm = tid % kMmTJ;   // matrix element e: row r0 + ti + 8 e
  long long mrow[kMt];
  unsigned rok = 0;
#pragma unroll
  for (int e = 0; e < kMt; ++e) {
    const int r = r0 + ti + kRowStep * e;
    mrow[e] = (long long)mm_row(a, r < a.rows ? r : 0) * a.ldm;
    if (r < a.rows) rok |= 1u << e;
  }
  auto fetch = [&](int j0) {
#pragma unroll
    for (int e = 0; e < kIn; ++e) {
      const int j = ROWWISE ? j0 + tj : j0 + tj + kJStep * e;
      const bool ok = ((lok >> e) & 1u) && j < a.K;
      const long long ad = ROWWISE ? lbase + (long long)(kLineStep * e) * lstride + j
                                   : lbase + (long long)j * a.Q;
      const float2 v = a.in[ok ? ad : 0];
      pin[e] = ok ? v : make_float2(0.f, 0.f);
    }
    const int jm = j0 + tjm;
#pragma unroll
    for (int e = 0; e < kMt; ++e) {
      const bool ok = ((rok >> e) & 1u) && jm < a.K;
      const float2 v = a.M[ok ? mrow[e] + jm : 0];
      pm[e] = ok ? v : make_float2(0.f, 0.f);
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int e = 0; e < kIn; ++e) {
      const int idx = tid + 256 * e;
      const int jj = ROWWISE ? idx % kMmTJ : idx / kMmTL;
      const int ll = ROWWISE ? idx / kMmTJ : idx % kMmTL;
      sIn[jj][ll] = pin[e];
    }
#pragma unroll
    for (int e = 0; e < kMt; ++e) {
      const int idx = tid + 256 * e;
      sM[idx % kMmTJ][idx / kMmTJ] = pm[e];
    }
  };
  fetch(0);
  for (int j0 = 0; j0 < a.K; j0 += kMmTJ) {
    stash();
    __syncthreads();
    if (j0 + kMmTJ < a.K) fetch(j0 + kMmTJ);
#pragma unroll
    for (int ks = 0; ks < kMmTJ / 4; ++ks) {
      const int k = 4 * ks + lk;
      float2 am[2], bx[2];
      float ams[2], bxs[2];
#pragma unroll
      for (int ib = 0; ib < 2; ++ib) {
        am[ib] = sM[k][wi + 16 * ib + lr];
        ams[ib] = am[ib].x + am[ib].y;
      }
#pragma unroll
      for (int lb = 0; lb < 2; ++lb) {
        bx[lb] = sIn[k][wl + 16 * lb + lr];
        bxs[lb] = bx[lb].x + bx[lb].y;
      }
#pragma unroll
      for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int lb = 0; lb < 2; ++lb) {
          p1[ib][lb] = __builtin_amdgcn_mfma_f32_16x16x4f32(am[ib].x, bx[lb].x, p1[ib][lb], 0, 0, 0);
          p2[ib][lb] = __builtin_amdgcn_mfma_f32_16x16x4f32(am[ib].y, bx[lb].y, p2[ib][lb], 0, 0, 0);
          p3[ib][lb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ams[ib], bxs[lb], p3[ib][lb], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  long long obase[2];
#pragma unroll
  for (int lb = 0; lb < 2; ++lb) obase[lb] = axis_addr(l0 + wl + 16 * lb + lr, 0, a.n, a.Q);
  // Epilogue in two phases: the values of out that the outputs add to are all
  // loaded first, so one thread's loads are in flight together instead of each
  // waiting behind the previous output's store (out2 and the compact buffer,
  // read by fewer outputs, are loaded in the second phase).
  const bool add_out = a.mode == kMmColFix || a.mode == kMmLayer ||
                       (a.accumulate && (a.mode == kMmPlain || a.mode == kMmSplit));
  float2 u1[2][2][4];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int lb = 0; lb < 2; ++lb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long long l = l0 + wl + 16 * lb + lr;
        const int rr = r0 + wi + 16 * ib + 4 * lk + q;
        u1[ib][lb][q] = make_float2(0.f, 0.f);
        if (add_out && l < a.L && rr < a.rows)
          u1[ib][lb][q] = a.out[obase[lb] + (long long)mm_row(a, rr) * a.Q];
      }
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int lb = 0; lb < 2; ++lb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long long l = l0 + wl + 16 * lb + lr;
        const int rr = r0 + wi + 16 * ib + 4 * lk + q;
        if (l < a.L && rr < a.rows) {
          const float re = p1[ib][lb][q] - p2[ib][lb][q];
          const float im = p3[ib][lb][q] - p1[ib][lb][q] - p2[ib][lb][q];
          const float2 v = make_float2(a.alpha * re, a.alpha * im);
          const float2 u = u1[ib][lb][q];
          if (a.mode == kMmCompact) {
            // stacked row rr -> layer voxel q (D rows, then D^2 rows) -> axis voxel
            const int ql = rr < 2 * a.p ? rr : rr - 2 * a.p;
            const float2 si = a.sinv[ql < a.p ? ql : ql + (a.n - 2 * a.p)];
            a.out[l * a.cld + rr] = cmul(make_float2(1.0f - si.x, -si.y), v);
            continue;
          }
          const int i = mm_row(a, rr);
          const long long o = obase[lb] + (long long)i * a.Q;
          if (a.mode == kMmColFix) {
            float2 w = cmul(a.sinv[i], v);
            if (i < a.p || i >= a.n - a.p) {   // the compact D^2 term on the layer rows
              const int ql = i < a.p ? i : i - (a.n - 2 * a.p);
              const float2 z = a.aux[l * a.cld + 2 * a.p + ql];
              w.x += a.alpha * z.x;
              w.y += a.alpha * z.y;
            }
            a.out[o] = make_float2(u.x + w.x, u.y + w.y);
          } else if (a.mode == kMmPlain) {
            a.out[o] = make_float2(v.x + u.x, v.y + u.y);
          } else if (a.mode == kMmLayer) {
            const float2 si = a.sinv[i];
            const float2 w2 = cmul(make_float2(si.x - 1.0f, si.y), v);   // (1/s - 1) acc
            a.out[o] = make_float2(w2.x + u.x, w2.y + u.y);
          } else {   // kMmSplit
            const float2 si = a.sinv[i];
            const float2 w = cmul(si, v), w2 = cmul(make_float2(si.x - 1.0f, si.y), v);
            const float2 u2 = a.accumulate ? a.out2[o] : make_float2(0.f, 0.f);
            a.out[o] = make_float2(w.x + u.x, w.y + u.y);
            a.out2[o] = make_float2(w2.x + u2.x, w2.y + u2.y);
          }
        }
      }
}

// ---------------------------------------------------------------------------
// GMRES vector kernels: fields of n complex FP32 values, reductions in FP64
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 block_sum_z(double sx, double sy, double2* red) {
  for (int o = 32; o > 0; o >>= 1) {
    sx += __shfl_down(sx, o);
    sy += __shfl_down(sy, o);
  }
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  if (lane == 0) red[wv] = make_double2(sx, sy);
  __syncthreads();
  double2 r = make_double2(0, 0);
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)blockDim.x / 64; ++k) r = zadd(r, red[k]);
  return r;   // valid in thread 0
}

// part[i][blk] = partial of sum_e conj(V_i[e]) w[e], i = blockIdx.y; fixed grid,
// fixed order, so the result does not depend on timing
__global__ void __launch_bounds__(kGmThreads)
k_gm_dots(const float2* V, long long vstride, const float2* w, long long n, double2* part) {
  __shared__ double2 red[kGmThreads / 64];
  const float2* v = V + blockIdx.y * vstride;
  double sx = 0, sy = 0;
  for (long long e = (long long)blockIdx.x * kGmThreads + threadIdx.x; e < n;
       e += (long long)gridDim.x * kGmThreads) {
    const float2 a = v[e], b = w[e];
    sx += (double)a.x * b.x + (double)a.y * b.y;
    sy += (double)a.x * b.y - (double)a.y * b.x;
  }
  const double2 r = block_sum_z(sx, sy, red);
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = r;
}

// h[i] = sum over blocks of part[i][.], one work-group per i
__global__ void __launch_bounds__(kGmThreads)
k_gm_dots_finish(const double2* part, int nblk, double2* h) {
  __shared__ double2 red[kGmThreads / 64];
  const double2* p = part + blockIdx.x * nblk;
  double sx = 0, sy = 0;
  for (int k = threadIdx.x; k < nblk; k += kGmThreads) {
    sx += p[k].x;
    sy += p[k].y;
  }
  const double2 r = block_sum_z(sx, sy, red);
  if (threadIdx.x == 0) h[blockIdx.x] = r;
}

// w += sign sum_{i < cnt} c_i V_i, coefficients c (FP64) in device memory
__global__ void __launch_bounds__(kGmThreads)
k_gm_update(const float2* V, long long vstride, int cnt, const double2* c, float sign,
            float2* w, long long n) {
  __shared__ float2 cf[kScpmlMaxRestart + 1];
  if (threadIdx.x < cnt)
    cf[threadIdx.x] = make_float2((float)(sign * c[threadIdx.x].x), (float)(sign * c[threadIdx.x].y));
  __syncthreads();
  for (long long e = (long long)blockIdx.x * kGmThreads + threadIdx.x; e < n;
       e += (long long)gridDim.x * kGmThreads) {
    float2 acc = w[e];
    for (int i = 0; i < cnt; ++i) {
      const float2 v = V[i * vstride + e];
      acc.x = fmaf(cf[i].x, v.x, fmaf(-cf[i].y, v.y, acc.x));
      acc.y = fmaf(cf[i].x, v.y, fmaf(cf[i].y, v.x, acc.y));
    }
    w[e] = acc;
  }
}

// w = s w
__global__ void k_gm_scale(float2* w, long long n, float s) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const float2 v = w[e];
    w[e] = make_float2(s * v.x, s * v.y);
  }
}

// w = a - w
__global__ void k_gm_rsub(const float2* a, float2* w, long long n) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const float2 x = a[e], v = w[e];
    w[e] = make_float2(x.x - v.x, x.y - v.y);
  }
}

// dst = src (or 0 when src is null)
__global__ void k_gm_copy(const float2* src, float2* dst, long long n) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = src ? src[e] : make_float2(0.f, 0.f);
}

}  // namespace cbs
