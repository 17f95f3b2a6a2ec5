// CBS iteration kernels for gfx950.
//
// One CBS iteration (vector CBS of references [25]/[26] of arXiv 2506.15411)
//     W = V E_s + S;  GW = F^-1 G^ F W;  E_s += gamma (GW - E_s)
// runs as four passes over HBM, each a batch of 1D FFTs along one axis:
//
//   KY(-)  forward FFT along y                               (W in place)
//   KZ     forward FFT along z, G^(p) 3x3 multiply (1/N folded in),
//          inverse FFT along z; all three components of a z-column
//          are in one workgroup                              (W in place)
//   KY(+)  inverse FFT along y                               (W in place)
//   K1     inverse FFT along x -> GW, CBS update of E_s with FP64 residual
//          partials, W = V E_s + S for the next iteration, forward FFT
//          along x                                           (W, E_s)
//
// Every 1D transform of length n = N1 * N2 is two register levels joined by
// one exchange through LDS: level A does N2 DFT-N1 over stride-N2 subsets
// (one per thread) and multiplies by exp(-+2 pi i j2 k1 / n); level B does
// N1 DFT-N2 over the contiguous groups (one per thread).  Level A writes its
// results to the LDS slots its inputs came from, so each exchange needs one
// buffer and one barrier.  The inter-level twiddles come from an FP64-built
// table stored [j2][k1], so each thread's twiddles are contiguous.  In K1 the
// inverse transform ends with thread t holding GW[t + N1 m]; the forward
// transform of the next W is chosen with the transposed split (DFT-N2 over
// exactly those elements first), so the update and the start of the forward
// transform run in registers without an LDS round trip.  In KZ the forward
// level B leaves each thread with all z-frequencies k1 + N1 k2 of its group
// for the three components, the Green multiply and the inverse level B run on
// those registers, and the z spectrum is never reordered.
//
// Work is in units of the voxel pitch: lengths are scaled by 1/d, potentials
// by d^2 (p d in [-pi, pi], kb^2 d^2, eps d^2), which leaves E_s unchanged.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "codelets.hpp"

namespace cbs {

enum SrcKind : int { SRC_NONE = 0, SRC_PLANE = 1, SRC_FIELD = 2, SRC_POINT = 3, SRC_FIELD_CONJ = 4 };
enum K1Mode : int { K1_FWD = 0, K1_ITER = 1, K1_INV = 2 };

constexpr int kHistCap = 1 << 16;
// Illuminations one batched solve advances together (same medium, own sources).
constexpr int kMaxIllum = 8;

// The spectral work field W is stored in bricks of 8 x-columns:
//   W[c][z][x / 8][y][x % 8]   (x padded to nxp = 8 * gx columns)
// so a y-pass tile (8 columns x ny rows) is one contiguous block, a z-pass
// column of one brick row is a 64-byte piece per plane (rows y and y+1 share a
// 128-byte line), and R consecutive rows of an x-line form 64 R-byte pieces.
constexpr int kBrick = 8;

// Wave priority a pass raises to while its work-groups issue their first
// loads, where few waves share a SIMD (x pass: at most two, y pass: at most
// three; the launchers decide from the occupancy API).
constexpr int kLoadPrio = 2;

// Device-resident solve state (lives in the workspace).
struct DevState {
  int done;        // 1: stop iterating (kernels return at entry)
  int iter;        // iterations applied
  int status;      // 0 running, 1 converged, 2 max_iter, 3 diverged
  int max_iter;
  double tol;
  double eta;      // last relative update norm
  float2 amp[3];   // point-source amplitude (already scaled by d^2)
  int record;      // keep eta history
  int pending;     // the x pass wrote residual partials that are not reduced yet
  double eta_b[kMaxIllum];   // last relative update norm of each illumination
};

// Fixed-order sum of the per-block partials, then the stopping rule.  The
// partials are summed in kResStreams interleaved streams (stream s takes
// partials s, s + kResStreams, ... in order), the stream sums are combined by
// one wave in a fixed order, so the result is the same double whichever kernel
// and block shape runs it (the lagged reduction in the y pass and the
// quantum-end k_residual must agree bit for bit: which of them reduces a given
// iteration depends on where the host's quanta end).  A batched solve has nb
// illuminations with per_b partials each: each gets its own eta, and the solve
// stops when the largest meets tol.  red holds 2 kResStreams doubles of LDS;
// THREADS is any multiple of 64.
constexpr int kResStreams = 256;
template <int THREADS>
__device__ __forceinline__ void residual_finish(const double* part, int per_b, int nb,
                                                DevState* st, double* hist, double* red) {
  static_assert(THREADS % 64 == 0, "whole waves");
  double eta = 0.0;      // the largest eta (meaningful in thread 0)
  bool bad = false;      // a non-finite eta
  for (int ib = 0; ib < nb; ++ib) {
    const double* pb = part + 2LL * ib * per_b;
    for (int s = threadIdx.x; s < kResStreams; s += THREADS) {
      double a = 0.0, b = 0.0;
      for (int i = s; i < per_b; i += kResStreams) {
        a += __builtin_nontemporal_load(pb + 2 * i);
        b += __builtin_nontemporal_load(pb + 2 * i + 1);
      }
      red[s] = a;
      red[kResStreams + s] = b;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      const int l = threadIdx.x;
      double nd = red[l], ne = red[kResStreams + l];
      #pragma unroll
      for (int q = 64; q < kResStreams; q += 64) {
        nd += red[l + q];
        ne += red[kResStreams + l + q];
      }
      #pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        nd += __shfl_xor(nd, o, 64);
        ne += __shfl_xor(ne, o, 64);
      }
      if (l == 0) {
        double e;
        if (ne > 0.0)
          e = sqrt(nd / ne);
        else
          e = (nd == 0.0) ? 0.0 : INFINITY;
        st->eta_b[ib] = e;
        if (!isfinite(e)) bad = true;
        else if (e > eta) eta = e;
      }
    }
    __syncthreads();   // red is rewritten for the next illumination
  }
  if (threadIdx.x == 0) {
    if (bad) eta = NAN;
    {
      const int it = st->iter + 1;
      st->iter = it;
      st->eta = eta;
      if (st->record && it <= kHistCap) hist[it - 1] = eta;
      if (!isfinite(eta)) {
        st->status = 3;
        st->done = 1;
      } else if (eta <= st->tol) {
        st->status = 1;
        st->done = 1;
      } else if (it >= st->max_iter) {
        st->status = 2;
        st->done = 1;
      }
    }
  }
}

struct CbsArgs {
  int nx, ny, nz, nxp;          // grid, padded row length of W (kBrick * gx)
  int gx, gy;                   // x bricks (nxp / kBrick), x-pass row groups (ceil(ny / rows))
  int px, py, pz;               // absorbing layer per side
  long long sW;                 // component stride of W  (nz * ny * nxp)
  long long sE;                 // component stride of E  (nz * ny * nx)
  float2* W;                    // spectral work field, bricked (see kBrick)
  float2* E;                    // E_s, caller layout [3][nz][ny][nx]
  const float2* V0;             // unshifted potential * d^2, [nz][ny][nx]
  const float2* twx;            // x split n1 x n2: twx[j2 n1 + k1] = exp(-2 pi i j2 k1 / nx)
  const float2* twy;            // same layout for the y split
  const float2* twz;            // same layout for the z split
  const float2* phase;          // [nb][3][nz] pol_c exp(i kz d z) of each illumination's wave
  const float2* fin;            // FIELD source / Green input
  float2* fout;                 // Green output
  double* partials;             // 2 doubles per K1 block
  int k1_blocks;                // K1 blocks per illumination (partials to reduce for each)
  int nb;                       // illuminations advanced together (1: an ordinary solve)
  long long sWb, sEb;           // stride between illuminations in W (3 sW) and E (3 sE)
  const float2* phx;            // [nb][nx] exp(i kx d x) of each illumination's plane wave
  const float2* phy;            // [nb][ny] exp(i ky d y)
  int oblique;                  // some illumination has kx or ky != 0 (phx, phy not all 1)
  int k1_prio;                  // x-pass: raise wave priority for the load phase (set by launch_k1)
  int ky_prio;                  // y pass: the same (set by launch_ky)
  double* hist;                 // residual history
  DevState* st;
  int src;                      // SrcKind
  int warm;                     // K1_FWD: W = V E + S from E (else E = 0)
  int green_in;                 // K1_FWD: W = fin
  int r0x, r0y, r0z;
  float src_scale;              // d^2: physical (1/m^2) sources and Green inputs
  float eps, inv_eps, kb2;      // eps d^2, 1/(eps d^2), kb^2 d^2
  float pfx, pfy, pfz;          // 2 pi / n_a
  float invN;                   // 1 / (nx ny nz)
};

// ---------------------------------------------------------------------------
// per-size geometry of the passes
// ---------------------------------------------------------------------------
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int round64(int t) { return (t + 63) / 64 * 64; }

// Rows per x-pass workgroup: TM threads serve one row.  The iteration kernel
// needs about 200 VGPRs (two waves per SIMD), so workgroups of at most two
// waves pack the CU fully; among R = 1..8 with R TM <= 128 pick the one whose
// lanes fill their waves best, the larger R on ties (measured: 621 = 27 x 23
// best at R = 4, 275 = 25 x 11 at R = 5; three-wave groups of R = 7 lose a
// quarter of the occupancy and run 10% slower).
constexpr int k1_rows_for(int tm) {
  int best = 1;
  for (int r = 2; r <= 8 && r * tm <= 128; ++r)
    if (r * tm * round64(best * tm) >= best * tm * round64(r * tm)) best = r;
  return best;
}
// Columns per z-pass workgroup: a whole brick row (8) unless the exchange
// buffer of 3 components x 8 columns (160 KB of LDS per CU) leaves room for
// fewer than three workgroups and those hold fewer than 12 waves per CU; then
// half a brick row (measured at 315: split 35 x 9 0.39 ms with 4 columns against
// 0.46 ms with 8; split 15 x 21, 8 waves per workgroup, 0.27 ms with 8 columns
// against 0.34 ms with 4).
constexpr int kz_tx_for(int n1, int n2) {
  const int n = n1 * n2;
  const int lds8 = 3 * n * 8 * 8 + n * 8;
  if (lds8 <= 53 * 1024) return 8;
  const int waves8 = round64(8 * cmax(3 * n2, n1)) / 64;
  return waves8 * ((160 * 1024) / lds8) >= 12 ? 8 : 4;
}

template <int N1, int N2>
struct XGeom {
  static constexpr int N = N1 * N2;
  static constexpr int TM = cmax(N1, N2);
  static constexpr int LINES = k1_rows_for(TM);
  static constexpr int THREADS = round64(LINES * TM);
};
template <int N1, int N2, int TX>
struct YGeom {
  static constexpr int N = N1 * N2;
  static constexpr int TM = cmax(N1, N2);
  static constexpr int THREADS = round64(TX * TM);
};
template <int N1, int N2, int TX>
struct ZGeom {
  static constexpr int N = N1 * N2;
  static constexpr int TM = cmax(3 * N2, N1);
  static constexpr int THREADS = round64(TX * TM);
};

// dimensionless frequency 2 pi m / n of FFT index k (m in FFT order) and the
// same with the Nyquist index of an even axis flagged
__device__ __forceinline__ float freq_of(int k, int n, float pf, bool& nyq) {
  const int m = (k < (n + 1) / 2) ? k : k - n;
  nyq = ((n & 1) == 0) && (2 * k == n);
  return pf * float(m);
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b mod 8), and each XCD has its own L2.  The y and z passes read 64-byte
// column tiles, half a 128-byte L2 line; remapping the linear block index so
// that each XCD walks a contiguous range of tiles puts both halves of a line
// in the same L2 at about the same time.  Bijective for any block count.
constexpr int kXcds = 8;
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned total) {
  const unsigned q = total / kXcds, r = total % kXcds;
  const unsigned k = b % kXcds, j = b / kXcds;
  return k * q + (k < r ? k : r) + j;
}

// A pass's inter-level twiddle table is copied to LDS by every workgroup.
// Staged: issue() starts all of this thread's table loads at once, the caller
// then issues its first data loads, and commit() writes the table to LDS
// before the barrier, so the table's latency overlaps the data loads instead
// of preceding them.
template <int N, int THREADS>
struct TwStage {
  static constexpr int K = (N + THREADS - 1) / THREADS;
  float2 v[K];
  // rounds that lie wholly inside the table need no bounds test
  template <int I>
  static constexpr bool kFull = (I + 1) * THREADS <= N;
  __device__ __forceinline__ void issue(const float2* g, int tid) {
    sfor<0, K>([&](auto I) {
      const int i = tid + CV(I) * THREADS;
      if (kFull<CV(I)> || i < N) v[CV(I)] = g[i];
    });
  }
  __device__ __forceinline__ void commit(float2* s, int tid) const {
    sfor<0, K>([&](auto I) {
      const int i = tid + CV(I) * THREADS;
      if (kFull<CV(I)> || i < N) s[i] = v[CV(I)];
    });
  }
};

// ---------------------------------------------------------------------------
// block reduction of two doubles (residual partials)
// ---------------------------------------------------------------------------
template <int THREADS>
__device__ __forceinline__ void block_sum2(double a, double b, double* red, double* out) {
  #pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[2 * wv] = a;
    red[2 * wv + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < THREADS / 64; ++w) {
      sa += red[2 * w];
      sb += red[2 * w + 1];
    }
    out[0] = sa;
    out[1] = sb;
  }
}

// ---------------------------------------------------------------------------
// K1: x-pass with the fused CBS update
// ---------------------------------------------------------------------------
// A workgroup transforms R consecutive rows (y0 .. y0+R-1) of one component
// at one z.  W is read and written in place in its bricks: element x of row y
// sits at brick x/8, offset 8 y + x%8, so the R rows of one brick form one
// contiguous 64 R-byte piece.  The inverse transform, the update and the
// forward transform share one LDS exchange buffer per row.
// OBL: some illumination is oblique, so the plane-wave source carries a per-
// element x phase (a separate instantiation keeps it out of the normal path)
template <int N1, int N2, int MODE, bool OBL>
__global__ void __launch_bounds__((XGeom<N1, N2>::THREADS))
k1_xpass(CbsArgs a) {
  using G = XGeom<N1, N2>;
  constexpr int N = G::N, TM = G::TM, R = G::LINES;
  __shared__ float2 lds[R * N];     // R rows of one component, natural x order
  __shared__ double red[2 * (G::THREADS / 64)];

  if (MODE == K1_ITER && a.st->done) return;

  const int tid = threadIdx.x;
  // with few waves per SIMD, a work-group's load phase would otherwise wait
  // behind the other waves' vector work
  if (a.k1_prio) __builtin_amdgcn_s_setprio(kLoadPrio);
  __shared__ float2 tw[N];
  TwStage<N, G::THREADS> tws;
  tws.issue(a.twx, tid);

  // block -> (illumination, component, row group, z); the 3 nb components of
  // the same rows are adjacent in the remapped order so V0 is shared in one L2
  const unsigned per = 3u * (unsigned)a.nb;
  const unsigned L = xcd_remap(blockIdx.x, per * (unsigned)a.gy * (unsigned)a.nz);
  const int cc = (int)(L % per);
  const int ib = cc / 3, c = cc - 3 * ib;
  const unsigned rest = L / per;
  const int yg = (int)(rest % (unsigned)a.gy);
  const int z = (int)(rest / (unsigned)a.gy);
  const int y0 = yg * R;
  const int rv = (a.ny - y0) < R ? (a.ny - y0) : R;   // valid rows in this group

  const int t = tid % TM;
  const int line = tid / TM;
  const bool ok = (line < rv);
  const int y = y0 + (ok ? line : 0);
  float2* Lr = lds + (line < R ? line : 0) * N;
  // W bricks of this (component, z, row group): brick xt starts at wb + xt * ny * 8
  float2* wb = a.W + ib * a.sWb + c * a.sW + ((long long)z * a.gx * a.ny + y0) * kBrick;
  const long long bstride = (long long)a.ny * kBrick;
  const long long ebase = ib * a.sEb + c * a.sE + ((long long)z * a.ny + y) * a.nx;  // E / fin / fout row
  const long long vbase = ((long long)z * a.ny + y) * a.nx;             // V0 row

  float2 v[N2];  // thread t (< N1): element t + N1 m, m < N2
  // early loads of the pointwise operands V0 and E_s (their latency hides
  // behind the inverse transform)
  constexpr bool PF = (MODE == K1_ITER);
  float2 pv[PF ? N2 : 1], pe[PF ? N2 : 1];
  const float2* v0t = a.V0 + vbase + t;   // this thread's elements are t + N1 m
  float2* et = a.E + ebase + t;
  if constexpr (PF) {
    if (ok && t < N1) {
      sfor<0, N2>([&](auto M) { pv[CV(M)] = v0t[N1 * CV(M)]; });
      sfor<0, N2>([&](auto M) { pe[CV(M)] = et[N1 * CV(M)]; });
    }
  }

  // element x of this thread's row in the bricks
  float2* wrow = wb + line * kBrick;
  auto wat = [&](int x) -> float2& { return wrow[(x / kBrick) * bstride + (x % kBrick)]; };
  // inverse level A input: thread j2 = t < N2 holds row[j2 + N2 j1]
  float2 b[N1];
  auto load_a = [&]() {
    if (ok && t < N2) sfor<0, N1>([&](auto J1) { b[CV(J1)] = wat(t + N2 * CV(J1)); });
  };
  if constexpr (MODE != K1_FWD) load_a();
  tws.commit(tw, tid);
  __syncthreads();   // the twiddle table is in LDS
  if (a.k1_prio) __builtin_amdgcn_s_setprio(0);

  if constexpr (MODE != K1_FWD) {
    // inverse level A: DFT-N1 over row[j2 + N2 j1]
    if (ok && t < N2) {
      dft<N1, +1>(b);
      const float2* twt = tw + t * N1;   // exp(-2 pi i t k1 / N), conjugated below
      sfor<0, N1>([&](auto K1) { b[CV(K1)] = cmulc(b[CV(K1)], twt[CV(K1)]); });
      sfor<0, N1>([&](auto K1) { Lr[t + N2 * CV(K1)] = b[CV(K1)]; });
    }
    __syncthreads();
    // inverse level B: thread k1 = t < N1, DFT-N2 over Lr[N2 k1 + j2]
    if (ok && t < N1) {
      sfor<0, N2>([&](auto J2) { v[CV(J2)] = Lr[N2 * t + CV(J2)]; });
      dft<N2, +1>(v);
    }
    __syncthreads();  // lds is rewritten below
  }

  if constexpr (MODE == K1_INV) {
    if (ok && t < N1) {
      sfor<0, N2>([&](auto M) { a.fout[ebase + t + N1 * CV(M)] = v[CV(M)]; });
    }
    return;
  }

  double sd = 0.0, se = 0.0;
  if (ok && t < N1) {
    const bool yin = (y >= a.py) && (y < a.ny - a.py);
    const bool zin = (z >= a.pz) && (z < a.nz - a.pz);
    // pol_c exp(i (ky y + kz z)); the x phase joins per element when oblique
    const float2 ph = a.phase[(ib * 3 + c) * a.nz + z];
    const float2 spl = OBL ? cmul(ph, a.phy[ib * a.ny + y]) : ph;
    const float2* phxb = a.phx + ib * a.nx;
    sfor<0, N2>([&](auto M) {
      const int x = t + N1 * CV(M);
      float2 e;
      float2 v0;
      if constexpr (PF) v0 = pv[CV(M)]; else v0 = v0t[N1 * CV(M)];
      if constexpr (MODE == K1_ITER) {
        e = pe[CV(M)];
        // gamma = 1 + i V0 / eps
        const float2 gm = make_float2(1.0f - v0.y * a.inv_eps, v0.x * a.inv_eps);
        const float2 d = cmul(gm, csub(v[CV(M)], e));
        e = cadd(e, d);
        sd += (double)(d.x * d.x + d.y * d.y);
        se += (double)(e.x * e.x + e.y * e.y);
        et[N1 * CV(M)] = e;
      } else if (a.warm) {
        e = et[N1 * CV(M)];
      } else {
        // cold start: E_s^(0) = 0, whatever the output buffer held
        e = make_float2(0.f, 0.f);
        if (!a.green_in) et[N1 * CV(M)] = e;
      }
      float2 w;
      if (MODE == K1_FWD && a.green_in) {
        w = cscale(a.fin[ebase + x], a.src_scale);
      } else {
        // W = (V0 - i eps) e + S
        w = cmul(make_float2(v0.x, v0.y - a.eps), e);
        if (a.src == SRC_PLANE) {
          const bool xin = (x >= a.px) && (x < a.nx - a.px);
          if (xin && yin && zin) {
            if constexpr (OBL)
              w = cadd(w, cmul(v0, cmul(spl, phxb[x])));
            else
              w = cadd(w, cmul(v0, spl));
          }
        } else if (a.src == SRC_FIELD) {
          w = cadd(w, cscale(a.fin[ebase + x], a.src_scale));
        } else if (a.src == SRC_FIELD_CONJ) {
          const float2 f = a.fin[ebase + x];
          w = cadd(w, make_float2(f.x * a.src_scale, -f.y * a.src_scale));
        } else if (a.src == SRC_POINT) {
          if (x == a.r0x && y == a.r0y && z == a.r0z) w = cadd(w, a.st->amp[c]);
        }
      }
      v[CV(M)] = w;
    });
    // forward level A' (split N2 x N1): DFT-N2 over v, twiddle, to Lr[t + N1 k1']
    dft<N2, -1>(v);
    const float2* twc = tw + t;   // exp(-2 pi i t k / N) sits at [k][t] of the table
    sfor<0, N2>([&](auto K) { Lr[t + N1 * CV(K)] = cmul(v[CV(K)], twc[N1 * CV(K)]); });
  }
  __syncthreads();
  // forward level B': thread k1' = t < N2, DFT-N1 over Lr[N1 k1' + j2']
  float2 bo[N1];
  if (ok && t < N2) {
    sfor<0, N1>([&](auto J) { bo[CV(J)] = Lr[N1 * t + CV(J)]; });
    dft<N1, -1>(bo);
    sfor<0, N1>([&](auto K) { wat(t + N2 * CV(K)) = bo[CV(K)]; });
  }
  if constexpr (MODE == K1_ITER) {
    const long long slot = (long long)ib * a.k1_blocks + (long long)rest * 3 + c;
    block_sum2<G::THREADS>(sd, se, red, a.partials + 2 * slot);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.st->pending = 1;
  }
}

// ---------------------------------------------------------------------------
// KY: FFT along y of TX adjacent columns of one (component, z) plane
// ---------------------------------------------------------------------------
template <int N1, int N2, int TX, int S>
__global__ void __launch_bounds__((YGeom<N1, N2, TX>::THREADS))
ky_pass(CbsArgs a) {
  using G = YGeom<N1, N2, TX>;
  constexpr int N = G::N;
  __shared__ float2 lds[N * TX];
  __shared__ float2 tw[N];
  if (a.st->done) return;
  const int tid = threadIdx.x;
  if (a.ky_prio) __builtin_amdgcn_s_setprio(kLoadPrio);
  if (S < 0 && blockIdx.x == 0 && a.st->pending) {
    // finish the previous iteration's residual (stream order: the x pass that
    // wrote the partials has completed); lds is still unused here
    constexpr bool kFits = sizeof(lds) >= 2 * kResStreams * sizeof(double);
    if constexpr (kFits) {
      residual_finish<G::THREADS>(a.partials, a.k1_blocks, a.nb, a.st, a.hist,
                                  reinterpret_cast<double*>(lds));
    } else {
      __shared__ double red[2 * kResStreams];
      residual_finish<G::THREADS>(a.partials, a.k1_blocks, a.nb, a.st, a.hist, red);
    }
    if (tid == 0) a.st->pending = 0;
    __syncthreads();
  }
  TwStage<N, G::THREADS> tws;
  tws.issue(a.twy, tid);
  const int xi = tid % TX;
  const int t = tid / TX;
  const unsigned gx = (unsigned)(a.nx + TX - 1) / TX;
  // component c < 3 nb: the W fields of a batch follow each other (sWb = 3 sW)
  const unsigned L = xcd_remap(blockIdx.x, gx * (unsigned)a.nz * 3u * (unsigned)a.nb);
  const int bx = (int)(L % gx);
  const unsigned rest = L / gx;
  const int z = (int)(rest % (unsigned)a.nz), c = (int)(rest / (unsigned)a.nz);
  static_assert(TX == kBrick, "y-pass tiles are one brick wide");
  const int x = bx * TX + xi;
  const bool xok = x < a.nx;
  // the tile is brick (c, z, bx): ny rows of 8 columns, contiguous
  float2* col = a.W + c * a.sW + ((long long)z * a.gx + bx) * a.ny * kBrick + xi;
  const long long ps = kBrick;
  float2 b[N1];
  auto load_a = [&]() {
    if (t < N2) {
      if (xok) {
        // per-thread base once; each load then adds a uniform stride
        const float2* ct = col + (long long)t * ps;
        const long long st = (long long)N2 * ps;
        sfor<0, N1>([&](auto J1) { b[CV(J1)] = ct[CV(J1) * st]; });
      } else {
        sfor<0, N1>([&](auto J1) { b[CV(J1)] = make_float2(0.f, 0.f); });
      }
    }
  };
  load_a();
  tws.commit(tw, tid);
  __syncthreads();
  if (a.ky_prio) __builtin_amdgcn_s_setprio(0);
  if (t < N2) {
    dft<N1, S>(b);
    const float2* twt = tw + t * N1;
    sfor<0, N1>([&](auto K1) {
      const float2 w = twt[CV(K1)];
      b[CV(K1)] = (S < 0) ? cmul(b[CV(K1)], w) : cmulc(b[CV(K1)], w);
    });
    sfor<0, N1>([&](auto K1) { lds[(t + N2 * CV(K1)) * TX + xi] = b[CV(K1)]; });
  }
  __syncthreads();
  if (t < N1 && xok) {
    float2 v[N2];
    sfor<0, N2>([&](auto J2) { v[CV(J2)] = lds[(N2 * t + CV(J2)) * TX + xi]; });
    dft<N2, S>(v);
    float2* ct = col + (long long)t * ps;
    const long long st = (long long)N1 * ps;
    sfor<0, N2>([&](auto K2) { ct[CV(K2) * st] = v[CV(K2)]; });
  }
}

// ---------------------------------------------------------------------------
// KZ: FFT along z, Green's tensor, inverse FFT along z (3 components)
// ---------------------------------------------------------------------------
template <int N1, int N2, int TX>
__global__ void __launch_bounds__((ZGeom<N1, N2, TX>::THREADS))
kz_pass(CbsArgs a) {
  using G = ZGeom<N1, N2, TX>;
  constexpr int N = G::N;
  __shared__ float2 lds[3 * N * TX];
  __shared__ float2 tw[N];
  if (a.st->done) return;
  const int tid = threadIdx.x;
  TwStage<N, G::THREADS> tws;
  tws.issue(a.twz, tid);
  const int xi = tid % TX;
  const int t = tid / TX;
  // remapped order: the kBrick / TX parts of one brick row, then y, then the
  // brick; rows y, y+1 of a brick share a 128-byte line
  static_assert(kBrick % TX == 0, "z-pass tiles split a brick row evenly");
  constexpr int PARTS = kBrick / TX;
  const unsigned per_b = (unsigned)(a.nxp / TX) * (unsigned)a.ny;
  const unsigned Lb = xcd_remap(blockIdx.x, per_b * (unsigned)a.nb);
  const int ib = (int)(Lb / per_b);
  const unsigned L = Lb - (unsigned)ib * per_b;
  const int part = (int)(L % PARTS);
  const int y = (int)((L / PARTS) % (unsigned)a.ny);
  const int brick = (int)(L / (PARTS * (unsigned)a.ny));
  const int bx = brick * PARTS + part;      // tile index along x
  const int x = bx * TX + xi;
  const bool xok = x < a.nx;
  const long long plane = (long long)a.ny * a.nxp;   // z stride (gx bricks of ny x 8)
  float2* colbase = a.W + ib * a.sWb + ((long long)brick * a.ny + y) * kBrick + part * TX + xi;

  const long long zst = (long long)N2 * plane;  // z stride between the samples of one DFT-N1
  // forward level A: thread (c, j2), DFT-N1 over z = j2 + N2 j1
  const int ca = t / N2;
  const int j2 = t - ca * N2;
  float2 b[N1];
  auto load_a = [&]() {
    if (t < 3 * N2) {
      const float2* col = colbase + ca * a.sW + (long long)j2 * plane;
      if (xok) {
        sfor<0, N1>([&](auto J1) { b[CV(J1)] = col[CV(J1) * zst]; });
      } else {
        sfor<0, N1>([&](auto J1) { b[CV(J1)] = make_float2(0.f, 0.f); });
      }
    }
  };
  load_a();
  tws.commit(tw, tid);
  __syncthreads();
  if (t < 3 * N2) {
    dft<N1, -1>(b);
    const float2* twt = tw + j2 * N1;
    sfor<0, N1>([&](auto K1) { b[CV(K1)] = cmul(b[CV(K1)], twt[CV(K1)]); });
    float2* Lc = lds + ca * N * TX;
    sfor<0, N1>([&](auto K1) { Lc[(j2 + N2 * CV(K1)) * TX + xi] = b[CV(K1)]; });
  }
  __syncthreads();

  // Green's tensor of the column's modes: the x/y parts are fixed per thread
  float2* L0 = lds;
  float2* L1 = lds + N * TX;
  float2* L2 = lds + 2 * N * TX;
  bool nyx, nyy;
  const float px = freq_of(x, a.nx, a.pfx, nyx);
  const float py = freq_of(y, a.ny, a.pfy, nyy);
  const float ptx = nyx ? 0.f : px, pty = nyy ? 0.f : py;
  const float pxy2 = px * px + py * py;
  const float nq_xy = (nyx ? px * px : 0.f) + (nyy ? py * py : 0.f);
  const float eps = a.eps, e2 = eps * eps;
  const bool nq_any = nyx || nyy;
  const float sb = __builtin_amdgcn_rcpf(a.kb2 * a.kb2 + e2);
  const float2 gb0 = make_float2(-a.kb2 * sb, eps * sb);
  // v <- G^(p) v / N at z-frequency index kz
  auto green = [&](float2& u0, float2& u1, float2& u2, int kz) {
    bool nyz;
    const float pz = freq_of(kz, a.nz, a.pfz, nyz);
    const float ptz = nyz ? 0.f : pz;
    const float p2 = pxy2 + pz * pz;
    // a = invN / (p2 - kb2 - i eps), b = 1 / (p2 - |pt|^2 - kb2 - i eps)
    const float r1 = p2 - a.kb2;
    const float s1 = a.invN * __builtin_amdgcn_rcpf(r1 * r1 + e2);
    const float2 ga = make_float2(r1 * s1, eps * s1);
    float2 gb = gb0;   // 1 / (-kb2 - i eps): every mode without a Nyquist component
    if (nq_any || nyz) {
      const float r2 = (nq_xy + (nyz ? pz * pz : 0.f)) - a.kb2;
      const float s2 = __builtin_amdgcn_rcpf(r2 * r2 + e2);
      gb = make_float2(r2 * s2, eps * s2);
    }
    const float2 sp = make_float2(ptx * u0.x + pty * u1.x + ptz * u2.x,
                                  ptx * u0.y + pty * u1.y + ptz * u2.y);
    const float2 bs = cmul(gb, sp);
    u0 = cmul(ga, make_float2(u0.x + ptx * bs.x, u0.y + ptx * bs.y));
    u1 = cmul(ga, make_float2(u1.x + pty * bs.x, u1.y + pty * bs.y));
    u2 = cmul(ga, make_float2(u2.x + ptz * bs.x, u2.y + ptz * bs.y));
  };

  if constexpr (N1 > N2) {
    // level B: thread k1 = t, all three components, Green multiply, inverse B
    if (t < N1) {
      float2 v0[N2], v1[N2], v2[N2];
      sfor<0, N2>([&](auto J) {
        const int o = (N2 * t + CV(J)) * TX + xi;
        v0[CV(J)] = L0[o];
        v1[CV(J)] = L1[o];
        v2[CV(J)] = L2[o];
      });
      dft<N2, -1>(v0);
      dft<N2, -1>(v1);
      dft<N2, -1>(v2);
      sfor<0, N2>([&](auto K2) {
        constexpr int k2 = CV(K2);
        green(v0[k2], v1[k2], v2[k2], t + N1 * k2);
      });
      dft<N2, +1>(v0);
      dft<N2, +1>(v1);
      dft<N2, +1>(v2);
      sfor<0, N2>([&](auto J) {
        const int o = (N2 * t + CV(J)) * TX + xi;
        L0[o] = v0[CV(J)];
        L1[o] = v1[CV(J)];
        L2[o] = v2[CV(J)];
      });
    }
  } else {
    // N1 <= N2: one thread per k1 would leave most lanes idle and hold 3 N2
    // values.  Split level B over the 3 N1 threads (component, k1): forward
    // DFT-N2 per component, the Green multiply spread over the same threads by
    // frequency, inverse DFT-N2 per component, with the spectra in LDS between.
    const int cb = t / N1, kb = t - cb * N1;
    float2* Lb = lds + (cb < 3 ? cb : 0) * N * TX;
    auto level_b = [&](auto sign) {
      if (t < 3 * N1) {
        float2 v[N2];
        sfor<0, N2>([&](auto J) { v[CV(J)] = Lb[(N2 * kb + CV(J)) * TX + xi]; });
        dft<N2, decltype(sign)::value>(v);
        sfor<0, N2>([&](auto J) { Lb[(N2 * kb + CV(J)) * TX + xi] = v[CV(J)]; });
      }
    };
    level_b(std::integral_constant<int, -1>{});
    __syncthreads();
    if (t < 3 * N1) {
      // thread (part, k1) handles k2 = part, part + 3, ...
      for (int k2 = cb; k2 < N2; k2 += 3) {
        const int o = (N2 * kb + k2) * TX + xi;
        float2 u0 = L0[o], u1 = L1[o], u2 = L2[o];
        green(u0, u1, u2, kb + N1 * k2);
        L0[o] = u0;
        L1[o] = u1;
        L2[o] = u2;
      }
    }
    __syncthreads();
    level_b(std::integral_constant<int, +1>{});
  }
  __syncthreads();

  // inverse level A: conj twiddle, inverse DFT-N1, store z = j2 + N2 j1
  if (t < 3 * N2 && xok) {
    float2* Lc = lds + ca * N * TX;
    float2 b[N1];
    sfor<0, N1>([&](auto K1) { b[CV(K1)] = Lc[(j2 + N2 * CV(K1)) * TX + xi]; });
    const float2* twt = tw + j2 * N1;
    sfor<0, N1>([&](auto K1) { b[CV(K1)] = cmulc(b[CV(K1)], twt[CV(K1)]); });
    dft<N1, +1>(b);
    float2* col = colbase + ca * a.sW + (long long)j2 * plane;
    sfor<0, N1>([&](auto J1) { col[CV(J1) * zst] = b[CV(J1)]; });
  }
}

// ---------------------------------------------------------------------------
// launchers and the per-size registry
// ---------------------------------------------------------------------------
using LaunchK1 = void (*)(const CbsArgs&, int mode, hipStream_t);
using LaunchKY = void (*)(const CbsArgs&, int sign, hipStream_t);
using LaunchKZ = void (*)(const CbsArgs&, hipStream_t);

struct SizeOps {
  int n;
  LaunchK1 k1;        // x axis
  LaunchKY ky;        // y axis
  LaunchKZ kz;        // z axis (nullptr: unsupported on z)
  int n1, n2;         // split of the x/y passes (twiddle table layout)
  int z1, z2;         // split of the z pass
  int k1_rows;        // rows per x-pass workgroup when this length is the x axis
};

constexpr int kTY = kBrick;   // columns per y-pass block

// Whether the iteration kernel holds at most two waves per SIMD (occupancy
// API, once per size): then its work-groups raise their priority for the load
// phase (measured at 621 = 27 x 23, two waves: x-pass 2.36 -> 2.30 ms; at
// 275 = 25 x 11, three waves: 0.58 -> 0.60 ms, so not there).
template <int N1, int N2>
int k1_low_occupancy() {
  static int v = -1;
  if (v < 0) {
    using G = XGeom<N1, N2>;
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k1_xpass<N1, N2, K1_ITER, false>, G::THREADS,
                                                     0) != hipSuccess || b <= 0)
      v = 0;
    else
      v = b * (G::THREADS / 64) <= 2 * 4 ? 1 : 0;   // 4 SIMDs per CU
  }
  return v;
}

template <int N1, int N2>
void launch_k1(const CbsArgs& a_in, int mode, hipStream_t s) {
  using G = XGeom<N1, N2>;
  CbsArgs a = a_in;
  a.k1_prio = k1_low_occupancy<N1, N2>();
  const unsigned nb = 3u * (unsigned)a.nb * (unsigned)a.gy * (unsigned)a.nz;
  const bool obl = a.oblique && a.src == SRC_PLANE;
  if (mode == K1_FWD && !obl)
    hipLaunchKernelGGL((k1_xpass<N1, N2, K1_FWD, false>), dim3(nb), dim3(G::THREADS), 0, s, a);
  else if (mode == K1_FWD)
    hipLaunchKernelGGL((k1_xpass<N1, N2, K1_FWD, true>), dim3(nb), dim3(G::THREADS), 0, s, a);
  else if (mode == K1_ITER && !obl)
    hipLaunchKernelGGL((k1_xpass<N1, N2, K1_ITER, false>), dim3(nb), dim3(G::THREADS), 0, s, a);
  else if (mode == K1_ITER)
    hipLaunchKernelGGL((k1_xpass<N1, N2, K1_ITER, true>), dim3(nb), dim3(G::THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((k1_xpass<N1, N2, K1_INV, false>), dim3(nb), dim3(G::THREADS), 0, s, a);
}

template <int N1, int N2>
int ky_low_occupancy() {
  static int v = -1;
  if (v < 0) {
    using G = YGeom<N1, N2, kTY>;
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, ky_pass<N1, N2, kTY, -1>, G::THREADS,
                                                     0) != hipSuccess || b <= 0)
      v = 0;
    else
      v = b * (G::THREADS / 64) <= 3 * 4 ? 1 : 0;
  }
  return v;
}

template <int N1, int N2>
void launch_ky(const CbsArgs& a_in, int sign, hipStream_t s) {
  using G = YGeom<N1, N2, kTY>;
  CbsArgs a = a_in;
  a.ky_prio = ky_low_occupancy<N1, N2>();
  dim3 grid((unsigned)((long long)((a.nx + kTY - 1) / kTY) * a.nz * 3 * a.nb));
  if (sign < 0)
    hipLaunchKernelGGL((ky_pass<N1, N2, kTY, -1>), grid, dim3(G::THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((ky_pass<N1, N2, kTY, +1>), grid, dim3(G::THREADS), 0, s, a);
}

template <int N1, int N2>
void launch_kz(const CbsArgs& a, hipStream_t s) {
  constexpr int TX = kz_tx_for(N1, N2);
  using G = ZGeom<N1, N2, TX>;
  dim3 grid((unsigned)((long long)(a.nxp / TX) * a.ny * a.nb));
  hipLaunchKernelGGL((kz_pass<N1, N2, TX>), grid, dim3(G::THREADS), 0, s, a);
}

#define CBS_SIZE_XYZ(n, a1, a2, z1, z2)                                                  \
  SizeOps {                                                                              \
    n, &launch_k1<a1, a2>, &launch_ky<a1, a2>, &launch_kz<z1, z2>, a1, a2, z1, z2,       \
        XGeom<a1, a2>::LINES                                                             \
  }
#define CBS_SIZE_XY(n, a1, a2) \
  SizeOps { n, &launch_k1<a1, a2>, &launch_ky<a1, a2>, nullptr, a1, a2, 0, 0, XGeom<a1, a2>::LINES }

// registry, defined in the size translation units
const SizeOps* find_size(int n);

}  // namespace cbs
