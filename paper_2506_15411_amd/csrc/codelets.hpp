// Register-resident DFT codelets for gfx950 (one thread, fully unrolled).
//
// dft<N, S>(a) replaces a[0..N) by  X[k] = sum_j a[j] exp(S * 2 pi i j k / N),
// S = -1 (forward) or +1 (inverse, unnormalised).  Composite N is split
// Cooley-Tukey style into register sub-transforms; odd primes use the
// conjugate-pair form  X[k] = a0 + sum_j (a_j + a_{N-j}) cos + i S sum_j
// (a_j - a_{N-j}) sin, which halves the multiplies of a direct DFT.  Every
// twiddle inside a codelet is a compile-time constant (cos/sin evaluated in
// double by a constexpr series on an exactly reduced angle, then rounded to
// float), and multiplications by 1, -1, +-i and the 45-degree roots are
// resolved at compile time.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#define CBS_HD __host__ __device__ __forceinline__

namespace cbs {

// ---------------------------------------------------------------------------
// compile-time helpers
// ---------------------------------------------------------------------------
template <int B, int E, class F>
CBS_HD void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}
#define CV(x) decltype(x)::value

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ct_sin_small(double x) {  // |x| <= pi/4, Taylor to 1e-18
  double x2 = x * x, term = x, sum = x;
  for (int n = 1; n <= 11; ++n) {
    term *= -x2 / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos_small(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n <= 11; ++n) {
    term *= -x2 / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}

struct CS {
  double c, s;
};

// cos and sin of 2 pi k / n for integers k, n > 0 (k reduced mod n exactly).
constexpr CS ct_cis(long long k, long long n) {
  k %= n;
  if (k < 0) k += n;
  const long long q = (4 * k) / n;        // quadrant
  const long long rem = 4 * k - q * n;    // angle in quadrant = (pi/2) rem / n
  double cr = 0, sr = 0;
  if (2 * rem <= n) {
    const double t = (kPi / 2) * double(rem) / double(n);
    cr = ct_cos_small(t);
    sr = ct_sin_small(t);
  } else {
    const double t = (kPi / 2) * double(n - rem) / double(n);
    cr = ct_sin_small(t);
    sr = ct_cos_small(t);
  }
  switch (q) {
    case 0: return CS{cr, sr};
    case 1: return CS{-sr, cr};
    case 2: return CS{-cr, -sr};
    default: return CS{sr, -cr};
  }
}

constexpr bool ct_is_prime(int n) {
  if (n < 2) return false;
  for (int d = 2; d * d <= n; ++d)
    if (n % d == 0) return false;
  return true;
}
constexpr int ct_first_radix(int n) {
  if (n % 4 == 0 && n > 4) return 4;
  for (int d = 2; d <= n; ++d)
    if (n % d == 0) return d;
  return n;
}

// ---------------------------------------------------------------------------
// complex helpers (float2 = re, im)
// ---------------------------------------------------------------------------
CBS_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
CBS_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
CBS_HD float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
CBS_HD float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
CBS_HD float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// v * exp(2 pi i K / N), K a compile-time integer (any sign).
template <int N, long long K>
CBS_HD float2 rot(float2 v) {
  constexpr long long k = ((K % N) + N) % N;
  if constexpr (k == 0) {
    return v;
  } else if constexpr (4 * k == N) {
    return make_float2(-v.y, v.x);
  } else if constexpr (2 * k == N) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (4 * k == 3 * N) {
    return make_float2(v.y, -v.x);
  } else if constexpr (8 * k == N) {
    constexpr float h = 0.70710678118654752440f;
    return make_float2((v.x - v.y) * h, (v.x + v.y) * h);
  } else if constexpr (8 * k == 3 * N) {
    constexpr float h = 0.70710678118654752440f;
    return make_float2((-v.x - v.y) * h, (v.x - v.y) * h);
  } else if constexpr (8 * k == 5 * N) {
    constexpr float h = 0.70710678118654752440f;
    return make_float2((v.y - v.x) * h, (-v.x - v.y) * h);
  } else if constexpr (8 * k == 7 * N) {
    constexpr float h = 0.70710678118654752440f;
    return make_float2((v.x + v.y) * h, (v.y - v.x) * h);
  } else {
    constexpr CS w = ct_cis(k, N);
    constexpr float c = float(w.c), s = float(w.s);
    return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// ---------------------------------------------------------------------------
// codelets
// ---------------------------------------------------------------------------
template <int S>
CBS_HD void dft3(float2& a0, float2& a1, float2& a2) {
  constexpr float h = 0.86602540378443864676f;  // sin(2 pi / 3)
  const float2 t1 = cadd(a1, a2);
  const float2 t2 = make_float2(a0.x - 0.5f * t1.x, a0.y - 0.5f * t1.y);
  const float2 d = csub(a1, a2);
  // i S h d
  const float2 r = make_float2(-float(S) * h * d.y, float(S) * h * d.x);
  a0 = cadd(a0, t1);
  a1 = cadd(t2, r);
  a2 = csub(t2, r);
}

template <int S>
CBS_HD void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const float2 t2 = cadd(a1, a3), d = csub(a1, a3);
  const float2 t3 = make_float2(-float(S) * d.y, float(S) * d.x);  // (S i) d
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <int P, int S>
CBS_HD void dft_prime(float2 (&a)[P]) {
  constexpr int H = (P - 1) / 2;
  float2 sm[H], df[H];
  sfor<1, H + 1>([&](auto J) {
    constexpr int j = CV(J);
    sm[j - 1] = cadd(a[j], a[P - j]);
    df[j - 1] = csub(a[j], a[P - j]);
  });
  const float2 x0 = a[0];
  float2 tot = x0;
  sfor<0, H>([&](auto J) { tot = cadd(tot, sm[CV(J)]); });
  sfor<1, H + 1>([&](auto K) {
    constexpr int k = CV(K);
    float2 A = x0, B = make_float2(0.f, 0.f);
    sfor<1, H + 1>([&](auto J) {
      constexpr int j = CV(J);
      constexpr CS w = ct_cis((long long)j * k, P);
      constexpr float c = float(w.c), s = float(w.s);
      A.x += sm[j - 1].x * c;
      A.y += sm[j - 1].y * c;
      B.x += df[j - 1].x * s;
      B.y += df[j - 1].y * s;
    });
    // X_k = A + i S B, X_{P-k} = A - i S B
    a[k] = make_float2(A.x - float(S) * B.y, A.y + float(S) * B.x);
    a[P - k] = make_float2(A.x + float(S) * B.y, A.y - float(S) * B.x);
  });
  a[0] = tot;
}

constexpr long long ct_powmod(long long b, long long e, long long m) {
  long long r = 1;
  b %= m;
  while (e > 0) {
    if (e & 1) r = r * b % m;
    b = b * b % m;
    e >>= 1;
  }
  return r;
}
// smallest primitive root of the prime p: g^((p-1)/q) != 1 for every prime q | p-1
constexpr int ct_primitive_root(int p) {
  for (int g = 2; g < p; ++g) {
    bool ok = true;
    for (int q = 2; q < p; ++q)
      if ((p - 1) % q == 0 && ct_is_prime(q) && ct_powmod(g, (p - 1) / q, p) == 1) ok = false;
    if (ok) return g;
  }
  return 1;
}

// Odd prime P with H = (P-1)/2 = 2M, M >= 4: the conjugate-pair form with its
// two H x H products taken in Rader order.  With g a primitive root, e_r =
// g^r mod P and f_q = g^-q mod P (r, q < H), and u_r = a[e_r] + a[P-e_r],
// v_r = a[e_r] - a[P-e_r]:
//   X[f_q]     = a0 + sum_r c_{r-q} u_r + i S sum_r s_{r-q} v_r,
//   X[P - f_q] = a0 + sum_r c_{r-q} u_r - i S sum_r s_{r-q} v_r,
// c_m = cos(2 pi g^m / P), s_m = sin(2 pi g^m / P); since g^H = -1, c has
// period H and s changes sign after H.  Split r = r0 + M r1, q = q0 + M q1:
// the cosine matrix is [[A, B], [B, A]], so it acts on u0 +- u1 through
// (A +- B)/2 (two M x M products instead of four); the sine matrix is
// [[A', B'], [-B', A']], taken as A'(v0 + v1) + (B' - A') v1 and
// A'(v0 + v1) - (A' + B') v0 (three instead of four).
template <int P, int S>
CBS_HD void dft_prime_split(float2 (&a)[P]) {
  constexpr int H = (P - 1) / 2;
  constexpr int M = H / 2;
  constexpr long long g = ct_primitive_root(P);
  constexpr long long ginv = ct_powmod(g, P - 2, P);
  float2 pu[M], mu[M], v0[M], v1[M], vs[M];
  sfor<0, M>([&](auto R0) {
    constexpr int r0 = CV(R0);
    constexpr int e0 = (int)ct_powmod(g, r0, P), e1 = (int)ct_powmod(g, r0 + M, P);
    const float2 u0 = cadd(a[e0], a[P - e0]), u1 = cadd(a[e1], a[P - e1]);
    v0[r0] = csub(a[e0], a[P - e0]);
    v1[r0] = csub(a[e1], a[P - e1]);
    pu[r0] = cadd(u0, u1);
    mu[r0] = csub(u0, u1);
    vs[r0] = cadd(v0[r0], v1[r0]);
  });
  const float2 x0 = a[0];
  float2 tot = x0;
  sfor<0, M>([&](auto R0) { tot = cadd(tot, pu[CV(R0)]); });
  sfor<0, M>([&](auto Q0) {
    constexpr int q0 = CV(Q0);
    float2 cp = x0, cm = make_float2(0.f, 0.f);
    float2 k1 = make_float2(0.f, 0.f), k2 = k1, k3 = k1;
    sfor<0, M>([&](auto R0) {
      constexpr int r0 = CV(R0);
      constexpr int d = ((r0 - q0) % (2 * H) + 2 * H) % (2 * H);
      constexpr CS w0 = ct_cis(ct_powmod(g, d, P), P);
      constexpr CS w1 = ct_cis(ct_powmod(g, d + M, P), P);
      constexpr float kp = float(0.5 * (w0.c + w1.c)), km = float(0.5 * (w0.c - w1.c));
      constexpr float al = float(w0.s), bm = float(w1.s - w0.s), ap = float(w0.s + w1.s);
      cp.x += kp * pu[r0].x;
      cp.y += kp * pu[r0].y;
      cm.x += km * mu[r0].x;
      cm.y += km * mu[r0].y;
      k1.x += al * vs[r0].x;
      k1.y += al * vs[r0].y;
      k2.x += bm * v1[r0].x;
      k2.y += bm * v1[r0].y;
      k3.x += ap * v0[r0].x;
      k3.y += ap * v0[r0].y;
    });
    const float2 At = cadd(cp, cm), Ab = csub(cp, cm);   // q = q0 and q = q0 + M
    const float2 Bt = cadd(k1, k2), Bb = csub(k1, k3);
    constexpr int ft = (int)ct_powmod(ginv, q0, P), fb = (int)ct_powmod(ginv, q0 + M, P);
    a[ft] = make_float2(At.x - float(S) * Bt.y, At.y + float(S) * Bt.x);
    a[P - ft] = make_float2(At.x + float(S) * Bt.y, At.y - float(S) * Bt.x);
    a[fb] = make_float2(Ab.x - float(S) * Bb.y, Ab.y + float(S) * Bb.x);
    a[P - fb] = make_float2(Ab.x + float(S) * Bb.y, Ab.y - float(S) * Bb.x);
  });
  a[0] = tot;
}

template <int N, int S>
CBS_HD void dft(float2 (&a)[N]) {
  static_assert(S == 1 || S == -1, "sign");
  if constexpr (N == 1) {
  } else if constexpr (N == 2) {
    const float2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  } else if constexpr (N == 3) {
    dft3<S>(a[0], a[1], a[2]);
  } else if constexpr (N == 4) {
    dft4<S>(a[0], a[1], a[2], a[3]);
  } else if constexpr (ct_is_prime(N) && (N - 1) % 4 == 0 && N >= 17) {
    dft_prime_split<N, S>(a);
  } else if constexpr (ct_is_prime(N)) {
    dft_prime<N, S>(a);
  } else {
    // N = R * M; input index j = j2 + M j1, output index k = k1 + R k2.
    constexpr int R = ct_first_radix(N);
    constexpr int M = N / R;
    float2 y[N];  // y[k1 * M + j2]
    sfor<0, M>([&](auto J2) {
      constexpr int j2 = CV(J2);
      float2 b[R];
      sfor<0, R>([&](auto J1) { b[CV(J1)] = a[j2 + M * CV(J1)]; });
      dft<R, S>(b);
      sfor<0, R>([&](auto K1) {
        constexpr int k1 = CV(K1);
        y[k1 * M + j2] = rot<N, (long long)S * j2 * k1>(b[k1]);
      });
    });
    sfor<0, R>([&](auto K1) {
      constexpr int k1 = CV(K1);
      float2 c[M];
      sfor<0, M>([&](auto J2) { c[CV(J2)] = y[k1 * M + CV(J2)]; });
      dft<M, S>(c);
      sfor<0, M>([&](auto K2) { a[k1 + R * CV(K2)] = c[CV(K2)]; });
    });
  }
}

}  // namespace cbs
