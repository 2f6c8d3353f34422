// fft_core.hpp - in-LDS mixed-radix Stockham FFT for gfx950 (wave64).
//
// A batch of NL lines of length N lives in LDS; element e of line l sits
// at s[l * ls + e * es].  Each stage of radix R with P = product of the
// radices already applied does, for every butterfly index i in [0, N/R):
//   read  x[i + t N/R]           (t = 0..R-1)
//   scale x_t by w^(t k),  k = i mod P,  w = exp(sign 2 pi i / (P R))
//   R-point DFT
//   write y[(i / P) P R + k + t P]
// which leaves the transform in natural order after the last stage (the
// self-sorting Stockham formulation).  The stage is done in place: every
// thread first loads all of its butterflies into registers, the workgroup
// synchronizes, then every thread writes; so one LDS buffer suffices.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

namespace lace {

template <typename T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };
template <typename T> using C = typename cplx<T>::type;

template <typename T> __host__ __device__ inline C<T> mk(T x, T y) {
  C<T> r; r.x = x; r.y = y; return r;
}
template <typename T> __device__ inline C<T> add(C<T> a, C<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ inline C<T> sub(C<T> a, C<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ inline C<T> mul(C<T> a, C<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T> __device__ inline C<T> cmul(C<T> a, C<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// a * conj(b)
template <typename T> __device__ inline C<T> mulc(C<T> a, C<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T> __device__ inline C<T> scl(C<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by sign * i  (sign = +1 or -1)
template <int SIGN, typename T> __device__ inline C<T> muli(C<T> a) {
  return SIGN > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// R-point DFTs, X_k = sum_t x_t exp(SIGN 2 pi i t k / R).  SIGN = -1 is the
// forward transform.  Constants are closed forms: cos(2pi/3) = -1/2,
// sin(2pi/3) = sqrt(3)/2, cos(2pi/5) = (sqrt5 - 1)/4, cos(4pi/5) =
// -(sqrt5 + 1)/4, sin(2pi/5) = sqrt((5 + sqrt5)/8), sin(4pi/5) =
// sqrt((5 - sqrt5)/8), cos(pi/4) = sqrt(2)/2.
// ---------------------------------------------------------------------------
template <int R, int SIGN, typename T> struct Dft;

template <int SIGN, typename T> struct Dft<2, SIGN, T> {
  __device__ static inline void run(C<T>* v) {
    C<T> a = v[0], b = v[1];
    v[0] = add<T>(a, b);
    v[1] = sub<T>(a, b);
  }
};

template <int SIGN, typename T> struct Dft<3, SIGN, T> {
  __device__ static inline void run(C<T>* v) {
    const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
    C<T> a = v[0], t1 = add<T>(v[1], v[2]), t2 = sub<T>(v[1], v[2]);
    C<T> m = mk<T>(a.x - T(0.5) * t1.x, a.y - T(0.5) * t1.y);
    C<T> r = muli<SIGN, T>(scl<T>(t2, h));
    v[0] = add<T>(a, t1);
    v[1] = add<T>(m, r);
    v[2] = sub<T>(m, r);
  }
};

template <int SIGN, typename T> struct Dft<4, SIGN, T> {
  __device__ static inline void run(C<T>* v) {
    C<T> s02 = add<T>(v[0], v[2]), d02 = sub<T>(v[0], v[2]);
    C<T> s13 = add<T>(v[1], v[3]), d13 = muli<SIGN, T>(sub<T>(v[1], v[3]));
    v[0] = add<T>(s02, s13);
    v[2] = sub<T>(s02, s13);
    v[1] = add<T>(d02, d13);
    v[3] = sub<T>(d02, d13);
  }
};

template <int SIGN, typename T> struct Dft<5, SIGN, T> {
  __device__ static inline void run(C<T>* v) {
    const T c1 = T(0.30901699437494742410229341718282);   // cos(2pi/5)
    const T c2 = T(-0.80901699437494742410229341718282);  // cos(4pi/5)
    const T s1 = T(0.95105651629515357211643933337938);   // sin(2pi/5)
    const T s2 = T(0.58778525229247312916870595463907);   // sin(4pi/5)
    C<T> a = v[0];
    C<T> t1 = add<T>(v[1], v[4]), t2 = add<T>(v[2], v[3]);
    C<T> t3 = sub<T>(v[1], v[4]), t4 = sub<T>(v[2], v[3]);
    C<T> m1 = mk<T>(a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y);
    C<T> m2 = mk<T>(a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y);
    C<T> r1 = muli<SIGN, T>(mk<T>(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
    C<T> r2 = muli<SIGN, T>(mk<T>(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
    v[0] = add<T>(a, add<T>(t1, t2));
    v[1] = add<T>(m1, r1);
    v[4] = sub<T>(m1, r1);
    v[2] = add<T>(m2, r2);
    v[3] = sub<T>(m2, r2);
  }
};

template <int SIGN, typename T> struct Dft<8, SIGN, T> {
  __device__ static inline void run(C<T>* v) {
    const T q = T(0.70710678118654752440084436210485);  // sqrt(2)/2
    C<T> e[4] = {v[0], v[2], v[4], v[6]};
    C<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, SIGN, T>::run(e);
    Dft<4, SIGN, T>::run(o);
    // o_k *= exp(SIGN 2 pi i k / 8)
    C<T> o1 = o[1];
    o[1] = mk<T>(q * (o1.x - SIGN * o1.y), q * (o1.y + SIGN * o1.x));
    o[2] = muli<SIGN, T>(o[2]);
    C<T> o3 = o[3];
    o[3] = mk<T>(q * (-o3.x - SIGN * o3.y), q * (-o3.y + SIGN * o3.x));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = add<T>(e[k], o[k]);
      v[k + 4] = sub<T>(e[k], o[k]);
    }
  }
};

// Prime-factor (Good-Thomas) DFT of length R = A B with gcd(A, B) = 1.
// Input n = (B a + A b) mod R and output k with k = ka (mod A), k = kb
// (mod B) turn the length-R DFT into B-point DFTs over b followed by A-point
// DFTs over a, with no twiddle factors between them.
constexpr int inv_mod(int x, int m) {
  for (int y = 1; y < m; ++y)
    if ((x * y) % m == 1) return y;
  return 1;
}
template <int A, int B, int SIGN, typename T> struct Pfa {
  static constexpr int R = A * B;
  static constexpr int EA = B * inv_mod(B % A, A);  // 1 mod A, 0 mod B
  static constexpr int EB = A * inv_mod(A % B, B);  // 0 mod A, 1 mod B
  __device__ static inline void run(C<T>* v) {
    C<T> u[A][B];
#pragma unroll
    for (int a = 0; a < A; ++a) {
#pragma unroll
      for (int b = 0; b < B; ++b) u[a][b] = v[(B * a + A * b) % R];
      Dft<B, SIGN, T>::run(u[a]);
    }
#pragma unroll
    for (int kb = 0; kb < B; ++kb) {
      C<T> col[A];
#pragma unroll
      for (int a = 0; a < A; ++a) col[a] = u[a][kb];
      Dft<A, SIGN, T>::run(col);
#pragma unroll
      for (int ka = 0; ka < A; ++ka) v[(EA * ka + EB * kb) % R] = col[ka];
    }
  }
};
template <int SIGN, typename T> struct Dft<6, SIGN, T> : Pfa<2, 3, SIGN, T> {};
template <int SIGN, typename T> struct Dft<10, SIGN, T> : Pfa<2, 5, SIGN, T> {};
template <int SIGN, typename T> struct Dft<12, SIGN, T> : Pfa<3, 4, SIGN, T> {};
template <int SIGN, typename T> struct Dft<15, SIGN, T> : Pfa<3, 5, SIGN, T> {};

// ---------------------------------------------------------------------------
// Radix plans for the supported lengths (product of the listed radices).
// ---------------------------------------------------------------------------
// Plan<N, 0>: the radices in the listed order; Plan<N, 1>: in reverse
// order (an equally valid factorization; which runs faster is left to the
// autotuner).
template <int N, int RO = 0> struct Plan;
#define LACE_PLAN(NN, NS, ...)                                   \
  template <> struct Plan<NN, 0> {                               \
    static constexpr int nst = NS;                               \
    static constexpr int r[NS] = {__VA_ARGS__};                  \
  };
LACE_PLAN(4, 1, 4)
LACE_PLAN(6, 1, 6)
LACE_PLAN(8, 1, 8)
LACE_PLAN(12, 1, 12)
LACE_PLAN(16, 2, 4, 4)
LACE_PLAN(24, 2, 8, 3)
LACE_PLAN(32, 2, 8, 4)
LACE_PLAN(40, 2, 8, 5)
LACE_PLAN(48, 2, 4, 12)
LACE_PLAN(60, 2, 4, 15)
LACE_PLAN(64, 2, 8, 8)
LACE_PLAN(80, 2, 8, 10)
LACE_PLAN(96, 2, 8, 12)
LACE_PLAN(120, 2, 8, 15)
#undef LACE_PLAN

template <int N, class Seq> struct RevPlan;
template <int N, int... I> struct RevPlan<N, std::integer_sequence<int, I...>> {
  static constexpr int nst = sizeof...(I);
  static constexpr int r[nst] = {Plan<N, 0>::r[nst - 1 - I]...};
};
template <int N>
struct Plan<N, 1> : RevPlan<N, std::make_integer_sequence<int, Plan<N, 0>::nst>> {};

template <int N, int S, int RO> struct StageP {  // product of radices before stage S
  static constexpr int value = StageP<N, S - 1, RO>::value * Plan<N, RO>::r[S - 1];
};
template <int N, int RO> struct StageP<N, 0, RO> { static constexpr int value = 1; };

// One Stockham stage.  LINES_FAST: consecutive threads walk consecutive
// lines (use when lines are adjacent in LDS, i.e. ls == 1), else
// consecutive butterflies of one line.  tw[m TWS] = exp(-2 pi i m / N): the
// table may belong to a TWS times longer transform.
template <typename T, int N, int R, int P, int NL, int NT, int SIGN,
          bool LINES_FAST, int TWS>
__device__ inline void lds_stage(C<T>* s, int ls, int es, const C<T>* tw) {
  constexpr int NR = N / R;
  constexpr int B = NL * NR;
  constexpr int NB = (B + NT - 1) / NT;
  const int tid = threadIdx.x;
  C<T> v[NB][R];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int idx = tid + b * NT;
    if ((B % NT == 0) || idx < B) {
      const int l = LINES_FAST ? idx % NL : idx / NR;
      const int i = LINES_FAST ? idx / NL : idx % NR;
      const C<T>* base = s + l * ls;
#pragma unroll
      for (int t = 0; t < R; ++t) v[b][t] = base[(i + t * NR) * es];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int idx = tid + b * NT;
    if ((B % NT == 0) || idx < B) {
      const int l = LINES_FAST ? idx % NL : idx / NR;
      const int i = LINES_FAST ? idx / NL : idx % NR;
      const int k = i % P;
      if (P > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) {
          C<T> w = tw[t * k * (N / (P * R)) * TWS];
          if (SIGN > 0) w.y = -w.y;
          v[b][t] = mul<T>(v[b][t], w);
        }
      }
      Dft<R, SIGN, T>::run(v[b]);
      const int j = (i / P) * P * R + k;
      C<T>* base = s + l * ls;
#pragma unroll
      for (int t = 0; t < R; ++t) base[(j + t * P) * es] = v[b][t];
    }
  }
  __syncthreads();
}

template <int N, int S, int RO> struct NextS {
  static constexpr int value = (S + 1 < Plan<N, RO>::nst) ? S + 1 : -1;
};

template <typename T, int N, int S, int NL, int NT, int SIGN, bool LF,
          int TWS, int RO>
struct StagesFrom {
  __device__ static inline void run(C<T>* s, int ls, int es, const C<T>* tw) {
    lds_stage<T, N, Plan<N, RO>::r[S], StageP<N, S, RO>::value, NL, NT, SIGN,
              LF, TWS>(s, ls, es, tw);
    StagesFrom<T, N, NextS<N, S, RO>::value, NL, NT, SIGN, LF, TWS, RO>::run(
        s, ls, es, tw);
  }
};
template <typename T, int N, int NL, int NT, int SIGN, bool LF, int TWS, int RO>
struct StagesFrom<T, N, -1, NL, NT, SIGN, LF, TWS, RO> {
  __device__ static inline void run(C<T>*, int, int, const C<T>*) {}
};

// Stages S .. E-1 of the plan, in plan order.
template <typename T, int N, int S, int E, int NL, int NT, int SIGN, bool LF,
          int TWS, int RO>
struct StagesRange {
  __device__ static inline void run(C<T>* s, int ls, int es, const C<T>* tw) {
    if constexpr (S < E) {
      lds_stage<T, N, Plan<N, RO>::r[S], StageP<N, S, RO>::value, NL, NT, SIGN,
                LF, TWS>(s, ls, es, tw);
      StagesRange<T, N, S + 1, E, NL, NT, SIGN, LF, TWS, RO>::run(s, ls, es, tw);
    }
  }
};

// The plan in reverse order, from stage index S down to 0: radix r[S] after
// the radices r[S+1..] already applied (P = N / (r[0] ... r[S])).  The
// reversed plan is an equally valid self-sorting Stockham factorization.
template <typename T, int N, int S, int NL, int NT, int SIGN, bool LF, int TWS,
          int RO>
struct StagesReversed {
  __device__ static inline void run(C<T>* s, int ls, int es, const C<T>* tw) {
    if constexpr (S >= 0) {
      lds_stage<T, N, Plan<N, RO>::r[S], N / StageP<N, S + 1, RO>::value, NL, NT,
                SIGN, LF, TWS>(s, ls, es, tw);
      StagesReversed<T, N, S - 1, NL, NT, SIGN, LF, TWS, RO>::run(s, ls, es, tw);
    }
  }
};

// NL length-N transforms in LDS.  Caller must __syncthreads() after filling
// s; the call ends with a barrier.  The twiddle table holds the roots of a
// length N * TWS transform.  RO picks the radix order (Plan<N, RO>).
template <typename T, int N, int NL, int NT, int SIGN, bool LINES_FAST,
          int TWS = 1, int RO = 0>
__device__ inline void lds_fft(C<T>* s, int ls, int es, const C<T>* tw) {
  StagesFrom<T, N, 0, NL, NT, SIGN, LINES_FAST, TWS, RO>::run(s, ls, es, tw);
}

}  // namespace lace
