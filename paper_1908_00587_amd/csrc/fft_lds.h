// LDS-resident mixed-radix FFTs for gfx950 (wave64).
//
// Lines of length n live in LDS, padded (one slot per 128 bytes).  Each stage is a
// Stockham autosort pass (natural-order in, natural-order out): butterfly j
// of a stage with accumulated length ns and radix R reads elements
// j + r n/R, multiplies them by the twiddles w^{r (j mod ns)} with
// w = e^{-+2 pi i / (ns R)}, applies a length-R DFT and writes to
// (j / ns) ns R + (j mod ns) + r ns.  All of a thread's butterflies are held
// in registers between a read phase and a write phase separated by block
// barriers, so a stage works in place.  Radices 2, 3, 4, 5, 8 cover the
// padded lengths 3 M_theta and 3 (K+1) of the 3/2-rule grid.
#pragma once
#include <hip/hip_runtime.h>

#include "nsc_internal.h"

namespace nsc {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {
  T x, y;
};

// Pointer into LDS (address space 3), so that out-of-line stage functions
// still issue ds_read/ds_write rather than flat accesses.
template <typename T>
using LdsC2 = __attribute__((address_space(3))) C2<T> *;
template <typename T>
__device__ __forceinline__ LdsC2<T> to_lds(C2<T> *p) {
  return (LdsC2<T>)p;
}
template <typename T>
__device__ __forceinline__ C2<T> lds_ld(LdsC2<T> p) {
  return C2<T>{p->x, p->y};
}
template <typename T>
__device__ __forceinline__ void lds_st(LdsC2<T> p, C2<T> v) {
  p->x = v.x;
  p->y = v.y;
}

template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by i*s (s = +1 or -1)
template <typename T>
__device__ __forceinline__ C2<T> cmul_is(C2<T> a, T s) { return {-s * a.y, s * a.x}; }

// Twiddle tables.  FP64: the values e^{-2 pi i t/n}.  FP32: compensated
// pairs (hi, lo), hi the FP32 rounding of the value and lo the FP32 rounding
// of the remainder, so that a product with hi + lo carries the twiddle to
// about 2^-48 instead of 2^-24; one 16-byte entry per twiddle either way.
template <typename T>
struct TwOf {
  using type = C2<T>;
};
struct alignas(16) TwF32 {
  float x, y, z, w;  // hi.re, hi.im, lo.re, lo.im
};
template <>
struct TwOf<float> {
  using type = TwF32;
};
template <typename T>
using TwT = typename TwOf<T>::type;
template <typename T>
using LdsTw = __attribute__((address_space(3))) TwT<T> *;
template <typename T>
__device__ __forceinline__ LdsTw<T> to_lds_tw(const TwT<T> *p) {
  return (LdsTw<T>)const_cast<TwT<T> *>(p);
}
// C2<T> slots of LDS taken by n twiddle entries
template <typename T>
__host__ __device__ constexpr int tw_slots(int n) {
  return n * (int)(sizeof(TwT<T>) / sizeof(C2<T>));
}

// v * w, w the table entry (conjugated for the inverse transform).  FP32:
// v * hi + v * lo, the small products first, so the twiddle's own rounding
// error does not enter the result.
template <typename T, bool INV>
__device__ __forceinline__ C2<T> twmul(C2<T> v, LdsTw<T> p) {
  if constexpr (sizeof(T) == 4) {
    const float hx = p->x, hy = INV ? -p->y : p->y, lx = p->z, ly = INV ? -p->w : p->w;
    const float cr = fmaf(v.x, lx, -v.y * ly), ci = fmaf(v.x, ly, v.y * lx);
    return {fmaf(v.x, hx, fmaf(-v.y, hy, cr)), fmaf(v.x, hy, fmaf(v.y, hx, ci))};
  } else {
    C2<T> w{p->x, p->y};
    if (INV) w.y = -w.y;
    return cmul(v, w);
  }
}

// a * s for a constant s of a butterfly: FP32 multiplies by the
// compensated pair (hi, lo) of the FP64 constant, FP64 by the constant.
template <typename T>
__device__ __forceinline__ T kmul(double s, T a) {
  if constexpr (sizeof(T) == 4) {
    const float hi = (float)s, lo = (float)(s - (double)hi);
    return fmaf(hi, a, lo * a);
  } else {
    return (T)s * a;
  }
}

// Length-R DFT in registers, y_k = sum_n x_n e^{sgn 2 pi i n k / R},
// sgn = -1 (forward) or +1 (inverse).
template <typename T, int R, bool INV>
struct Dft;

template <typename T, bool INV>
struct Dft<T, 2, INV> {
  __device__ __forceinline__ static void run(C2<T> *v) {
    C2<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <typename T, bool INV>
struct Dft<T, 3, INV> {
  __device__ __forceinline__ static void run(C2<T> *v) {
    const T s = INV ? T(1) : T(-1);
    constexpr double h = 0.86602540378443864676372317075294;  // sqrt(3)/2
    C2<T> a = v[0], b = v[1], c = v[2];
    C2<T> t1 = cadd(b, c);
    C2<T> t2 = {a.x - T(0.5) * t1.x, a.y - T(0.5) * t1.y};
    const C2<T> bmc = csub(b, c);
    C2<T> t3 = cmul_is(C2<T>{kmul<T>(h, bmc.x), kmul<T>(h, bmc.y)}, s);
    v[0] = cadd(a, t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  }
};

template <typename T, bool INV>
struct Dft<T, 4, INV> {
  __device__ __forceinline__ static void run(C2<T> *v) {
    const T s = INV ? T(1) : T(-1);
    C2<T> a = v[0], b = v[1], c = v[2], d = v[3];
    C2<T> apc = cadd(a, c), amc = csub(a, c);
    C2<T> bpd = cadd(b, d), bmd = cmul_is(csub(b, d), s);
    v[0] = cadd(apc, bpd);
    v[1] = cadd(amc, bmd);
    v[2] = csub(apc, bpd);
    v[3] = csub(amc, bmd);
  }
};

template <typename T, bool INV>
struct Dft<T, 5, INV> {
  __device__ __forceinline__ static void run(C2<T> *v) {
    const T s = INV ? T(1) : T(-1);
    constexpr double c1 = 0.30901699437494742410229341718282;   // cos(2 pi/5)
    constexpr double c2 = -0.80901699437494742410229341718282;  // cos(4 pi/5)
    constexpr double s1 = 0.95105651629515357211643933337938;   // sin(2 pi/5)
    constexpr double s2 = 0.58778525229247312916870595463907;   // sin(4 pi/5)
    C2<T> a = v[0];
    C2<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    C2<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    C2<T> r1 = {a.x + kmul<T>(c1, t1.x) + kmul<T>(c2, t2.x), a.y + kmul<T>(c1, t1.y) + kmul<T>(c2, t2.y)};
    C2<T> r2 = {a.x + kmul<T>(c2, t1.x) + kmul<T>(c1, t2.x), a.y + kmul<T>(c2, t1.y) + kmul<T>(c1, t2.y)};
    C2<T> i1 = cmul_is(C2<T>{kmul<T>(s1, t3.x) + kmul<T>(s2, t4.x), kmul<T>(s1, t3.y) + kmul<T>(s2, t4.y)}, s);
    C2<T> i2 = cmul_is(C2<T>{kmul<T>(s2, t3.x) - kmul<T>(s1, t4.x), kmul<T>(s2, t3.y) - kmul<T>(s1, t4.y)}, s);
    v[0] = cadd(a, cadd(t1, t2));
    v[1] = cadd(r1, i1);
    v[4] = csub(r1, i1);
    v[2] = cadd(r2, i2);
    v[3] = csub(r2, i2);
  }
};

template <typename T, bool INV>
struct Dft<T, 8, INV> {
  __device__ __forceinline__ static void run(C2<T> *v) {
    const T s = INV ? T(1) : T(-1);
    constexpr double q = 0.70710678118654752440084436210485;
    C2<T> e[4] = {v[0], v[2], v[4], v[6]};
    C2<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<T, 4, INV>::run(e);
    Dft<T, 4, INV>::run(o);
    // twiddles w8^k, w8 = e^{s i pi/4}
    C2<T> o1 = {kmul<T>(q, o[1].x - s * o[1].y), kmul<T>(q, o[1].y + s * o[1].x)};
    C2<T> o2 = cmul_is(o[2], s);
    C2<T> o3 = {kmul<T>(q, -o[3].x - s * o[3].y), kmul<T>(q, -o[3].y + s * o[3].x)};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// LDS line layout: one padding slot after every 8 elements of a line, so that
// the strided writes of the early Stockham stages (stride R elements) and the
// transposed tile accesses spread over the LDS banks.
template <typename T>
__host__ __device__ constexpr int pad_shift() { return 3; }  // stage_body's default SH
template <typename T>
__device__ __forceinline__ int PD(int i) { return i + (i >> pad_shift<T>()); }
template <typename T>
__host__ __device__ constexpr int lds_line(int n) { return n + (n >> pad_shift<T>()) + 1; }
// The same with a pad period of 2^SH elements (the long lines of the
// workgroup-scope theta pass use one slot per 32, to fit two line sets)
template <int SH>
__device__ __forceinline__ int PDs(int i) { return i + (i >> SH); }
template <int SH>
__host__ __device__ constexpr int lds_line_s(int n) { return n + (n >> SH) + 1; }


// Logical (x, y, z) block coordinates after the XCD remap.
__device__ __forceinline__ void xcd_block(int &bx, int &by, int &bz) {
  const int gx = gridDim.x, gy = gridDim.y;
  const int G = gx * gy * gridDim.z;
  const int w = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int L = xcd_remap(w, G);
  bx = L % gx;
  by = (L / gx) % gy;
  bz = L / (gx * gy);
}

// As xcd_block, with z varying fastest in the logical order, then y: the
// workgroups of all fields of one (x, y) tile run next to each other on one
// XCD, and consecutive tiles step along y (the radial row) for a fixed x, so
// the 9-row stencil window a tile reads stays small enough for that XCD's
// L2 and most rows come from it instead of HBM.
__device__ __forceinline__ void xcd_block_zfirst(int &bx, int &by, int &bz) {
  const int gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const int G = gx * gy * gz;
  const int w = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int L = xcd_remap(w, G);
  bz = L % gz;
  const int rest = L / gz;
  by = rest % gy;
  bx = rest / gy;
}

// Copy the n twiddle entries of a plan into LDS (caller synchronises).
template <typename E>
__device__ __forceinline__ void load_twiddles(E *dst, const E *__restrict__ src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// Wavefront-level ordering point: the LDS executes one wavefront's
// instructions in program order, so only the compiler has to be kept from
// moving LDS accesses across it or caching values over it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Affine addressing: with the pad period P (elements), the element offsets
// j + r n/R of a butterfly's reads map to PD(j) + r (n/R)(1 + 1/P) when P
// divides n/R, and its writes base + r ns to PD(base) + r ns (1 + 1/P) when
// P divides ns, or to PD(base) + r when ns = 1 and R divides P.  The stage
// then needs one add per access instead of a pad computation.
template <typename T>
__device__ __forceinline__ bool affine_stage(int n, int R, int ns) {
  constexpr int P = 1 << pad_shift<T>();
  const int nb = n / R;
  return nb % P == 0 && (ns % P == 0 || (ns == 1 && P % R == 0));
}

// One Stockham stage over `nlines` lines (stride ls) of length n, executed
// by `nthr` threads (tid = 0..nthr-1) that each hold MW butterflies in
// registers between the read and the write phase.  BLOCK: the threads are
// the workgroup (barriers); otherwise one wavefront (compiler fences only).
// Requires nlines * n / R <= MW * nthr.
template <typename T, int R, bool INV, int MW, bool BLOCK, bool AFF, bool CT = false,
          bool SKIPMID = false, int SH = 3>
__device__ __forceinline__ void stage_body(LdsC2<T> buf, int nlines, int n, int ls, int ns,
                                           LdsTw<T> tw, int tid, int nthr) {
  const int nb = n / R;
  const int total = nlines * nb;
  const int step = n / (ns * R);
  const bool pow2 = (ns & (ns - 1)) == 0;
  const float inb = 1.0f / (float)nb;
  const int nbp = nb + (nb >> SH);                 // padded read stride (AFF)
  const int nsp = ns == 1 ? 1 : ns + (ns >> SH);   // padded write stride (AFF)
  C2<T> v[MW][R];
  int wl[MW], wa[MW];
#pragma unroll
  for (int q = 0; q < MW; ++q) {
    const int b = tid + q * nthr;
    if (b < total) {
      int line, j;
      if (CT) {  // compile-time n: exact division by a constant
        line = b / nb;
        j = b - line * nb;
      } else {
        line = (int)(((float)b + 0.5f) * inb);
        j = b - line * nb;
        if (j < 0) {
          --line;
          j += nb;
        } else if (j >= nb) {
          ++line;
          j -= nb;
        }
      }
      const int k = pow2 ? (j & (ns - 1)) : (j % ns);
      LdsC2<T> L = buf + line * ls;
      if (AFF) {
        LdsC2<T> L0 = L + PDs<SH>(j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = lds_ld(L0 + r * nbp);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = lds_ld(L + PDs<SH>(j + r * nb));
      }
      if (ns > 1) {  // the first stage has unit twiddles
        const int ks = k * step;
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = twmul<T, INV>(v[q][r], tw + r * ks);
      }
      Dft<T, R, INV>::run(v[q]);
      const int base = (j - k) * R + k;  // (j / ns) ns R + j mod ns
      wl[q] = line * ls;
      wa[q] = AFF ? PDs<SH>(base) : base;
    }
  }
  if (BLOCK) __syncthreads();
  else wave_sync();
#pragma unroll
  for (int q = 0; q < MW; ++q) {
    if (tid + q * nthr < total) {
      LdsC2<T> L = buf + wl[q];
      // SKIPMID (last radix-3 stage of a forward theta transform): the middle
      // third of the outputs, the modes the truncation drops, is not stored
      if (AFF) {
        LdsC2<T> W0 = L + wa[q];
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (!(SKIPMID && r == 1)) lds_st(W0 + r * nsp, v[q][r]);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (!(SKIPMID && r == 1)) lds_st(L + PDs<SH>(wa[q] + r * ns), v[q][r]);
      }
    }
  }
  if (BLOCK) __syncthreads();
  else wave_sync();
}

// Block-scope stage: one butterfly per thread (out of line, so that the
// callers' registers stay free).
template <typename T, int R, bool INV, int MAXB>
__device__ __attribute__((noinline)) void fft_stage(LdsC2<T> buf, int nlines, int n, int ls,
                                                    int ns, LdsTw<T> tw) {
  if (affine_stage<T>(n, R, ns))
    stage_body<T, R, INV, MAXB, true, true>(buf, nlines, n, ls, ns, tw, (int)threadIdx.x,
                                            (int)blockDim.x);
  else
    stage_body<T, R, INV, MAXB, true, false>(buf, nlines, n, ls, ns, tw, (int)threadIdx.x,
                                             (int)blockDim.x);
}

// Full transform of `nlines` LDS lines; forward (e^{-}) or inverse (e^{+}),
// unnormalised.  tw: n twiddles e^{-2 pi i t / n} (in LDS).  Lines
// are transformed in groups small enough that every stage's butterflies fit
// MAXB per thread (the host guarantees n / min_radix <= MAXB * blockDim.x).
template <typename T, bool INV, int MAXB>
__device__ void fft_lines(C2<T> *buf, int nlines, int ls, const FftPlan &plan,
                          const TwT<T> *tw) {
  const int n = plan.n;
  int gl = (MAXB * (int)blockDim.x * plan.min_radix) / n;
  if (gl < 1) gl = 1;
  LdsTw<T> twl = to_lds_tw<T>(tw);
  for (int l0 = 0; l0 < nlines; l0 += gl) {
    const int nl = nlines - l0 < gl ? nlines - l0 : gl;
    LdsC2<T> b0 = to_lds(buf + l0 * ls);
    int ns = 1;
    for (int s = 0; s < plan.nst; ++s) {
      const int R = plan.radix[s];
      switch (R) {
        case 2: fft_stage<T, 2, INV, MAXB>(b0, nl, n, ls, ns, twl); break;
        case 3: fft_stage<T, 3, INV, MAXB>(b0, nl, n, ls, ns, twl); break;
        case 4: fft_stage<T, 4, INV, MAXB>(b0, nl, n, ls, ns, twl); break;
        case 5: fft_stage<T, 5, INV, MAXB>(b0, nl, n, ls, ns, twl); break;
        default: fft_stage<T, 8, INV, MAXB>(b0, nl, n, ls, ns, twl); break;
      }
      ns *= R;
    }
  }
}

// ---------------------------------------------------------------------------
// Wavefront-scope transforms.  The lines belong to one wavefront, which alone
// reads and writes them.  The LDS executes the instructions of a wavefront in
// program order, so a stage needs no workgroup barrier: a compiler-level
// barrier keeps the reads of a stage ahead of its writes and stops values
// from being held in registers across stages.
// ---------------------------------------------------------------------------

// One stage over `nlines` lines of one wavefront; every butterfly of the
// lane is held in registers between the read and the write phase
// (host guarantee: nlines * n / R <= 64 * (kWaveRegs / R)).  Out of line:
// inlined into the callers' stage loops, the per-radix index math gets
// hoisted across stages and exhausts the registers.
template <typename T, int R, bool INV>
__device__ __attribute__((noinline)) void wave_stage(LdsC2<T> buf, int nlines, int n, int ls,
                                                     int ns, LdsTw<T> tw, int lane) {
  constexpr int MW = kWaveRegs / R;
  if (affine_stage<T>(n, R, ns))
    stage_body<T, R, INV, MW, false, true>(buf, nlines, n, ls, ns, tw, lane, 64);
  else
    stage_body<T, R, INV, MW, false, false>(buf, nlines, n, ls, ns, tw, lane, 64);
}

// Transform of `nlines` lines owned by one wavefront, in groups of
// plan.wave_lines lines.  Forward (e^{-}) or inverse (e^{+}), unnormalised.
template <typename T, bool INV>
__device__ void fft_wave(C2<T> *buf, int nlines, int ls, const FftPlan &plan, const TwT<T> *tw,
                         int lane) {
  const int n = plan.n;
  const int gl = plan.wave_lines;
  LdsTw<T> twl = to_lds_tw<T>(tw);
  for (int l0 = 0; l0 < nlines; l0 += gl) {
    const int nl = nlines - l0 < gl ? nlines - l0 : gl;
    LdsC2<T> b0 = to_lds(buf + l0 * ls);
    int ns = 1;
    for (int s = 0; s < plan.nst; ++s) {
      const int R = plan.radix[s];
      const int ln = lane;
      switch (R) {
        case 2: wave_stage<T, 2, INV>(b0, nl, n, ls, ns, twl, ln); break;
        case 3: wave_stage<T, 3, INV>(b0, nl, n, ls, ns, twl, ln); break;
        case 4: wave_stage<T, 4, INV>(b0, nl, n, ls, ns, twl, ln); break;
        case 5: wave_stage<T, 5, INV>(b0, nl, n, ls, ns, twl, ln); break;
        default: wave_stage<T, 8, INV>(b0, nl, n, ls, ns, twl, ln); break;
      }
      ns *= R;
    }
  }
}

// ---------------------------------------------------------------------------
// Fixed-length wavefront transforms.  For the transform lengths of the
// configured grids the stage sequence, strides, padded line length and
// affine-address choice are compile-time constants, so the index arithmetic
// of the butterflies folds into immediates (instruction offsets, constant
// divisors).  Same stages, same order and same arithmetic as fft_wave.
// ---------------------------------------------------------------------------
struct CtRadices {
  int nst;
  int r[kMaxStages];
};

// The planner's radix order (8s, a 4 when the power of two needs it, a 2,
// then 3s, then 5s) as a compile-time function of n.
constexpr CtRadices ct_radices(int n) {
  CtRadices p{0, {}};
  int rem = n, a = 0, n3 = 0, n5 = 0;
  while (rem % 5 == 0) { rem /= 5; ++n5; }
  while (rem % 3 == 0) { rem /= 3; ++n3; }
  while (rem % 2 == 0) { rem /= 2; ++a; }
  while (a >= 3 && a != 4) { p.r[p.nst++] = 8; a -= 3; }
  while (a >= 2) { p.r[p.nst++] = 4; a -= 2; }
  if (a == 1) p.r[p.nst++] = 2;
  for (int i = 0; i < n3; ++i) p.r[p.nst++] = 3;
  for (int i = 0; i < n5; ++i) p.r[p.nst++] = 5;
  return p;
}

constexpr int ct_ns(int n, int s) {
  int ns = 1;
  for (int i = 0; i < s; ++i) ns *= ct_radices(n).r[i];
  return ns;
}

// Complex values per lane in a fixed-length stage: kWaveRegs, and 24 for
// lines past 768 points (a 1536-point line: three radix-8 butterflies or
// eight radix-3 ones per lane).
constexpr int ct_wave_regs(int n) { return n > 768 ? 24 : kWaveRegs; }

// Lines one wavefront carries through every stage (the planner's rule).
constexpr int ct_wave_lines(int n) {
  const CtRadices p = ct_radices(n);
  int gl = 0;
  for (int l = 1; l <= 8; ++l) {
    bool ok = true;
    for (int i = 0; i < p.nst; ++i)
      if ((l * (n / p.r[i]) + 63) / 64 > ct_wave_regs(n) / p.r[i]) ok = false;
    if (!ok) break;
    gl = l;
  }
  return gl;
}

template <typename T, bool INV, int N, int S>
__device__ __forceinline__ void ct_stages(LdsC2<T> b0, int nl, LdsTw<T> tw, int lane) {
  constexpr CtRadices P = ct_radices(N);
  if constexpr (S < P.nst) {
    constexpr int R = P.r[S];
    constexpr int NS = ct_ns(N, S);
    constexpr int PP = 1 << pad_shift<T>();
    constexpr bool AFF = (N / R) % PP == 0 && (NS % PP == 0 || (NS == 1 && PP % R == 0));
    stage_body<T, R, INV, ct_wave_regs(N) / R, false, AFF, true>(b0, nl, N, lds_line<T>(N), NS,
                                                                 tw, lane, 64);
    ct_stages<T, INV, N, S + 1>(b0, nl, tw, lane);
  }
}

// fft_wave for the fixed length N (line stride lds_line<T>(N)).
template <typename T, bool INV, int N>
__device__ __forceinline__ void fft_wave_ct(C2<T> *buf, int nlines, const TwT<T> *tw, int lane) {
  constexpr int GL = ct_wave_lines(N);
  static_assert(GL > 0, "length too long for a wavefront-scope transform");
  constexpr int LS = lds_line<T>(N);
  LdsTw<T> twl = to_lds_tw<T>(tw);
  for (int l0 = 0; l0 < nlines; l0 += GL) {
    const int nl = nlines - l0 < GL ? nlines - l0 : GL;
    ct_stages<T, INV, N, 0>(to_lds(buf + l0 * LS), nl, twl, lane);
  }
}

// Radix orders of the fixed lengths n = 3 * 2^a: ORD_PLAN the planner's
// (powers of two, then radix 3), ORD_3FIRST radix 3 first, then the
// planner's powers of two.  In a 3-first transform the first stage's
// butterflies read elements j, j + n/3, j + 2n/3, so the zero third of a
// Hermitian-extended line (positions M..2M of a 3M-point line) falls on the
// middle leg of every butterfly.
enum { ORD_PLAN = 0, ORD_3FIRST = 1 };

constexpr CtRadices ct_order(int n, int ord) {
  const CtRadices p = ct_radices(n);
  if (ord == ORD_PLAN) return p;
  CtRadices q{0, {}};
  q.r[q.nst++] = 3;
  bool dropped = false;
  for (int i = 0; i < p.nst; ++i) {
    if (p.r[i] == 3 && !dropped) {
      dropped = true;
      continue;
    }
    q.r[q.nst++] = p.r[i];
  }
  return q;
}

constexpr int ct_ns_ord(int n, int ord, int s) {
  int ns = 1;
  for (int i = 0; i < s; ++i) ns *= ct_order(n, ord).r[i];
  return ns;
}

// Stages S.. of the order ORD; SKIP: the last stage, if radix 3, stores only
// its outer two output thirds.
template <typename T, bool INV, int N, int ORD, int S, bool SKIP>
__device__ __forceinline__ void ct_stages_ord(LdsC2<T> b0, int nl, LdsTw<T> tw, int lane) {
  constexpr CtRadices P = ct_order(N, ORD);
  if constexpr (S < P.nst) {
    constexpr int R = P.r[S];
    constexpr int NS = ct_ns_ord(N, ORD, S);
    constexpr int PP = 1 << pad_shift<T>();
    constexpr bool AFF = (N / R) % PP == 0 && (NS % PP == 0 || (NS == 1 && PP % R == 0));
    constexpr bool SKIPMID = SKIP && S == P.nst - 1 && R == 3;
    stage_body<T, R, INV, ct_wave_regs(N) / R, false, AFF, true, SKIPMID>(
        b0, nl, N, lds_line<T>(N), NS, tw, lane, 64);
    ct_stages_ord<T, INV, N, ORD, S + 1, SKIP>(b0, nl, tw, lane);
  }
}

// Stages S0.. of the order ORD over `nlines` lines of one wavefront (line
// stride lds_line<T>(N)), in groups of the lines a wavefront carries.
template <typename T, bool INV, int N, int ORD, int S0, bool SKIP>
__device__ __forceinline__ void fft_wave_ct_ord(C2<T> *buf, int nlines, const TwT<T> *tw,
                                                int lane) {
  constexpr int GL = ct_wave_lines(N);
  static_assert(GL > 0, "length too long for a wavefront-scope transform");
  constexpr int LS = lds_line<T>(N);
  LdsTw<T> twl = to_lds_tw<T>(tw);
  for (int l0 = 0; l0 < nlines; l0 += GL) {
    const int nl = nlines - l0 < GL ? nlines - l0 : GL;
    ct_stages_ord<T, INV, N, ORD, S0, SKIP>(to_lds(buf + l0 * LS), nl, twl, lane);
  }
}

// Stages S.. of the order ORD over NL lines (stride lds_line_s<SH>(N)) by a
// group of G threads (tid = 0..G-1) of a workgroup whose groups all run the
// same stages: each thread holds its ceil(NL N / (R G)) butterflies of a
// stage in registers between the read and the write phase, which are
// separated by workgroup barriers.
template <typename T, bool INV, int N, int ORD, int S, bool SKIP, int NL, int G, int SH>
__device__ __forceinline__ void ct_stages_grp(LdsC2<T> b0, LdsTw<T> tw, int tid) {
  constexpr CtRadices P = ct_order(N, ORD);
  if constexpr (S < P.nst) {
    constexpr int R = P.r[S];
    constexpr int NS = ct_ns_ord(N, ORD, S);
    constexpr int PP = 1 << SH;
    constexpr bool AFF = (N / R) % PP == 0 && (NS % PP == 0 || (NS == 1 && PP % R == 0));
    constexpr bool SKIPMID = SKIP && S == P.nst - 1 && R == 3;
    constexpr int MW = (NL * (N / R) + G - 1) / G;
    stage_body<T, R, INV, MW, true, AFF, true, SKIPMID, SH>(b0, NL, N, lds_line_s<SH>(N), NS, tw,
                                                             tid, G);
    ct_stages_grp<T, INV, N, ORD, S + 1, SKIP, NL, G, SH>(b0, tw, tid);
  }
}

// The nl lines of a workgroup: with a wavefront-scope plan each wavefront
// transforms a contiguous share of them and the workgroup meets once at the
// end; otherwise the whole workgroup works on each group of lines together.
// NF > 0: the line length is the compile-time constant NF.
template <typename T, bool INV, int MAXB, int NF = 0>
__device__ __forceinline__ void fft_block(C2<T> *buf, int nl, int ls, const FftPlan &plan,
                                          const TwT<T> *tw) {
  if (NF > 0 || plan.wave_lines > 0) {  // (fixed lengths always fit a wavefront)
    const int nw = (int)(blockDim.x >> 6), w = (int)(threadIdx.x >> 6);
    const int per = (nl + nw - 1) / nw;
    const int l0 = w * per;
    const int cnt = nl - l0 < per ? nl - l0 : per;
    const int lane = (int)(threadIdx.x & 63);
    if (cnt > 0) {
      if constexpr (NF > 0) fft_wave_ct<T, INV, NF>(buf + l0 * ls, cnt, tw, lane);
      else fft_wave<T, INV>(buf + l0 * ls, cnt, ls, plan, tw, lane);
    }
    __syncthreads();
  } else if constexpr (NF == 0) {
    fft_lines<T, INV, MAXB>(buf, nl, ls, plan, tw);
  }
}

}  // namespace nsc
