// Pseudospectral nonlinear term on gfx950 (section 2.1 of the nsCouette
// paper: Fourier--Galerkin in theta and z, pseudospectral products).
//
// Three passes over HBM:
//   k_zinv   spectral state [F][N_r][M_theta][M_z] -> derived fields (u,
//            curl u, grad T) per (r, m) line, zero-padded to N_z, inverse
//            FFT in z, stored transposed as Z[n_in][N_r][N_z][M_theta]
//            (theta-lines contiguous);
//   k_theta  per (r, z) line: pairs of real fields packed into one complex
//            Hermitian-extended line of length N_theta, inverse FFT, pointwise
//            u x omega and -u . grad T plus the CFL bound, forward FFT,
//            unpacking, W[n_out][N_r][N_z][M_theta];
//   k_zfwd   W -> forward FFT in z, truncation to |k| <= K, scaling
//            1/(N_theta N_z), buoyancy N_z += Gr T, Hermitian m = 0 column.
// T = double (FP64) or float (mixed precision); the spectral state and the
// output stay FP64.
#include <cfloat>
#include <climits>
#include <type_traits>

#include "fft_lds.h"

namespace nsc {
namespace {

constexpr int kMaxB = 1;
constexpr int kThetaWaveThreads = 256;  // at most four line sets per workgroup  // one butterfly per thread per stage: low register use, high occupancy

// Items (row, col) of a rows x cols index space taken by thread t of n in
// row-major order (item t + i n), stepped without a division per item.
struct Walk2 {
  int r, c, dr, dc, cols;
  __device__ __forceinline__ Walk2(int t, int n, int cols_) : cols(cols_) {
    r = t / cols;
    c = t - r * cols;
    dr = n / cols;
    dc = n - dr * cols;
  }
  __device__ __forceinline__ void next() {
    r += dr;
    c += dc;
    if (c >= cols) {
      c -= cols;
      ++r;
    }
  }
};

// Field F of the derived set at radial row j, mode (m, kk): 0..2 u_r,
// u_theta, u_z; 3..5 omega_r, omega_theta, omega_z; 6..8 grad T.  With
// drop_mean the mode (0,0) -- the r-only mean flow, whose products are
// formed exactly per mode in k_zfwd -- is left out of the transforms.  PIPE:
// the radial derivative of an order-m coefficient uses the rows of its
// parity in r, (-1)^(m+1) for u_r and u_theta, (-1)^m for u_z.  The field is
// a compile-time constant so that the row and weight addresses, uniform over
// a workgroup (one row, one field), are formed once outside the item loop.
template <bool PIPE>
struct DerivedRow {
  const Dims &d;
  const Grid &g;
  const double2 *__restrict__ u;
  int j, s;
  bool drop_mean;
  __device__ DerivedRow(const Dims &d_, const Grid &g_, const double2 *__restrict__ u_, int j_,
                        bool drop)
      : d(d_), g(g_), u(u_), j(j_), s(g_.s[j_]), drop_mean(drop) {}
  __device__ __forceinline__ double2 U(int fld, int row, size_t md) const {
    return u[((size_t)fld * d.nr + row) * (size_t)d.nmodes + md];
  }
  __device__ __forceinline__ double2 D1(int fld, int m, size_t md) const {
    const double *w = g.d1 + j * kStencil;
    if constexpr (PIPE) w += odd_off(g, fld == 1 ? m + 1 : m);
    double2 acc = {0.0, 0.0};
#pragma unroll
    for (int t = 0; t < kStencil; ++t) {
      double2 v = U(fld, s + t, md);
      acc.x = fma(w[t], v.x, acc.x);
      acc.y = fma(w[t], v.y, acc.y);
    }
    return acc;
  }
  template <int F>
  __device__ __forceinline__ double2 get(int m, int kk) const {
    const size_t md = (size_t)m * d.mz + kk;
    if (drop_mean && m == 0 && kk == d.kmax) return make_double2(0.0, 0.0);
    const double kap = (double)(kk - d.kmax) * d.kz;
    const double mr = (double)m * g.rinv[j];
    if constexpr (F <= 2) {
      return U(F, j, md);
    } else if constexpr (F == 3) {  // (i m / r) u_z - i kappa u_theta
      double2 a = U(2, j, md), b = U(1, j, md);
      double re = mr * a.x - kap * b.x, im = mr * a.y - kap * b.y;
      return {-im, re};
    } else if constexpr (F == 4) {  // i kappa u_r - D1 u_z
      double2 a = U(0, j, md), dz = D1(2, m, md);
      return {-kap * a.y - dz.x, kap * a.x - dz.y};
    } else if constexpr (F == 5) {  // D1 u_theta + u_theta / r - (i m / r) u_r
      double2 dt = D1(1, m, md), b = U(1, j, md), a = U(0, j, md);
      const double ri = g.rinv[j];
      return {dt.x + b.x * ri + mr * a.y, dt.y + b.y * ri - mr * a.x};
    } else if constexpr (F == 6) {
      return D1(3, m, md);
    } else if constexpr (F == 7) {  // (i m / r) T
      double2 a = U(3, j, md);
      return {-mr * a.y, mr * a.x};
    } else {  // i kappa T
      double2 a = U(3, j, md);
      return {-kap * a.y, kap * a.x};
    }
  }
};

// Mean-flow profiles of mode (0,0) at radial row j (real parts, as carried
// by the physical field) and their discrete derivatives: mean[.][j] = U_r,
// V, W, T_m, Om_theta = -D1 W, Om_z = D1 V + V/r, G = D1 T_m.
__device__ void mean_row(const Dims &d, const Grid &g, const double2 *__restrict__ u,
                         double *__restrict__ mean, int j) {
  const int n = d.nr;
  const size_t P = d.nmodes;
  auto M = [&](int f, int row) { return u[((size_t)f * n + row) * P + d.kmax].x; };
  const int s = g.s[j];
  const double *w = g.d1 + j * kStencil;
  const double *wv = w + g.podd;  // V = u_theta of order 0: odd in r in the pipe
  double dv = 0.0, dw = 0.0, dt = 0.0;
  for (int t = 0; t < kStencil; ++t) {
    dv = fma(wv[t], M(1, s + t), dv);
    dw = fma(w[t], M(2, s + t), dw);
    if (d.heated) dt = fma(w[t], M(3, s + t), dt);
  }
  mean[j] = M(0, j);
  mean[n + j] = M(1, j);
  mean[2 * n + j] = M(2, j);
  mean[3 * n + j] = d.heated ? M(3, j) : 0.0;
  mean[4 * n + j] = -dw;
  mean[5 * n + j] = dv + M(1, j) * g.rinv[j];
  mean[6 * n + j] = dt;
}

constexpr int ZU = 4;  // z-pass items per round of loads (2: about half the gain)
template <typename T, int NF, bool PIPE = false>
__global__ void __launch_bounds__(kFftThreads) k_zinv(Dims d, Grid g, FftPlan pz, const double2 *__restrict__ u,
                       C2<T> *__restrict__ Z, const TwT<T> *__restrict__ tw, int tm, int drop_mean,
                       double *__restrict__ mean) {
  extern __shared__ __align__(16) unsigned char smem[];
  TwT<T> *tws = reinterpret_cast<TwT<T> *>(smem);
  C2<T> *buf = reinterpret_cast<C2<T> *>(tws + d.nz);
  int bx, j, f;
  xcd_block_zfirst(bx, j, f);  // the fields of one tile share their u rows
  const int nz = d.nz, K = d.kmax;
  const int ls = lds_line<T>(nz);
  const int mt0 = bx * tm;
  const int nl = min(tm, d.mt - mt0);
  load_twiddles(tws, tw, nz);
  // one workgroup per radial row also records the mean-flow profiles there
  if (bx == 0 && f == 0 && threadIdx.x == 0) mean_row(d, g, u, mean, j);
  // retained modes: one item per (line, k) so that every thread's loads are
  // independent and issued together; then the zero padding.  (A pruned
  // radix-3-first variant that fed the derived values of the two retained
  // modes of each butterfly straight into it measured slower on the
  // 1536-point lines and no faster on the 192-point ones.)
  const int mz = d.mz;
  // ZU items per round, their loads issued together (items past the tile
  // repeat its last line and are not stored); one loop per field
  const DerivedRow<PIPE> der(d, g, u, j, drop_mean != 0);
  auto fill = [&](auto field) {
    constexpr int FLD = decltype(field)::value;
    Walk2 w(threadIdx.x, blockDim.x, mz);
    while (w.r < nl) {
      int li[ZU], kk[ZU];
#pragma unroll
      for (int i = 0; i < ZU; ++i) {
        li[i] = w.r;
        kk[i] = w.c;
        w.next();
      }
      double2 v[ZU];
#pragma unroll
      for (int i = 0; i < ZU; ++i)
        v[i] = der.template get<FLD>(mt0 + (li[i] < nl ? li[i] : nl - 1), kk[i]);
#pragma unroll
      for (int i = 0; i < ZU; ++i) {
        const int k = kk[i] - K;
        if (li[i] < nl) buf[li[i] * ls + PD<T>((k >= 0 ? k : nz + k))] = {T(v[i].x), T(v[i].y)};
      }
    }
  };
  switch (f) {
    case 0: fill(std::integral_constant<int, 0>{}); break;
    case 1: fill(std::integral_constant<int, 1>{}); break;
    case 2: fill(std::integral_constant<int, 2>{}); break;
    case 3: fill(std::integral_constant<int, 3>{}); break;
    case 4: fill(std::integral_constant<int, 4>{}); break;
    case 5: fill(std::integral_constant<int, 5>{}); break;
    case 6: fill(std::integral_constant<int, 6>{}); break;
    case 7: fill(std::integral_constant<int, 7>{}); break;
    default: fill(std::integral_constant<int, 8>{}); break;
  }
  const int npad = nz - mz;
  for (Walk2 w(threadIdx.x, blockDim.x, npad); w.r < nl; w.next())
    buf[w.r * ls + PD<T>(K + 1 + w.c)] = {T(0), T(0)};
  __syncthreads();
  fft_block<T, true, kMaxB, NF>(buf, nl, ls, pz, tws);
  C2<T> *out = Z + ((size_t)f * d.nr + j) * nz * d.mt;
  for (Walk2 w(threadIdx.x, blockDim.x, nl); w.r < nz; w.next()) {
    const int b = w.r;
    const int li = w.c;
    out[(size_t)b * d.mt + mt0 + li] = buf[li * ls + PD<T>(b)];
  }
}

// Lines p = 0..np-1 of buf: Z_m = F_{2p,m} + i F_{2p+1,m} for 0 < m < M_theta,
// Z_{N-m} = conj F_{2p,m} + i conj F_{2p+1,m}, Z_0 = Re F_{2p,0} + i Re F_{2p+1,0},
// zero elsewhere, so that the inverse FFT yields the two real fields.
template <typename T>
__device__ __forceinline__ void pack_pairs(C2<T> *buf, int ls, const C2<T> *__restrict__ zl,
                                           size_t fstride, int nf, int np, int nt, int mt,
                                           int gt, int gsz) {
  for (Walk2 w(gt, gsz, mt); w.r < np; w.next()) {
    const int p = w.r;
    const int m = w.c;
    const int f1 = 2 * p, f2 = 2 * p + 1;
    const C2<T> F1 = zl[f1 * fstride + m];
    const C2<T> F2 = f2 < nf ? zl[f2 * fstride + m] : C2<T>{T(0), T(0)};
    C2<T> *L = buf + p * ls;
    if (m == 0) {
      L[0] = {F1.x, F2.x};
    } else {
      L[PD<T>(m)] = {F1.x - F2.y, F1.y + F2.x};
      L[PD<T>(nt - m)] = {F1.x + F2.y, F2.x - F1.y};
    }
  }
  const int nzero = nt - 2 * mt + 1;
  for (Walk2 w(gt, gsz, nzero); w.r < np; w.next())
    buf[w.r * ls + PD<T>(mt + w.c)] = {T(0), T(0)};
}

// Work group of the theta pass: with WAVE one wavefront per (r, z) line set
// (several sets per workgroup, no workgroup barrier after the twiddle load),
// otherwise the whole workgroup on one set.
struct ThetaGroup {
  int set, gt, gsz, slot;
};

template <bool WAVE>
__device__ __forceinline__ ThetaGroup theta_group() {
  ThetaGroup t;
  if (WAVE) {
    const int nw = (int)(blockDim.x >> 6);
    t.slot = (int)(threadIdx.x >> 6);
    t.set = xcd_remap((int)blockIdx.x, (int)gridDim.x) * nw + t.slot;
    t.gt = (int)(threadIdx.x & 63);
    t.gsz = 64;
  } else {
    int bx, by, unused;
    xcd_block(bx, by, unused);
    t.set = by * (int)gridDim.x + bx;
    t.slot = 0;
    t.gt = (int)threadIdx.x;
    t.gsz = (int)blockDim.x;
  }
  return t;
}

template <bool WAVE>
__device__ __forceinline__ void group_sync() {
  if (WAVE) wave_sync();
  else __syncthreads();
}

template <typename T, bool WAVE, bool INV, int NF>
__device__ __forceinline__ void group_fft(C2<T> *buf, int nl, int ls, const FftPlan &p,
                                          const TwT<T> *tw, int gt) {
  if constexpr (WAVE && NF > 0) fft_wave_ct<T, INV, NF>(buf, nl, tw, gt);
  else if constexpr (WAVE) fft_wave<T, INV>(buf, nl, ls, p, tw, gt);
  else fft_lines<T, INV, kMaxB>(buf, nl, ls, p, tw);
}

template <typename T, bool WAVE, int NF>
__global__ void __launch_bounds__(WAVE ? kThetaWaveThreads : kFftThreads)
k_theta(Dims d, Grid g, FftPlan pt, const C2<T> *__restrict__ Z,
                        C2<T> *__restrict__ W, const TwT<T> *__restrict__ tw, int n_in,
                        double dth, double dzs, double *__restrict__ cfl_part,
                        int want_cfl, const double *__restrict__ mean) {
  extern __shared__ __align__(16) unsigned char smem[];
  TwT<T> *tws = reinterpret_cast<TwT<T> *>(smem);
  __shared__ double red[3 * (kFftThreads / 64)];
  const int nt = d.nt, mt = d.mt;
  const int ls = lds_line<T>(nt);
  const int npi = (n_in + 1) / 2;
  const ThetaGroup grp = theta_group<WAVE>();
  const int gt = grp.gt, gsz = grp.gsz;
  load_twiddles(tws, tw, nt);
  __syncthreads();
  if (grp.set >= d.nz * d.nr) return;  // wavefronts past the last set (WAVE only)
  const int j = grp.set / d.nz, b = grp.set - j * d.nz;  // radial row, z index
  C2<T> *buf = reinterpret_cast<C2<T> *>(tws + nt) + (size_t)grp.slot * npi * ls;
  const size_t fstride = (size_t)d.nr * d.nz * mt;
  const C2<T> *zl = Z + ((size_t)j * d.nz + b) * mt;
  // pack pairs of real fields into Hermitian-extended complex lines: one
  // item per (pair, m) fills positions m and N_theta - m
  pack_pairs(buf, ls, zl, fstride, n_in, npi, nt, mt, gt, gsz);
  group_sync<WAVE>();
  group_fft<T, WAVE, true, NF>(buf, npi, ls, pt, tws, gt);
  // pointwise products and CFL bound
  // CFL: the spacings are constant along the line set, so the smallest
  // Delta_i / |u_i| is Delta_i / max |u_i| (the same rounded value): the
  // maxima are reduced and three divisions close the set
  const double mur = mean[j], mut = mean[d.nr + j], muz = mean[2 * d.nr + j];
  const int nr = d.nr;
  const T mU = T(mur), mV = T(mut), mW = T(muz), mOt = T(mean[4 * nr + j]),
          mOz = T(mean[5 * nr + j]), mG = T(mean[6 * nr + j]);
  // running max |u_r|, |u_theta|, |u_z| in the working precision (the FP32
  // velocities of the mixed path gain nothing from FP64 maxima)
  T mr = T(0), mt_ = T(0), mz_ = T(0);
  bool bad = false;
  const bool heated = n_in > 6;
  for (int a = gt; a < nt; a += gsz) {
    const int pa = PD<T>(a);
    C2<T> l0 = buf[pa], l1 = buf[ls + pa], l2 = buf[2 * ls + pa];
    const T ur = l0.x, ut = l0.y, uz = l1.x, wr = l1.y, wt = l2.x, wz = l2.y;
    // u' x omega' + U x omega' + u' x Omega (Omega_r = 0); U x Omega is exact
    // in mode (0,0)
    const T nr_ = (ut * wz - uz * wt) + (mV * wz - mW * wt) + (ut * mOz - uz * mOt);
    const T nth = (uz * wr - ur * wz) + (mW * wr - mU * wz) - ur * mOz;
    const T nzz = (ur * wt - ut * wr) + (mU * wt - mV * wr) + ur * mOt;
    T ntt = T(0);
    if (heated) {
      // -(u' . grad T' + U . grad T' + u_r' dT_m/dr); -U_r dT_m/dr in mode (0,0)
      C2<T> l3 = buf[3 * ls + pa], l4 = buf[4 * ls + pa];
      ntt = -((ur * l3.x + ut * l3.y + uz * l4.x) + (mU * l3.x + mV * l3.y + mW * l4.x) +
              ur * mG);
    }
    buf[pa] = {nr_, nth};
    buf[ls + pa] = {nzz, ntt};
    if (want_cfl) {
      const T aur = fabs(ur + mU), aut = fabs(ut + mV), auz = fabs(uz + mW);
      if (!(isfinite(aur) && isfinite(aut) && isfinite(auz))) bad = true;
      mr = fmax(mr, aur);
      mt_ = fmax(mt_, aut);
      mz_ = fmax(mz_, auz);
    }
  }
  group_sync<WAVE>();
  group_fft<T, WAVE, false, NF>(buf, 2, ls, pt, tws, gt);
  // unpack the two real transforms of each line, keep m < M_theta
  const int nout = heated ? 4 : 3;
  C2<T> *wl = W + ((size_t)j * d.nz + b) * mt;
  for (Walk2 w(gt, gsz, mt); w.r < 2; w.next()) {
    const int p = w.r;
    const int m = w.c;
    const C2<T> zm = buf[p * ls + PD<T>(m)];
    const C2<T> zc = buf[p * ls + PD<T>(m == 0 ? 0 : nt - m)];
    // X = (Z_m + conj Z_{-m}) / 2, Y = (Z_m - conj Z_{-m}) / (2 i)
    const C2<T> x = {T(0.5) * (zm.x + zc.x), T(0.5) * (zm.y - zc.y)};
    const C2<T> y = {T(0.5) * (zm.y + zc.y), T(0.5) * (zc.x - zm.x)};
    wl[(size_t)(2 * p) * fstride + m] = x;
    if (2 * p + 1 < nout) wl[(size_t)(2 * p + 1) * fstride + m] = y;
  }
  if (want_cfl) {
    double xr = (double)mr, xt = (double)mt_, xz = (double)mz_;
    if (bad) xr = NAN;
    // wavefront reduction (max, NaN-propagating), then across the workgroup
    auto mx = [](double a, double b) { return (isnan(a) || isnan(b)) ? NAN : fmax(a, b); };
    for (int off = 32; off > 0; off >>= 1) {
      xr = mx(xr, __shfl_down(xr, off, 64));
      xt = mx(xt, __shfl_down(xt, off, 64));
      xz = mx(xz, __shfl_down(xz, off, 64));
    }
    auto bound = [&](double ar, double at, double az) {
      if (isnan(ar)) return (double)NAN;
      double v = DBL_MAX;
      if (ar > 0.0) v = fmin(v, g.dr[j] / ar);
      if (at > 0.0) v = fmin(v, g.r[j] * dth / at);
      if (az > 0.0) v = fmin(v, dzs / az);
      return v;
    };
    if (WAVE) {
      if (gt == 0) cfl_part[grp.set] = bound(xr, xt, xz);
    } else {
      const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
      if (lane == 0) {
        red[wid] = xr;
        red[16 + wid] = xt;
        red[32 + wid] = xz;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double ar = red[0], at = red[16], az = red[32];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
          ar = mx(ar, red[w]);
          at = mx(at, red[16 + w]);
          az = mx(az, red[32 + w]);
        }
        cfl_part[grp.set] = bound(ar, at, az);
      }
    }
  }
}

// Maximum over the wavefront of 32-bit values (DPP row shifts, then the
// row broadcasts), in every lane.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Theta pass for the fixed lengths N = 3 M (M = M_theta) with NI = 6 or 9
// derived fields (isothermal, heated).  A group of G threads per (r, z) line
// set, blockDim.x / G sets per workgroup sharing one twiddle table: G = 64,
// one wavefront per set, needs no workgroup barrier in the transforms (the
// short lines, 48..768 points); G > 64 (the long lines) runs each stage at
// workgroup scope.  LDS lines have one pad slot per 2^SH elements.
//   * Packing and the first inverse stage are one step: the inverse runs
//     radix 3 first, whose butterfly q reads positions q, q + M, q + 2M of
//     the Hermitian-extended line -- Z_q (mode q), zero (the padding), and
//     Z_{N-(M-q)} (the conjugate half, mode M - q) -- so each thread loads
//     the two modes from the intermediate array, forms the pruned radix-3
//     butterfly in registers and writes its three outputs: no zero fill and
//     no LDS round trip for the packing.
//   * The forward transform runs radix 3 last and stores only the outer two
//     thirds of that stage's outputs (modes below M and their mirrors).
//   * The CFL maxima of the FP32 path are taken on the bit patterns of |u|
//     (non-negative floats order as unsigned integers, NaN and infinity above
//     every finite value, so the maximum also flags them), reduced across
//     each wavefront by DPP.
template <typename T, int N, int NI, int G, int SH>
__global__ void __launch_bounds__(G == 64 ? kThetaWaveThreads : kFftThreads)
k_theta_fx(Dims d, Grid g, const C2<T> *__restrict__ Z, C2<T> *__restrict__ W,
           const TwT<T> *__restrict__ tw, double dth, double dzs, double *__restrict__ cfl_part,
           int want_cfl, const double *__restrict__ mean) {
  constexpr int MT = N / 3;
  constexpr int LS = lds_line_s<SH>(N);
  constexpr int NP = (NI + 1) / 2;  // packed lines
  constexpr bool HEATED = NI > 6;
  constexpr bool WAVE = G == 64;
  constexpr int NW = G / 64;  // wavefronts per set
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[3][kFftThreads / 64];
  TwT<T> *tws = reinterpret_cast<TwT<T> *>(smem);
  const int sets = (int)blockDim.x / G;
  const int slot = (int)threadIdx.x / G, tid = (int)threadIdx.x - slot * G;
  const int nsets = d.nz * d.nr;
  const int set0 = xcd_remap((int)blockIdx.x, (int)gridDim.x) * sets + slot;
  const bool valid = set0 < nsets;
  load_twiddles(tws, tw, N);
  __syncthreads();
  if (WAVE && !valid) return;  // wavefronts past the last set (no barrier follows)
  // a group past the last set (G > 64) repeats the last set's work for the
  // workgroup barriers, and stores nothing
  const int set = valid ? set0 : nsets - 1;
  const int j = set / d.nz, b = set - j * d.nz;  // radial row, z index
  C2<T> *buf = reinterpret_cast<C2<T> *>(tws + N) + (size_t)slot * NP * LS;
  LdsC2<T> bl = to_lds(buf);
  LdsTw<T> twl = to_lds_tw<T>(tws);
  const size_t fstride = (size_t)d.nr * d.nz * MT;
  const C2<T> *zl = Z + ((size_t)j * d.nz + b) * MT;
  // packing + pruned radix-3 stage (inverse: w = e^{+2 pi i/3}); butterfly
  // (p, q): a = Z_q, c = Z_{N-(M-q)} (zero for q = 0: mode M is not kept)
  constexpr double H3 = 0.86602540378443864676372317075294;  // sqrt(3)/2
  // all loads of the thread's items first (kept ahead of the butterflies by
  // a scheduling barrier), so that they are in flight together; q = 0 reads
  // its own mode in place of the mirror and drops it
  constexpr int NIT = (NP * MT + G - 1) / G;
  C2<T> F1[NIT], F2[NIT], G1[NIT], G2[NIT];
#pragma unroll
  for (int i = 0; i < NIT; ++i) {
    const int it = i * G + tid;
    const int p = (it < NP * MT ? it : 0) / MT, q = (it < NP * MT ? it : 0) - p * MT;
    const int qm = q == 0 ? 0 : MT - q;
    const C2<T> *f1 = zl + (size_t)(2 * p) * fstride;
    const bool two = 2 * p + 1 < NI;
    F1[i] = f1[q];
    G1[i] = f1[qm];
    F2[i] = two ? f1[fstride + q] : C2<T>{T(0), T(0)};
    G2[i] = two ? f1[fstride + qm] : C2<T>{T(0), T(0)};
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < NIT; ++i) {
    const int it = i * G + tid;
    if (it < NP * MT) {
      const int p = it / MT, q = it - p * MT;
      C2<T> a, c;
      if (q == 0) {
        a = {F1[i].x, F2[i].x};
        c = {T(0), T(0)};
      } else {
        a = {F1[i].x - F2[i].y, F1[i].y + F2[i].x};
        c = {G1[i].x + G2[i].y, G2[i].x - G1[i].y};
      }
      // y0 = a + c, y1 = a + e^{4 pi i/3} c, y2 = a + e^{2 pi i/3} c
      const C2<T> t = {a.x - T(0.5) * c.x, a.y - T(0.5) * c.y};
      const C2<T> hc = {kmul<T>(H3, c.x), kmul<T>(H3, c.y)};
      LdsC2<T> L = bl + p * LS;
      lds_st(L + PDs<SH>(3 * q), cadd(a, c));
      lds_st(L + PDs<SH>(3 * q + 1), C2<T>{t.x + hc.y, t.y - hc.x});
      lds_st(L + PDs<SH>(3 * q + 2), C2<T>{t.x - hc.y, t.y + hc.x});
    }
  }
  if constexpr (WAVE) {
    wave_sync();
    fft_wave_ct_ord<T, true, N, ORD_3FIRST, 1, false>(buf, NP, tws, tid);
  } else {
    __syncthreads();
    ct_stages_grp<T, true, N, ORD_3FIRST, 1, false, NP, G, SH>(bl, twl, tid);
  }
  // pointwise products and CFL maxima
  const int nr = d.nr;
  const T mU = T(mean[j]), mV = T(mean[nr + j]), mW = T(mean[2 * nr + j]),
          mOt = T(mean[4 * nr + j]), mOz = T(mean[5 * nr + j]), mG = T(mean[6 * nr + j]);
  unsigned br = 0, bt = 0, bz = 0;  // FP32: bit patterns of the maxima
  T mr = T(0), mt_ = T(0), mz_ = T(0);
  bool bad = false;
#pragma unroll
  for (int a0 = 0; a0 < N; a0 += G) {
    const int a = a0 + tid;
    if (a < N) {
      LdsC2<T> P0 = bl + PDs<SH>(a);
      const C2<T> l0 = lds_ld(P0), l1 = lds_ld(P0 + LS), l2 = lds_ld(P0 + 2 * LS);
      const T ur = l0.x, ut = l0.y, uz = l1.x, wr = l1.y, wt = l2.x, wz = l2.y;
      // u' x omega' + U x omega' + u' x Omega (Omega_r = 0); U x Omega is
      // exact in mode (0,0)
      const T nr_ = (ut * wz - uz * wt) + (mV * wz - mW * wt) + (ut * mOz - uz * mOt);
      const T nth = (uz * wr - ur * wz) + (mW * wr - mU * wz) - ur * mOz;
      const T nzz = (ur * wt - ut * wr) + (mU * wt - mV * wr) + ur * mOt;
      T ntt = T(0);
      if constexpr (HEATED) {
        // -(u' . grad T' + U . grad T' + u_r' dT_m/dr)
        const C2<T> l3 = lds_ld(P0 + 3 * LS), l4 = lds_ld(P0 + 4 * LS);
        ntt = -((ur * l3.x + ut * l3.y + uz * l4.x) + (mU * l3.x + mV * l3.y + mW * l4.x) +
                ur * mG);
      }
      lds_st(P0, C2<T>{nr_, nth});
      lds_st(P0 + LS, C2<T>{nzz, ntt});
      if (want_cfl) {
        const T aur = fabs(ur + mU), aut = fabs(ut + mV), auz = fabs(uz + mW);
        if constexpr (sizeof(T) == 4) {
          br = max(br, __float_as_uint(aur));
          bt = max(bt, __float_as_uint(aut));
          bz = max(bz, __float_as_uint(auz));
        } else {
          if (!(isfinite(aur) && isfinite(aut) && isfinite(auz))) bad = true;
          mr = fmax(mr, aur);
          mt_ = fmax(mt_, aut);
          mz_ = fmax(mz_, auz);
        }
      }
    }
  }
  if constexpr (WAVE) {
    wave_sync();
    fft_wave_ct_ord<T, false, N, ORD_PLAN, 0, true>(buf, 2, tws, tid);
  } else {
    __syncthreads();
    ct_stages_grp<T, false, N, ORD_PLAN, 0, true, 2, G, SH>(bl, twl, tid);
  }
  // unpack the two real transforms of each line, keep m < M_theta
  C2<T> *wl = W + ((size_t)j * d.nz + b) * MT;
  if (valid) {
#pragma unroll
    for (int it0 = 0; it0 < 2 * MT; it0 += G) {
      const int it = it0 + tid;
      if (it < 2 * MT) {
        const int p = it / MT, m = it - p * MT;
        const C2<T> zm = lds_ld(bl + p * LS + PDs<SH>(m));
        const C2<T> zc = lds_ld(bl + p * LS + PDs<SH>(m == 0 ? 0 : N - m));
        // X = (Z_m + conj Z_{-m}) / 2, Y = (Z_m - conj Z_{-m}) / (2 i)
        wl[(size_t)(2 * p) * fstride + m] = {T(0.5) * (zm.x + zc.x), T(0.5) * (zm.y - zc.y)};
        if (HEATED || p == 0)
          wl[(size_t)(2 * p + 1) * fstride + m] = {T(0.5) * (zm.y + zc.y), T(0.5) * (zc.x - zm.x)};
      }
    }
  }
  if (want_cfl) {
    // this wavefront's maxima (xr NaN: a value was not finite)
    double xr, xt, xz;
    auto mx = [](double u, double v) { return (isnan(u) || isnan(v)) ? NAN : fmax(u, v); };
    if constexpr (sizeof(T) == 4) {
      br = wave_max_u32(br);
      bt = wave_max_u32(bt);
      bz = wave_max_u32(bz);
      const unsigned inf = 0x7f800000u;
      xr = (br >= inf || bt >= inf || bz >= inf) ? (double)NAN : (double)__uint_as_float(br);
      xt = (double)__uint_as_float(bt);
      xz = (double)__uint_as_float(bz);
    } else {
      xr = (double)mr;
      xt = (double)mt_;
      xz = (double)mz_;
      if (bad) xr = NAN;
      for (int off = 32; off > 0; off >>= 1) {  // total in lane 0
        xr = mx(xr, __shfl_down(xr, off, 64));
        xt = mx(xt, __shfl_down(xt, off, 64));
        xz = mx(xz, __shfl_down(xz, off, 64));
      }
    }
    if constexpr (!WAVE) {  // across the group's wavefronts
      const int w = tid >> 6;
      if ((tid & 63) == 0) {
        red[0][slot * NW + w] = xr;
        red[1][slot * NW + w] = xt;
        red[2][slot * NW + w] = xz;
      }
      __syncthreads();
      xr = red[0][slot * NW];
      xt = red[1][slot * NW];
      xz = red[2][slot * NW];
#pragma unroll
      for (int k = 1; k < NW; ++k) {
        xr = mx(xr, red[0][slot * NW + k]);
        xt = mx(xt, red[1][slot * NW + k]);
        xz = mx(xz, red[2][slot * NW + k]);
      }
    }
    if (tid == 0 && valid) {
      double v = DBL_MAX;
      if (isnan(xr)) {
        v = NAN;
      } else {
        if (xr > 0.0) v = fmin(v, g.dr[j] / xr);
        if (xt > 0.0) v = fmin(v, g.r[j] * dth / xt);
        if (xz > 0.0) v = fmin(v, dzs / xz);
      }
      cfl_part[set] = v;
    }
  }
}

// Spectral terms added to output field f at (j, m, kk): in mode (0,0) the
// mean-flow products U x Omega and -U_r dT_m/dr (r only, formed exactly),
// and the buoyancy Gr T in the axial component.  mean[.][j]: U_r, V, W, T_m,
// Om_theta = -D1 W, Om_z = D1 V + V/r, G = D1 T_m.
template <bool GR>
__device__ __forceinline__ double2 spectral_terms(const Dims &d, const double *__restrict__ mean,
                                                  int f, int j, int m, int kk, double2 t) {
  const int n = d.nr;
  double2 o = make_double2(0.0, 0.0);
  if (m == 0 && kk == d.kmax) {
    const double Ur = mean[j], V = mean[n + j], W = mean[2 * n + j];
    const double Ot = mean[4 * n + j], Oz = mean[5 * n + j], G = mean[6 * n + j];
    if (f == 0) o.x = V * Oz - W * Ot;
    else if (f == 1) o.x = -Ur * Oz;
    else if (f == 2) o.x = Ur * Ot;
    else o.x = -Ur * G;
  }
  if constexpr (GR) {  // u_z of a heated run: t the temperature coefficient
    o.x += d.gr * t.x;
    o.y += d.gr * t.y;
  }
  return o;
}

// Minimum of the per-line CFL bounds over the whole grid (a NaN anywhere
// gives NaN), by one workgroup: written to the device result and, when
// given, to a host-mapped pinned scalar, so that the host reads the bound
// without a separate copy.
__device__ void cfl_reduce(const double *__restrict__ part, int n, double *out, double *out_host) {
  __shared__ double red[kFftThreads / 64];
  auto nanmin = [](double a, double b) { return (isnan(a) || isnan(b)) ? NAN : fmin(a, b); };
  // eight loads in flight per thread (the minimum does not depend on the order)
  const int bd = blockDim.x;
  double acc[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) acc[a] = DBL_MAX;
  int i = threadIdx.x;
  for (; i + 7 * bd < n; i += 8 * bd) {
    double p[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) p[a] = part[i + a * bd];
#pragma unroll
    for (int a = 0; a < 8; ++a) acc[a] = nanmin(acc[a], p[a]);
  }
  for (; i < n; i += bd) acc[0] = nanmin(acc[0], part[i]);
  double v = acc[0];
#pragma unroll
  for (int a = 1; a < 8; ++a) v = nanmin(v, acc[a]);
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_down(v, off, 64);
    v = (isnan(o) || isnan(v)) ? NAN : fmin(v, o);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < (int)((blockDim.x + 63) >> 6); ++w)
      r = (isnan(r) || isnan(red[w])) ? NAN : fmin(r, red[w]);
    out[0] = r;
    if (out_host) out_host[0] = r;
  }
}

template <typename T, int NF>
__global__ void __launch_bounds__(kFftThreads) k_zfwd(Dims d, Grid g, FftPlan pz, const C2<T> *__restrict__ W,
                       const double2 *__restrict__ u, double2 *__restrict__ nh,
                       const TwT<T> *__restrict__ tw, int tm, double scale,
                       const double *__restrict__ mean, const double *__restrict__ cfl_part,
                       int cfl_n, double *cfl_out, double *cfl_host) {
  extern __shared__ __align__(16) unsigned char smem[];
  TwT<T> *tws = reinterpret_cast<TwT<T> *>(smem);
  C2<T> *buf = reinterpret_cast<C2<T> *>(tws + d.nz);
  // the first workgroup dispatched also reduces the CFL bounds of the theta
  // pass (complete: that kernel ended before this one started)
  if (cfl_out && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0)
    cfl_reduce(cfl_part, cfl_n, cfl_out, cfl_host);
  int bx, j, f;
  xcd_block(bx, j, f);
  const int nz = d.nz, K = d.kmax, mz = d.mz;
  const int ls = lds_line<T>(nz);
  const int mt0 = bx * tm;
  const int nl = min(tm, d.mt - mt0);
  load_twiddles(tws, tw, nz);
  const C2<T> *in = W + ((size_t)f * d.nr + j) * nz * d.mt;
  // FP32: ZU items per round, their loads issued together (items past the
  // last z row repeat it and are not stored; 768-point lines 454 -> 347 us,
  // 1536-point 6.5 -> 5.8 ms).  FP64 keeps one item per round (four were
  // two percent slower).
  constexpr int ZF = sizeof(T) == 4 ? ZU : 1;
  Walk2 w(threadIdx.x, blockDim.x, nl);
  while (w.r < nz) {
    int bz[ZF], li[ZF];
#pragma unroll
    for (int i = 0; i < ZF; ++i) {
      bz[i] = w.r;
      li[i] = w.c;
      w.next();
    }
    C2<T> v[ZF];
#pragma unroll
    for (int i = 0; i < ZF; ++i) v[i] = in[(size_t)(bz[i] < nz ? bz[i] : nz - 1) * d.mt + mt0 + li[i]];
#pragma unroll
    for (int i = 0; i < ZF; ++i)
      if (bz[i] < nz) buf[li[i] * ls + PD<T>(bz[i])] = v[i];
  }
  __syncthreads();
  if constexpr (NF > 0) {
    // fixed lengths: radix 3 last, whose middle third of outputs (|k| > K,
    // dropped by the truncation) is not stored
    const int nw = (int)(blockDim.x >> 6), wv = (int)(threadIdx.x >> 6);
    const int per = (nl + nw - 1) / nw;
    const int l0 = wv * per;
    const int cnt = nl - l0 < per ? nl - l0 : per;
    if (cnt > 0)
      fft_wave_ct_ord<T, false, NF, ORD_PLAN, 0, true>(buf + l0 * ls, cnt, tws,
                                                       (int)(threadIdx.x & 63));
    __syncthreads();
  } else {
    fft_block<T, false, kMaxB, NF>(buf, nl, ls, pz, tws);
  }
  const size_t plane = (size_t)d.nmodes;
  // one loop per case: with the buoyancy term (u_z of a heated run) each
  // round of items requests its temperature coefficients together (FP32:
  // ZU items per round, about 7 % less time on the 192-, 768- and
  // 1536-point grids; FP64 one item, as rounds of four were 8 % faster on
  // the 192-point grid but 9 % slower on the 768-point one)
  auto store = [&](auto buoyancy) {
    constexpr bool GR = decltype(buoyancy)::value;
    constexpr int ZS = sizeof(T) == 4 ? ZU : 1;
    const double2 *__restrict__ tr = u + ((size_t)3 * d.nr + j) * plane;
    Walk2 w(threadIdx.x, blockDim.x, mz);
    while (w.r < nl) {
      int li[ZS], kk[ZS];
#pragma unroll
      for (int i = 0; i < ZS; ++i) {
        li[i] = w.r;
        kk[i] = w.c;
        w.next();
      }
      double2 t[ZS] = {}, tm[ZS] = {};
      if constexpr (GR) {
#pragma unroll
        for (int i = 0; i < ZS; ++i) {
          const int m = mt0 + (li[i] < nl ? li[i] : nl - 1);
          t[i] = tr[(size_t)m * mz + kk[i]];
          tm[i] = m == 0 ? tr[mz - 1 - kk[i]] : make_double2(0.0, 0.0);
        }
      }
#pragma unroll
      for (int i = 0; i < ZS; ++i) {
        if (li[i] >= nl) continue;
        const int m = mt0 + li[i];
        const int k = kk[i] - K;
        const C2<T> v = buf[li[i] * ls + PD<T>((k >= 0 ? k : nz + k))];
        const double2 bt = spectral_terms<GR>(d, mean, f, j, m, kk[i], t[i]);
        double2 o = {(double)v.x * scale + bt.x, (double)v.y * scale + bt.y};
        const size_t md = (size_t)m * mz + kk[i];
        if (m == 0) {
          const int kkm = mz - 1 - kk[i];
          const C2<T> vm = buf[li[i] * ls + PD<T>((k <= 0 ? -k : nz - k))];
          const double2 bm = spectral_terms<GR>(d, mean, f, j, m, kkm, tm[i]);
          const double2 om = {(double)vm.x * scale + bm.x, (double)vm.y * scale + bm.y};
          o = {0.5 * (o.x + om.x), 0.5 * (o.y - om.y)};
        }
        nh[((size_t)f * d.nr + j) * plane + md] = o;
      }
    }
  };
  if (f == 2 && d.heated)
    store(std::true_type{});
  else
    store(std::false_type{});
}


// ---------------------------------------------------------------------------
// Vector--Jacobian product of the nonlinear term.  With the inverse transform
// Inv(x)_ab = Re sum c_m x_mk e^{i phi} and the forward F(f) = (N_theta N_z)^-1
// sum f e^{-i phi}, the transposes are F^T g = Inv(g / c_m) / (N_theta N_z)
// and Inv^T f = c_m * (unnormalised forward DFT of f).  For N = u x omega:
// ubar = omega x Nbar, omegabar = Nbar x u; for N_T = -u . G: ubar -= Nbar_T G,
// Gbar = -Nbar_T u.  Buoyancy: Tbar += Gr Nbar_z.
// ---------------------------------------------------------------------------

// Nbar (Hermitian-projected, divided by c_m and N_theta N_z) -> inverse z FFT.
template <typename T, int NF>
__global__ void __launch_bounds__(kFftThreads)
k_zinv_adj(Dims d, FftPlan pz, const double2 *__restrict__ nb, C2<T> *__restrict__ W,
           const TwT<T> *__restrict__ tw, int tm, double scale) {
  extern __shared__ __align__(16) unsigned char smem[];
  TwT<T> *tws = reinterpret_cast<TwT<T> *>(smem);
  C2<T> *buf = reinterpret_cast<C2<T> *>(tws + d.nz);
  int bx, j, f;
  xcd_block(bx, j, f);
  const int nz = d.nz, K = d.kmax, mz = d.mz;
  const int ls = lds_line<T>(nz);
  const int mt0 = bx * tm;
  const int nl = min(tm, d.mt - mt0);
  load_twiddles(tws, tw, nz);
  const size_t plane = (size_t)d.nmodes;
  const double2 *src = nb + ((size_t)f * d.nr + j) * plane;
  for (Walk2 w(threadIdx.x, blockDim.x, mz); w.r < nl; w.next()) {
    const int li = w.r;
    const int kk = w.c;
    const int k = kk - K;
    const int m = mt0 + li;
    double2 v = src[(size_t)m * mz + kk];
    if (m == 0) {
      const double2 w = src[mz - 1 - kk];
      v = make_double2(0.5 * (v.x + w.x), 0.5 * (v.y - w.y));
    }
    const double s = (m == 0 ? 1.0 : 0.5) * scale;
    buf[li * ls + PD<T>((k >= 0 ? k : nz + k))] = {T(v.x * s), T(v.y * s)};
  }
  const int npad = nz - mz;
  for (Walk2 w(threadIdx.x, blockDim.x, npad); w.r < nl; w.next())
    buf[w.r * ls + PD<T>(K + 1 + w.c)] = {T(0), T(0)};
  __syncthreads();
  fft_block<T, true, kMaxB, NF>(buf, nl, ls, pz, tws);
  C2<T> *out = W + ((size_t)f * d.nr + j) * nz * d.mt;
  for (Walk2 w(threadIdx.x, blockDim.x, nl); w.r < nz; w.next()) {
    const int b = w.r;
    const int li = w.c;
    out[(size_t)b * d.mt + mt0 + li] = buf[li * ls + PD<T>(b)];
  }
}

// Per (r, z) line: forward fields from Z, adjoint outputs from W; pointwise
// adjoint products; forward theta FFT of the input adjoints back into Z.
template <typename T, bool WAVE, int NF>
__global__ void __launch_bounds__(WAVE ? kThetaWaveThreads : kFftThreads)
k_theta_adj(Dims d, FftPlan pt, C2<T> *__restrict__ Z, const C2<T> *__restrict__ W,
            const TwT<T> *__restrict__ tw, int n_in, int n_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  TwT<T> *tws = reinterpret_cast<TwT<T> *>(smem);
  const int nt = d.nt, mt = d.mt;
  const int ls = lds_line<T>(nt);
  const int npi = (n_in + 1) / 2;
  const ThetaGroup grp = theta_group<WAVE>();
  const int gt = grp.gt, gsz = grp.gsz;
  load_twiddles(tws, tw, nt);
  __syncthreads();
  if (grp.set >= d.nz * d.nr) return;
  const int j = grp.set / d.nz, b = grp.set - j * d.nz;
  C2<T> *buf = reinterpret_cast<C2<T> *>(tws + nt) + (size_t)grp.slot * (npi + 2) * ls;
  const size_t fstride = (size_t)d.nr * d.nz * mt;
  C2<T> *zl = Z + ((size_t)j * d.nz + b) * mt;
  const C2<T> *wl = W + ((size_t)j * d.nz + b) * mt;
  pack_pairs(buf, ls, zl, fstride, n_in, npi, nt, mt, gt, gsz);
  pack_pairs(buf + npi * ls, ls, wl, fstride, n_out, 2, nt, mt, gt, gsz);
  group_sync<WAVE>();
  group_fft<T, WAVE, true, NF>(buf, npi + 2, ls, pt, tws, gt);
  const bool heated = n_in > 6;
  for (int a = gt; a < nt; a += gsz) {
    const int pa = PD<T>(a);
    const C2<T> l0 = buf[pa], l1 = buf[ls + pa], l2 = buf[2 * ls + pa];
    const C2<T> n0 = buf[npi * ls + pa], n1 = buf[(npi + 1) * ls + pa];
    const T ur = l0.x, ut = l0.y, uz = l1.x, wr = l1.y, wt = l2.x, wz = l2.y;
    const T nr_ = n0.x, nth = n0.y, nzz = n1.x, ntt = n1.y;
    T bur = wt * nzz - wz * nth;
    T but = wz * nr_ - wr * nzz;
    T buz = wr * nth - wt * nr_;
    const T bwr = nth * uz - nzz * ut;
    const T bwt = nzz * ur - nr_ * uz;
    const T bwz = nr_ * ut - nth * ur;
    if (heated) {
      const C2<T> l3 = buf[3 * ls + pa], l4 = buf[4 * ls + pa];
      bur -= ntt * l3.x;
      but -= ntt * l3.y;
      buz -= ntt * l4.x;
      buf[3 * ls + pa] = {-ntt * ur, -ntt * ut};
      buf[4 * ls + pa] = {-ntt * uz, T(0)};
    }
    buf[pa] = {bur, but};
    buf[ls + pa] = {buz, bwr};
    buf[2 * ls + pa] = {bwt, bwz};
  }
  group_sync<WAVE>();
  group_fft<T, WAVE, false, NF>(buf, npi, ls, pt, tws, gt);
  for (Walk2 w(gt, gsz, mt); w.r < npi; w.next()) {
    const int p = w.r;
    const int m = w.c;
    const C2<T> zm = buf[p * ls + PD<T>(m)];
    const C2<T> zc = buf[p * ls + PD<T>(m == 0 ? 0 : nt - m)];
    const C2<T> x = {T(0.5) * (zm.x + zc.x), T(0.5) * (zm.y - zc.y)};
    const C2<T> y = {T(0.5) * (zm.y + zc.y), T(0.5) * (zc.x - zm.x)};
    zl[(size_t)(2 * p) * fstride + m] = x;
    if (2 * p + 1 < n_in) zl[(size_t)(2 * p + 1) * fstride + m] = y;
  }
}

// Forward z FFT of the input adjoints, times c_m -> Dbar[n_in][N_r][modes].
template <typename T, int NF>
__global__ void __launch_bounds__(kFftThreads)
k_zfwd_adj(Dims d, FftPlan pz, const C2<T> *__restrict__ Z, double2 *__restrict__ db,
           const TwT<T> *__restrict__ tw, int tm) {
  extern __shared__ __align__(16) unsigned char smem[];
  TwT<T> *tws = reinterpret_cast<TwT<T> *>(smem);
  C2<T> *buf = reinterpret_cast<C2<T> *>(tws + d.nz);
  int bx, j, f;
  xcd_block(bx, j, f);
  const int nz = d.nz, K = d.kmax, mz = d.mz;
  const int ls = lds_line<T>(nz);
  const int mt0 = bx * tm;
  const int nl = min(tm, d.mt - mt0);
  load_twiddles(tws, tw, nz);
  const C2<T> *in = Z + ((size_t)f * d.nr + j) * nz * d.mt;
  for (Walk2 w(threadIdx.x, blockDim.x, nl); w.r < nz; w.next()) {
    const int b = w.r;
    const int li = w.c;
    buf[li * ls + PD<T>(b)] = in[(size_t)b * d.mt + mt0 + li];
  }
  __syncthreads();
  fft_block<T, false, kMaxB, NF>(buf, nl, ls, pz, tws);
  const size_t plane = (size_t)d.nmodes;
  for (Walk2 w(threadIdx.x, blockDim.x, mz); w.r < nl; w.next()) {
    const int li = w.r;
    const int kk = w.c;
    const int m = mt0 + li;
    const int k = kk - K;
    const C2<T> v = buf[li * ls + PD<T>((k >= 0 ? k : nz + k))];
    const double cm = m == 0 ? 1.0 : 2.0;
    double2 o = make_double2(cm * (double)v.x, cm * (double)v.y);
    db[((size_t)f * d.nr + j) * plane + (size_t)m * mz + kk] = o;
  }
}

// ubar += D(u)^T dbar (transposes of the spectral curl/gradient) + buoyancy.
__global__ void k_derived_adj(Dims d, Grid g, const double2 *__restrict__ db,
                              const double2 *__restrict__ nb, double2 *__restrict__ ub) {
  const int md = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const int n = d.nr;
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  const double kap = (double)(kk - d.kmax) * d.kz;
  const double ri = g.rinv[j];
  const double mr = (double)m * ri;
  auto D = [&](int f) { return db[((size_t)f * n + j) * P + md]; };
  // (D1^T v)_j over the rows whose window holds j
  auto D1T = [&](int f) {
    double2 acc = make_double2(0.0, 0.0);
    const int lo = j - 8 < 0 ? 0 : j - 8;
    const int hi = j + 8 > n - 1 ? n - 1 : j + 8;
    for (int i = lo; i <= hi; ++i) {
      const int t = j - g.s[i];
      if (t >= 0 && t < kStencil) {
        const double w = g.d1[i * kStencil + t];
        const double2 v = db[((size_t)f * n + i) * P + md];
        acc.x = fma(w, v.x, acc.x);
        acc.y = fma(w, v.y, acc.y);
      }
    }
    return acc;
  };
  auto mul_i = [](double s, double2 v) { return make_double2(-s * v.y, s * v.x); };  // i s v
  auto add = [&](int f, double2 v) {
    double2 *p = ub + ((size_t)f * n + j) * P + md;
    p->x += v.x;
    p->y += v.y;
  };
  const double2 d0 = D(0), d1 = D(1), d2 = D(2), d3 = D(3), d4 = D(4), d5 = D(5);
  const double2 a4 = mul_i(-kap, d4), a5 = mul_i(mr, d5);
  add(0, make_double2(d0.x + a4.x + a5.x, d0.y + a4.y + a5.y));
  const double2 b3 = mul_i(kap, d3), t5 = D1T(5);
  add(1, make_double2(d1.x + b3.x + t5.x + ri * d5.x, d1.y + b3.y + t5.y + ri * d5.y));
  const double2 c3 = mul_i(-mr, d3), t4 = D1T(4);
  add(2, make_double2(d2.x + c3.x - t4.x, d2.y + c3.y - t4.y));
  if (d.heated) {
    const double2 t6 = D1T(6), e7 = mul_i(-mr, D(7)), e8 = mul_i(-kap, D(8));
    auto NB = [&](int fo) {
      double2 a = nb[((size_t)fo * n + j) * P + md];
      if (md < d.mz) {
        const double2 w = nb[((size_t)fo * n + j) * P + (d.mz - 1 - md)];
        a = make_double2(0.5 * (a.x + w.x), 0.5 * (a.y - w.y));
      }
      return a;
    };
    const double2 nz = NB(2);
    add(3, make_double2(t6.x + e7.x + e8.x + d.gr * nz.x, t6.y + e7.y + e8.y + d.gr * nz.y));
  }
}

int min_radix(const FftPlan &p) { return p.min_radix; }

// Padded LDS line length for element size esize (bytes of one complex value).
int line_len(int n, size_t esize) { return esize == 8 ? lds_line<float>(n) : lds_line<double>(n); }

// Threads so that nlines * n / min_radix butterflies fit kMaxB per thread,
// capped at the FFT kernels' launch bound (then lines go in groups).
int block_for(const FftPlan &p, int nlines, int floor_threads) {
  const int bf = nlines * p.n / min_radix(p);
  int t = (bf + kMaxB - 1) / kMaxB;
  t = ((t + 63) / 64) * 64;
  if (t < floor_threads) t = floor_threads;
  if (t > kFftThreads) t = kFftThreads;
  return t;
}

// Lines per block for the z passes: LDS budget and butterfly budget.
int z_lines(const nsc_ctx *c, size_t esize) {
  const size_t budget = (size_t)c->lds_max - (size_t)c->d.nz * 16;  // twiddle entries
  int tm = (int)(budget / ((size_t)line_len(c->d.nz, esize) * esize));
  // at most 8 lines, a power of two: the transposed accesses (tm consecutive
  // theta modes of each z row) then stay within aligned 64- or 128-byte
  // segments, and smaller tiles let more workgroups share a compute unit
  // (11-line tiles of the 1536-point FP32 lines, 88-byte segments across
  // cache-line boundaries, took 29 % longer in the z-inverse pass; 16-line
  // tiles of 768-point lines, one workgroup per CU, 3 % and 11 % longer in
  // the FP32 z passes)
  if (tm > 8) tm = 8;
  if (tm > 1) tm = 1 << (31 - __builtin_clz((unsigned)tm));
  if (tm > c->d.mt) tm = c->d.mt;
  if (tm < 1) tm = 1;
  return tm;
}

// Threads of a z-pass workgroup of tm lines: with a wavefront-scope plan,
// wavefronts of up to four lines each; otherwise the block-scope rule.
int z_threads(const FftPlan &p, int tm) {
  if (p.wave_lines > 0) {
    const int per = p.wave_lines < 4 ? p.wave_lines : 4;
    int nw = (tm + per - 1) / per;
    if (nw > kFftThreads / 64) nw = kFftThreads / 64;
    return 64 * nw;
  }
  return block_for(p, tm, 256);
}

// Theta-pass launch shape: wavefront-scope sets when a wavefront can carry
// at least two lines per stage and a set's lines fit a modest LDS share,
// else one set per workgroup.
struct ThetaLaunch {
  bool wave;
  int waves;      // sets per workgroup (wave mode)
  dim3 grid;
  int threads;
  size_t shm;
};

ThetaLaunch theta_launch(const nsc_ctx *c, int nlines, size_t esize, bool one_line = false) {
  ThetaLaunch L;
  const size_t line = (size_t)line_len(c->d.nt, esize) * esize;
  const size_t tws = (size_t)c->d.nt * 16;  // 16-byte twiddle entries in both precisions
  const int nsets = c->d.nz * c->d.nr;
  // wavefront scope: lines that fit a wavefront's registers two at a time
  // and a line set of at most 24 KB; one_line: also one line at a time and
  // any line set the LDS holds (768-point lines: measured faster than the
  // workgroup-scope stages)
  L.wave = one_line ? (c->plan_t.wave_lines >= 1 && (size_t)nlines * line + tws <= (size_t)c->lds_max)
                    : (c->plan_t.wave_lines >= 2 && (size_t)nlines * line <= 24 * 1024);
  if (L.wave) {
    int w = (int)(((size_t)c->lds_max - tws) / ((size_t)nlines * line));
    if (w > 4) w = 4;
    if (w < 1) w = 1;
    L.waves = w;
    L.grid = dim3((nsets + w - 1) / w);
    L.threads = 64 * w;
    L.shm = tws + (size_t)w * nlines * line;
  } else {
    L.waves = 1;
    L.grid = dim3(c->d.nz, c->d.nr);
    L.threads = block_for(c->plan_t, nlines, 256);
    L.shm = tws + (size_t)nlines * line;
  }
  return L;
}

// Transform lengths with compile-time kernels (the padded grids of the
// configured workloads: 3 x 16, 32, 64 and 256 modes; with LONG also 3 x 512,
// whose lines the runtime plan can only transform at workgroup scope); others
// run the runtime-length stages.  f receives std::integral_constant<int, NF>.
template <bool LONG = false, class F>
hipError_t with_fixed_len(int n, bool allow, F f) {
  if (allow) {
    switch (n) {
      case 48: return f(std::integral_constant<int, 48>{});
      case 96: return f(std::integral_constant<int, 96>{});
      case 192: return f(std::integral_constant<int, 192>{});
      case 768: return f(std::integral_constant<int, 768>{});
      default: break;
    }
  }
  if constexpr (LONG) {
    if (n == 1536) return f(std::integral_constant<int, 1536>{});
  }
  return f(std::integral_constant<int, 0>{});
}

template <typename T>
hipError_t zinv_impl(const nsc_ctx *c, const double *u, const T *tw) {
  const int tm = z_lines(c, sizeof(C2<T>));
  dim3 grid((c->d.mt + tm - 1) / tm, c->d.nr, c->n_in);
  const int threads = z_threads(c->plan_z, tm);
  const size_t shm = ((size_t)tm * lds_line<T>(c->d.nz) + tw_slots<T>(c->d.nz)) * sizeof(C2<T>);
  // FP32 1536-point lines: the fixed-length wavefront stages
  return with_fixed_len<sizeof(T) == 4>(c->d.nz, c->plan_z.wave_lines > 0, [&](auto nf) {
    constexpr int NF = decltype(nf)::value;
    auto kern = c->d.pipe ? k_zinv<T, NF, true> : k_zinv<T, NF, false>;
    hipLaunchKernelGGL(kern, grid, dim3(threads), shm, c->stream, c->d, c->g, c->plan_z,
                       reinterpret_cast<const double2 *>(u), reinterpret_cast<C2<T> *>(c->zbuf),
                       reinterpret_cast<const TwT<T> *>(tw), tm, 1, c->s_mean);
    return hipGetLastError();
  });
}

// Launch shape of the fixed-length theta kernel: G threads per line set,
// line pad period 2^SH, and the sets per workgroup that put the most line
// sets on a compute unit's LDS (up to 1024 threads); sets = 0 if one set
// does not fit.
struct FxLaunch {
  int sets;
  dim3 grid;
  size_t shm;
};

FxLaunch fx_launch(const nsc_ctx *c, size_t esize, int np, int G, int SH) {
  const int nt = c->d.nt;
  const size_t line = (size_t)(nt + (nt >> SH) + 1) * esize;
  const size_t tws = (size_t)nt * 16;
  FxLaunch L{0, dim3(1), 0};
  int best = 0;
  const int maxt = G == 64 ? kThetaWaveThreads : kFftThreads;  // the kernel's launch bound
  for (int s = 1; s * G <= maxt; ++s) {
    const size_t shm = tws + (size_t)s * np * line;
    if (shm > (size_t)c->lds_max) break;
    const int per_cu = (int)((size_t)c->lds_cu / shm) * s;
    if (per_cu > best) {
      best = per_cu;
      L.sets = s;
      L.shm = shm;
    }
  }
  if (L.sets > 0) {
    const int nsets = c->d.nz * c->d.nr;
    L.grid = dim3((nsets + L.sets - 1) / L.sets);
  }
  return L;
}

template <typename T, int N, int G, int SH>
hipError_t theta_fx(const nsc_ctx *c, const T *tw, int want_cfl, double dth, double dzs) {
  const bool heated = c->n_in > 6;
  const FxLaunch L = fx_launch(c, sizeof(C2<T>), heated ? 5 : 3, G, SH);
  if (L.sets == 0) return hipErrorInvalidValue;  // (callers check theta_fits first)
  auto kern = heated ? k_theta_fx<T, N, 9, G, SH> : k_theta_fx<T, N, 6, G, SH>;
  hipLaunchKernelGGL(kern, L.grid, dim3(L.sets * G), L.shm, c->stream, c->d, c->g,
                     reinterpret_cast<const C2<T> *>(c->zbuf), reinterpret_cast<C2<T> *>(c->wbuf),
                     reinterpret_cast<const TwT<T> *>(tw), dth, dzs, c->cfl_part, want_cfl,
                     c->s_mean);
  return hipGetLastError();
}

template <typename T>
hipError_t theta_impl(const nsc_ctx *c, const T *tw, int want_cfl) {
  const double dth = 2.0 * M_PI / c->d.nt;
  const double dzs = c->d.lz / c->d.nz;
  // fixed lengths: the pruned, fused-packing kernel, one wavefront per line
  // set for the short lines, a workgroup-scope group per set for the long
  switch (c->d.nt) {
    case 48: return theta_fx<T, 48, 64, 3>(c, tw, want_cfl, dth, dzs);
    case 96: return theta_fx<T, 96, 64, 3>(c, tw, want_cfl, dth, dzs);
    case 192: return theta_fx<T, 192, 64, 3>(c, tw, want_cfl, dth, dzs);
    case 768: return theta_fx<T, 768, 192, 3>(c, tw, want_cfl, dth, dzs);
    case 1536:
      if constexpr (sizeof(T) == 4) return theta_fx<T, 1536, 512, 5>(c, tw, want_cfl, dth, dzs);
      break;
    default: break;
  }
  // other lengths: the runtime-length stages
  const int npi = (c->n_in + 1) / 2;
  const ThetaLaunch L = theta_launch(c, npi, sizeof(C2<T>), true);
  auto kern = L.wave ? k_theta<T, true, 0> : k_theta<T, false, 0>;
  hipLaunchKernelGGL(kern, L.grid, dim3(L.threads), L.shm, c->stream, c->d, c->g, c->plan_t,
                     reinterpret_cast<const C2<T> *>(c->zbuf), reinterpret_cast<C2<T> *>(c->wbuf),
                     reinterpret_cast<const TwT<T> *>(tw), c->n_in, dth, dzs, c->cfl_part,
                     want_cfl, c->s_mean);
  return hipGetLastError();
}

// Launch parameters (G, SH) of the fixed-length theta kernel for the padded
// length nt at the given precision; false where the runtime-length kernel runs.
bool theta_fixed(int nt, bool fp32, int *G, int *SH) {
  switch (nt) {
    case 48: case 96: case 192: *G = 64; *SH = 3; return true;
    case 768: *G = 192; *SH = 3; return true;
    case 1536: *G = 512; *SH = 5; return fp32;
    default: return false;
  }
}

template <typename T>
hipError_t zfwd_impl(const nsc_ctx *c, const double *u, double *nh, const T *tw, double *cfl_out,
                     double *cfl_host) {
  const int tm = z_lines(c, sizeof(C2<T>));
  dim3 grid((c->d.mt + tm - 1) / tm, c->d.nr, c->n_out);
  const int threads = z_threads(c->plan_z, tm);
  const size_t shm = ((size_t)tm * lds_line<T>(c->d.nz) + tw_slots<T>(c->d.nz)) * sizeof(C2<T>);
  const double scale = 1.0 / ((double)c->d.nt * (double)c->d.nz);
  return with_fixed_len<sizeof(T) == 4>(c->d.nz, c->plan_z.wave_lines > 0, [&](auto nf) {
    hipLaunchKernelGGL((k_zfwd<T, decltype(nf)::value>), grid, dim3(threads), shm, c->stream,
                       c->d, c->g, c->plan_z, reinterpret_cast<const C2<T> *>(c->wbuf),
                       reinterpret_cast<const double2 *>(u), reinterpret_cast<double2 *>(nh),
                       reinterpret_cast<const TwT<T> *>(tw), tm, scale, c->s_mean, c->cfl_part,
                       c->cfl_nblk, cfl_out, cfl_host);
    return hipGetLastError();
  });
}


template <typename T>
hipError_t nonlinear_vjp_impl(const nsc_ctx *c, const double *u, const double *nbar, double *ubar,
                              const T *twz, const T *twt) {
  const int tm = z_lines(c, sizeof(C2<T>));
  const int zthreads = z_threads(c->plan_z, tm);
  const size_t zshm = ((size_t)tm * lds_line<T>(c->d.nz) + tw_slots<T>(c->d.nz)) * sizeof(C2<T>);
  // forward fields on the (r, theta-spectral, z-physical) grid
  const dim3 gin((c->d.mt + tm - 1) / tm, c->d.nr, c->n_in);
  const dim3 gout((c->d.mt + tm - 1) / tm, c->d.nr, c->n_out);
  const double scale = 1.0 / ((double)c->d.nt * (double)c->d.nz);
  hipError_t e = with_fixed_len(c->d.nz, c->plan_z.wave_lines > 0, [&](auto nf) {
    constexpr int NF = decltype(nf)::value;
    hipLaunchKernelGGL((k_zinv<T, NF>), gin, dim3(zthreads), zshm, c->stream, c->d, c->g,
                       c->plan_z, reinterpret_cast<const double2 *>(u),
                       reinterpret_cast<C2<T> *>(c->zbuf), reinterpret_cast<const TwT<T> *>(twz),
                       tm, 0, c->s_mean);
    hipLaunchKernelGGL((k_zinv_adj<T, NF>), gout, dim3(zthreads), zshm, c->stream, c->d,
                       c->plan_z, reinterpret_cast<const double2 *>(nbar),
                       reinterpret_cast<C2<T> *>(c->wbuf), reinterpret_cast<const TwT<T> *>(twz),
                       tm, scale);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  const int npi = (c->n_in + 1) / 2;
  const ThetaLaunch L = theta_launch(c, npi + 2, sizeof(C2<T>));
  e = with_fixed_len(c->d.nt, L.wave, [&](auto nf) {
    constexpr int NF = decltype(nf)::value;
    auto tkern = L.wave ? k_theta_adj<T, true, NF> : k_theta_adj<T, false, 0>;
    hipLaunchKernelGGL(tkern, L.grid, dim3(L.threads), L.shm, c->stream, c->d, c->plan_t,
                       reinterpret_cast<C2<T> *>(c->zbuf),
                       reinterpret_cast<const C2<T> *>(c->wbuf),
                       reinterpret_cast<const TwT<T> *>(twt), c->n_in, c->n_out);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  e = with_fixed_len(c->d.nz, c->plan_z.wave_lines > 0, [&](auto nf) {
    hipLaunchKernelGGL((k_zfwd_adj<T, decltype(nf)::value>), gin, dim3(zthreads), zshm,
                       c->stream, c->d, c->plan_z, reinterpret_cast<const C2<T> *>(c->zbuf),
                       reinterpret_cast<double2 *>(c->s_adj),
                       reinterpret_cast<const TwT<T> *>(twz), tm);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_derived_adj, dim3((c->d.nmodes + 255) / 256, c->d.nr), dim3(256), 0, c->stream,
                     c->d, c->g, reinterpret_cast<const double2 *>(c->s_adj),
                     reinterpret_cast<const double2 *>(nbar), reinterpret_cast<double2 *>(ubar));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_zinv(const nsc_ctx *c, int prec, const double *u) {
  if (prec == NSC_MIXED) return zinv_impl<float>(c, u, c->tw32_z);
  return zinv_impl<double>(c, u, c->tw64_z);
}

bool theta_fits(const nsc_ctx *c, int prec, int adjoint) {
  const int npi = (c->n_in + 1) / 2;
  const size_t esize = prec == NSC_MIXED ? sizeof(C2<float>) : sizeof(C2<double>);
  int G, SH;
  if (!adjoint && theta_fixed(c->d.nt, prec == NSC_MIXED, &G, &SH))
    return fx_launch(c, esize, npi, G, SH).sets > 0;
  return theta_launch(c, adjoint ? npi + 2 : npi, esize, !adjoint).shm <= (size_t)c->lds_max;
}

hipError_t launch_theta(const nsc_ctx *c, int prec, int want_cfl) {
  if (prec == NSC_MIXED) return theta_impl<float>(c, c->tw32_t, want_cfl);
  return theta_impl<double>(c, c->tw64_t, want_cfl);
}

hipError_t launch_zfwd(const nsc_ctx *c, int prec, const double *u, double *n_hat, double *cfl_out,
                       double *cfl_host) {
  if (prec == NSC_MIXED) return zfwd_impl<float>(c, u, n_hat, c->tw32_z, cfl_out, cfl_host);
  return zfwd_impl<double>(c, u, n_hat, c->tw64_z, cfl_out, cfl_host);
}

hipError_t launch_nonlinear_vjp(const nsc_ctx *c, int prec, const double *u, const double *nbar,
                                double *ubar) {
  if (prec == NSC_MIXED) return nonlinear_vjp_impl<float>(c, u, nbar, ubar, c->tw32_z, c->tw32_t);
  return nonlinear_vjp_impl<double>(c, u, nbar, ubar, c->tw64_z, c->tw64_t);
}

}  // namespace nsc
