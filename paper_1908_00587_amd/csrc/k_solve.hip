// Per-Fourier-mode radial solves on gfx950 (section 2.2 of the nsCouette
// paper: the linear terms are independent per mode).  All FP64.
//
// Operators (q = azimuthal order of the family, kappa = k kz):
//   L_q = D2 + R^-1 D1 - q^2 R^-2 - kappa^2 I  (nine-point rows)
//   Helmholtz  H = alpha I - beta L_q, identity (Dirichlet) wall rows;
//   Poisson    L_q with D1 (Neumann) wall rows;
//   mean head  (D2 + D1/r) rows, p(r_i) = 0 in row 0, D1 row at r_o.
// Factors: LU without pivoting (growth factor < 1 on these operators), kept
// in the matrix envelope: row j stores L_{j,j-4..j-1}, 1/U_jj, U_{j,j+1..j+4}
// plus the wider one-sided rows 0..3 (U up to column 8) and N-4..N-1 (L from
// column N-9).  One thread per operator (factor) or per mode (solve); modes
// are laid out so that a wavefront's lanes read consecutive addresses.
#include <cfloat>

#include <type_traits>

#include "nsc_internal.h"

namespace nsc {
namespace {

__device__ __forceinline__ int edge_off(int t) { return t * 4 - (t * (t - 1)) / 2; }

struct Cd {
  double x, y;
};
__device__ __forceinline__ Cd operator+(Cd a, Cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ Cd operator-(Cd a, Cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ Cd operator*(double s, Cd a) { return {s * a.x, s * a.y}; }
__device__ __forceinline__ Cd ci(Cd a) { return {-a.y, a.x}; }  // i * a
__device__ __forceinline__ Cd ld(const double2 *p) {
  double2 v = *p;
  return {v.x, v.y};
}
__device__ __forceinline__ void st(double2 *p, Cd v) { *p = make_double2(v.x, v.y); }
__device__ __forceinline__ Cd fmac(double w, Cd v, Cd acc) { return {fma(w, v.x, acc.x), fma(w, v.y, acc.y)}; }

// Matrix entry A[i][c] of an operator for c in the window of row i.  pipe:
// row 0 is an inner row (the axis is no boundary) and the derivative rows
// are those of the operator's parity (off: their element offset).
struct OpRow {
  int kind;
  double alpha, beta, q2, k2;
  int pipe, off;
  __device__ __forceinline__ void row(const Grid &g, int n, int i, double *a, int &s) const {
    s = g.s[i];
    const double *w1 = g.d1 + off + i * kStencil;
    const double *w2 = g.d2 + off + i * kStencil;
    const double ri = g.rinv[i];
    const bool inner_wall = i == 0 && !pipe;
    if (kind == OP_HELMHOLTZ) {
      if (inner_wall || i == n - 1) {
#pragma unroll
        for (int t = 0; t < kStencil; ++t) a[t] = (s + t == i) ? 1.0 : 0.0;
        return;
      }
#pragma unroll
      for (int t = 0; t < kStencil; ++t) {
        double v = -beta * (w2[t] + w1[t] * ri);
        if (s + t == i) v += alpha + beta * (q2 * ri * ri + k2);
        a[t] = v;
      }
    } else if (kind == OP_POISSON) {
      if (inner_wall || i == n - 1) {
#pragma unroll
        for (int t = 0; t < kStencil; ++t) a[t] = w1[t];
        return;
      }
#pragma unroll
      for (int t = 0; t < kStencil; ++t) {
        double v = w2[t] + w1[t] * ri;
        if (s + t == i) v -= q2 * ri * ri + k2;
        a[t] = v;
      }
    } else {  // mean pressure head: (D2 + D1/r) p inside, p(r_i) = 0, D1 row at r_o
              // (pipe: p = 0 at the wall, the axis no boundary)
      if (inner_wall || (pipe && i == n - 1)) {
#pragma unroll
        for (int t = 0; t < kStencil; ++t) a[t] = (s + t == i) ? 1.0 : 0.0;
        return;
      }
      if (i == n - 1) {
#pragma unroll
        for (int t = 0; t < kStencil; ++t) a[t] = w1[t];
        return;
      }
#pragma unroll
      for (int t = 0; t < kStencil; ++t) a[t] = w2[t] + w1[t] * ri;
    }
  }
};

constexpr int kBW = 17;  // band window width: columns i-8 .. i+8
constexpr int kFacThreads = 32;

// One thread per operator: op = q*(K+1) + |k|.  Band elimination without
// pivoting over a sliding 9-row window held in LDS.  blockIdx.y picks one of
// two operator sets of the same kind and shift (velocity and temperature
// Helmholtz operators differ only in beta): both factorise in one launch.
__global__ void __launch_bounds__(kFacThreads)
k_factor(Dims d, Grid g, Factors F0, Factors F1, int kind, double alpha, double beta0,
         double beta1, int q_off) {
  __shared__ double win[9 * kBW * kFacThreads];
  const Factors F = blockIdx.y == 0 ? F0 : F1;
  const double beta = blockIdx.y == 0 ? beta0 : beta1;
  const int tid = threadIdx.x;
  const int op = blockIdx.x * kFacThreads + tid;
  if (op >= F.nops) return;
  auto W = [&](int ring, int bi) -> double & { return win[(ring * kBW + bi) * kFacThreads + tid]; };
  const int n = d.nr;
  const int kp1 = d.kmax + 1;
  const int q = op / kp1 + q_off;
  const int ka = op - (op / kp1) * kp1;
  const double kap = (double)ka * d.kz;
  OpRow R{kind, alpha, beta, (double)q * (double)q, kap * kap, d.pipe, odd_off(g, q)};
  const size_t nops = F.nops;
  // the pure-Neumann Poisson operator of (q = 0, kappa = 0) is singular and
  // never used; its slot holds the mean pressure-head operator instead
  if (kind == OP_POISSON && q == 0 && ka == 0) R.kind = OP_MEAN_PRESSURE;
  auto store_row = [&](int i, const double *a, int s) {
    const int ring = i % 9;
    for (int bi = 0; bi < kBW; ++bi) W(ring, bi) = 0.0;
    for (int t = 0; t < kStencil; ++t) W(ring, s + t - i + 8) = a[t];
  };
  const int first = n < 9 ? n : 9;
  for (int i = 0; i < first; ++i) {
    double a[kStencil];
    int s;
    R.row(g, n, i, a, s);
    store_row(i, a, s);
  }
  // Elimination of column k from the B rows below the pivot over the B
  // columns to its right: every operand is read before any result is
  // written (the rows are distinct ring slots), so the reads issue together.
  auto eliminate = [&](auto bsz, int rk, double dinv) {
    constexpr int B = decltype(bsz)::value;
    double pk[B], lv[B], rw[B][B];
#pragma unroll
    for (int t = 0; t < B; ++t) pk[t] = W(rk, 9 + t);
#pragma unroll
    for (int r = 1; r <= B; ++r) {
      const int ri = rk + r < 9 ? rk + r : rk + r - 9;
      lv[r - 1] = W(ri, 8 - r);
#pragma unroll
      for (int t = 1; t <= B; ++t) rw[r - 1][t - 1] = W(ri, 8 - r + t);
    }
#pragma unroll
    for (int r = 1; r <= B; ++r) {
      const int ri = rk + r < 9 ? rk + r : rk + r - 9;
      const double l = lv[r - 1] * dinv;
      W(ri, 8 - r) = l;
#pragma unroll
      for (int t = 1; t <= B; ++t) W(ri, 8 - r + t) = rw[r - 1][t - 1] - l * pk[t - 1];
    }
  };
  for (int k = 0; k < n; ++k) {
    // the row entering the window at the end of this step: its table reads
    // are issued first and consumed last
    double anx[kStencil];
    int snx = 0;
    const bool more = k + 9 < n;
    if (more) R.row(g, n, k + 9, anx, snx);
    const int rk = k % 9;
    const double dinv = 1.0 / W(rk, 8);
    // Rows k+5.. have no entry in column k and row k none right of k+4 when
    // the 9-point windows of rows k-4..k+8 are all centred; near the walls
    // the one-sided windows reach 8 rows and columns.  Columns past N-1 hold
    // zeros in every live row; ring slots of rows past N-1 hold rows already
    // written out, whose updates are never read.
    if (k >= 4 && more)
      eliminate(std::integral_constant<int, 4>{}, rk, dinv);
    else
      eliminate(std::integral_constant<int, 8>{}, rk, dinv);
    // row k is final
    double lo[4], up[4];
    for (int t = 1; t <= 4; ++t) {
      const int c = k - t;
      lo[4 - t] = c >= 0 ? W(rk, c - k + 8) : 0.0;
      const int cu = k + t;
      up[t - 1] = cu < n ? W(rk, cu - k + 8) : 0.0;
    }
    double *v = F.vals + (size_t)k * kSlots * nops + op;
    for (int t = 0; t < 4; ++t) {
      v[(size_t)t * nops] = lo[t];
      v[(size_t)(5 + t) * nops] = up[t];
    }
    v[(size_t)4 * nops] = dinv;
    if (F.pk) {
      auto at = [&](double *base, int row, int part) {
        return base + (((size_t)row * 2 + part) * nops + op) * 4;
      };
      for (int t = 0; t < 4; ++t) {
        at(F.pk, k, 0)[t] = lo[t];
        at(F.pk, k, 1)[t] = up[t];
      }
      // L(k, k - t) in column k - t, U(k, k + t) in column k + t
      if (F.pc)
        for (int t = 1; t <= 4; ++t) {
          if (k - t >= 0) at(F.pc, k - t, 0)[t - 1] = lo[4 - t];
          if (k + t < n) at(F.pc, k + t, 1)[t - 1] = up[t - 1];
        }
    }
    if (k <= 3)
      for (int c = k + 5; c <= 8 && c < n; ++c)
        F.edge[(size_t)(edge_off(k) + c - (k + 5)) * nops + op] = W(rk, c - k + 8);
    if (k >= n - 4) {
      const int t = n - 1 - k;
      for (int c = n - 9; c <= k - 5; ++c)
        if (c >= 0) F.edge[(size_t)(10 + edge_off(t) + c - (n - 9)) * nops + op] = W(rk, c - k + 8);
    }
    if (more) store_row(k + 9, anx, snx);
  }
}

// Forward/back substitution for one lane.  RHS(j) gives b_j, COL(j) the
// storage of y_j then x_j (LDS or global, read back by the same lane).  The
// bulk rows carry no branches: the envelope slots outside the matrix are
// stored as zeros, so every row issues the same independent loads and the
// compiler can schedule them ahead of the recurrence; only the one-sided
// wall rows (U to column 8 in rows 0..3, L from column N-9 in rows N-4..N-1)
// take the extra edge terms, in peeled loops.
template <typename V, int NR = 0, typename RHS, typename COL>
__device__ __forceinline__ void lu_solve(const Factors &F, int op, int nrt, RHS rhs, COL col) {
  // NR > 0: the row count is a compile-time constant and every loop unrolls
  // fully (COL may then name registers)
  const int n = NR > 0 ? NR : nrt;
  constexpr int kU = NR > 0 ? NR : 4;
  const size_t nops = F.nops;
  const double *__restrict__ vals = F.vals + op;
  const double *__restrict__ edge = F.edge + op;
  V y1{}, y2{}, y3{}, y4{};
#pragma unroll kU
  for (int j = 0; j < n - 4; ++j) {
    const double *v = vals + (size_t)j * kSlots * nops;
    const double l4 = v[0], l3 = v[nops], l2 = v[2 * nops], l1 = v[3 * nops];
    V y = rhs(j);
    y = y - l1 * y1;
    y = y - l2 * y2;
    y = y - l3 * y3;
    y = y - l4 * y4;
    y4 = y3;
    y3 = y2;
    y2 = y1;
    y1 = y;
    col(j) = y;
  }
#pragma unroll
  for (int j = n - 4; j < n; ++j) {
    const double *v = vals + (size_t)j * kSlots * nops;
    V y = rhs(j);
#pragma unroll
    for (int t = 1; t <= 4; ++t) y = y - v[(size_t)(4 - t) * nops] * col(j - t);
    const int tt = n - 1 - j;
#pragma unroll
    for (int c = n - 9; c <= j - 5; ++c) y = y - edge[(size_t)(10 + edge_off(tt) + c - (n - 9)) * nops] * col(c);
    col(j) = y;
  }
  V x1{}, x2{}, x3{}, x4{};
#pragma unroll kU
  for (int j = n - 1; j >= 4; --j) {
    const double *v = vals + (size_t)j * kSlots * nops;
    const double di = v[4 * nops], u1 = v[5 * nops], u2 = v[6 * nops], u3 = v[7 * nops], u4 = v[8 * nops];
    V x = col(j);
    x = x - u1 * x1;
    x = x - u2 * x2;
    x = x - u3 * x3;
    x = x - u4 * x4;
    x = di * x;
    x4 = x3;
    x3 = x2;
    x2 = x1;
    x1 = x;
    col(j) = x;
  }
#pragma unroll
  for (int j = 3; j >= 0; --j) {
    const double *v = vals + (size_t)j * kSlots * nops;
    V x = col(j);
#pragma unroll
    for (int t = 1; t <= 4; ++t) x = x - v[(size_t)(4 + t) * nops] * col(j + t);
#pragma unroll
    for (int c = j + 5; c <= 8; ++c) x = x - edge[(size_t)(edge_off(j) + c - (j + 5)) * nops] * col(c);
    col(j) = v[(size_t)4 * nops] * x;
  }
}

struct Rd {
  double v;
};
__device__ __forceinline__ Rd operator-(Rd a, Rd b) { return {a.v - b.v}; }
__device__ __forceinline__ Rd operator*(double s, Rd a) { return {s * a.v}; }

__device__ __forceinline__ double d1_row(const Grid &g, int j, const double *x, size_t stride,
                                        int off = 0) {
  const int s = g.s[j];
  const double *w = g.d1 + off + j * kStencil;
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < kStencil; ++t) acc = fma(w[t], x[(size_t)(s + t) * stride], acc);
  return acc;
}

// Homogeneous responses and inverse influence matrices per (m, |k|), in
// three passes: the pressure responses p_j (Neumann data e_0, e_{N-1}; do not
// depend on the step size, computed once), then the six velocity responses
// (X+, X-, h for each p_j) in parallel, then the 2x2 influence matrices.
__global__ void __launch_bounds__(64) k_influence_p(Dims d, Factors fp, Influence I) {
  const int op = blockIdx.x * blockDim.x + threadIdx.x;
  const int jj = blockIdx.y;  // 0: data at r_i, 1: at r_o
  if (op >= I.nops) return;
  const int n = d.nr;
  const int kp1 = d.kmax + 1;
  const int m = op / kp1;
  const int ka = op - m * kp1;
  const size_t ns = I.nops;
  double *Pj = I.resp + (size_t)jj * n * ns + op;
  if (m == 0 && ka == 0) {
    for (int j = 0; j < n; ++j) Pj[(size_t)j * ns] = 0.0;
    return;
  }
  const int wall = jj == 0 ? 0 : n - 1;
  lu_solve<Rd>(fp, op, n, [&](int j) { return Rd{j == wall ? 1.0 : 0.0}; },
               [&](int j) -> Rd & { return *reinterpret_cast<Rd *>(&Pj[(size_t)j * ns]); });
}

template <bool USE_LDS>
__global__ void __launch_bounds__(64) k_influence_x(Dims d, Grid g, Factors fv, Influence I) {
  extern __shared__ double inf_lds[];  // USE_LDS: [2][N_r][64] pressure and solution columns
  const int op = blockIdx.x * blockDim.x + threadIdx.x;
  const int jj = blockIdx.y;    // which pressure response
  const int kind = blockIdx.z;  // 0: X+, 1: X-, 2: h
  if (op >= I.nops) return;
  const int n = d.nr;
  const int kp1 = d.kmax + 1;
  const int m = op / kp1;
  const int ka = op - m * kp1;
  const size_t ns = I.nops;
  double *out = I.resp + (size_t)(2 + 2 * kind + jj) * n * ns + op;
  if (m == 0 && ka == 0) {
    for (int j = 0; j < n; ++j) out[(size_t)j * ns] = 0.0;
    return;
  }
  const double mm = (double)m;
  const double *Pj = I.resp + (size_t)jj * n * ns + op;
  const int q = kind == 0 ? m + 1 : (kind == 1 ? (m >= 1 ? m - 1 : 1 - m) : m);
  // X+ = H_{m+1}^-1 (-(D1 p - m p / r)), X- = H_{|m-1|}^-1 (-(D1 p + m p / r)),
  // h = H_m^-1 p so that X_z = -i kappa h
  auto rhs = [&](int j, const double *p, size_t stride) {
    if ((j == 0 && !d.pipe) || j == n - 1) return Rd{0.0};
    const double pj = p[(size_t)j * stride];
    if (kind == 2) return Rd{pj};
    const double dp = d1_row(g, j, p, stride, odd_off(g, m));  // p of order m
    const double mp = mm * g.rinv[j] * pj;
    return Rd{kind == 0 ? -(dp - mp) : -(dp + mp)};
  };
  if constexpr (USE_LDS) {
    // each lane owns one pressure column and one solution column in LDS (no
    // sharing, so no barrier): the back substitution and the stencil reads
    // stay on chip
    double *pl = inf_lds + threadIdx.x;
    double *xl = inf_lds + (size_t)n * 64 + threadIdx.x;
#pragma unroll 8
    for (int j = 0; j < n; ++j) pl[j * 64] = Pj[(size_t)j * ns];
    lu_solve<Rd>(fv, q * kp1 + ka, n, [&](int j) { return rhs(j, pl, 64); },
                 [&](int j) -> Rd & { return *reinterpret_cast<Rd *>(&xl[j * 64]); });
#pragma unroll 8
    for (int j = 0; j < n; ++j) out[(size_t)j * ns] = xl[j * 64];
  } else {
    lu_solve<Rd>(fv, q * kp1 + ka, n, [&](int j) { return rhs(j, Pj, ns); },
                 [&](int j) -> Rd & { return *reinterpret_cast<Rd *>(&out[(size_t)j * ns]); });
  }
}

__global__ void __launch_bounds__(64) k_influence_a(Dims d, Grid g, Influence I) {
  const int op = blockIdx.x * blockDim.x + threadIdx.x;
  if (op >= I.nops) return;
  const int n = d.nr;
  const int kp1 = d.kmax + 1;
  const int m = op / kp1;
  const int ka = op - m * kp1;
  const size_t ns = I.nops;
  if (m == 0 && ka == 0) {
    for (int e = 0; e < 4; ++e) I.ainv[(size_t)e * ns + op] = 0.0;
    return;
  }
  const double mm = (double)m;
  // A[w][jj] = wall divergence of response jj (walls carry zero velocity)
  double A[2][2];
  const int off = odd_off(g, m + 1);  // X+- of orders m +- 1
  for (int jj = 0; jj < 2; ++jj) {
    const double *Xp = I.resp + (size_t)(2 + jj) * n * ns + op;
    const double *Xm = I.resp + (size_t)(4 + jj) * n * ns + op;
    for (int w = 0; w < 2; ++w) {
      const int j = w == 0 ? 0 : n - 1;
      const double ri = g.rinv[j];
      A[w][jj] = 0.5 * ((d1_row(g, j, Xp, ns, off) + (1.0 + mm) * ri * Xp[(size_t)j * ns]) +
                        (d1_row(g, j, Xm, ns, off) + (1.0 - mm) * ri * Xm[(size_t)j * ns]));
    }
  }
  if (d.pipe) {
    // one wall: the first condition becomes lambda_1 = 0 (k_influence gives
    // it a zero right side), the second is the wall's
    A[0][0] = 1.0;
    A[0][1] = 0.0;
  }
  const double det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
  I.ainv[0 * ns + op] = A[1][1] / det;
  I.ainv[1 * ns + op] = -A[0][1] / det;
  I.ainv[2 * ns + op] = -A[1][0] / det;
  I.ainv[3 * ns + op] = A[0][0] / det;
}

// Nine-point stencil sums over R consecutive rows j0 .. j0+nrow-1 of NF
// fields (field f at x + f * fstride, rows strided by P), with the weights w
// ([N_r][9], row j's window starting at s_j): acc[f][jj] = sum_t
// w[j][t] x_f[s_j + t], summed from the left as a single row would, and
// cen[f][jj] = x_f[j].  The rows the windows share are read once: R + 8 rows
// when every window is centred, from the first window's start to the last
// window's end otherwise.
template <int R, int NF>
__device__ __forceinline__ void stencil_rows(const Grid &g, const double *__restrict__ w, int n,
                                             int j0, int nrow, const double2 *x, size_t fstride,
                                             size_t P, Cd (&acc)[NF][R], Cd (&cen)[NF][R]) {
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int jj = 0; jj < R; ++jj) acc[f][jj] = cen[f][jj] = Cd{0, 0};
  if (j0 >= 4 && j0 + R - 1 <= n - 5) {
    // row j0+jj reads rows j0+jj-4 .. j0+jj+4
#pragma unroll
    for (int rr = 0; rr < R + kStencil - 1; ++rr) {
      const size_t r = (size_t)(j0 - 4 + rr);
      Cd xv[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) xv[f] = ld(x + f * fstride + r * P);
#pragma unroll
      for (int jj = 0; jj < R; ++jj) {
        const int t = rr - jj;
        if (t >= 0 && t < kStencil) {
          const double wt = w[(j0 + jj) * kStencil + t];
#pragma unroll
          for (int f = 0; f < NF; ++f) acc[f][jj] = fmac(wt, xv[f], acc[f][jj]);
        }
        if (t == 4)
#pragma unroll
          for (int f = 0; f < NF; ++f) cen[f][jj] = xv[f];
      }
    }
  } else {
    const int lo = g.s[j0];
    const int hi = g.s[j0 + nrow - 1] + kStencil;
    for (int r = lo; r < hi; ++r) {
      Cd xv[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) xv[f] = ld(x + f * fstride + (size_t)r * P);
#pragma unroll
      for (int jj = 0; jj < R; ++jj) {
        const int j = j0 + jj;
        if (jj < nrow) {
          const int t = r - g.s[j];
          if (t >= 0 && t < kStencil) {
            const double wt = w[j * kStencil + t];
#pragma unroll
            for (int f = 0; f < NF; ++f) acc[f][jj] = fmac(wt, xv[f], acc[f][jj]);
          }
          if (r == j)
#pragma unroll
            for (int f = 0; f < NF; ++f) cen[f][jj] = xv[f];
        }
      }
    }
  }
}

// f_X = X^n/dt + (1-c) L_q X^n + c N^q + (1-c) N^n for X in {+, -, z, T}.
// blockIdx.z: 0 the +- pair (from u_r, u_theta), 1 u_z, 2 T -- one stencil
// family per thread keeps the registers (and so the occupancy) of a
// memory-bound kernel moderate.  blockIdx.y: a chunk of R rows per lane.
template <int R, bool PIPE = false>
__global__ void __launch_bounds__(256) k_rhs(Dims d, Grid g, const double2 *__restrict__ u,
                      const double2 *__restrict__ nn, const double2 *__restrict__ nq,
                      double2 *__restrict__ sf, double idt, double cc, int rows_first) {
  int bx, cy, part;
  stencil_block(rows_first, bx, cy, part);
  const int md = bx * blockDim.x + threadIdx.x;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const int n = d.nr;
  const int j0 = cy * R;
  const int nrow = n - j0 < R ? n - j0 : R;
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  const double kap = (double)(kk - d.kmax) * d.kz;
  const double ce = 1.0 - cc;
  const double k2 = kap * kap;
  const size_t fs = (size_t)n * P;  // field stride
  auto N = [&](int f, int j) -> Cd {
    if (!nn) return Cd{0, 0};
    const size_t o = ((size_t)f * n + j) * P + md;
    return cc * ld(nq + o) + ce * ld(nn + o);
  };
  if (part == 0) {
    // stencil sums of (D2 + D1/r) applied to u_r and u_theta (pipe: the
    // rows of parity (-1)^(m+1), per lane)
    Cd l[2][R], x[2][R];
    stencil_rows<R, 2>(g, PIPE ? g.lw + odd_off(g, m + 1) : g.lw, n, j0, nrow, u + md, fs, P, l, x);
    const double qp = (double)(m + 1), qm = (double)(m >= 1 ? m - 1 : 1 - m);
#pragma unroll
    for (int jj = 0; jj < R; ++jj) {
      if (jj >= nrow) break;
      const int j = j0 + jj;
      const double ri = g.rinv[j];
      const double r2 = ri * ri;
      const Cd lr = l[0][jj], lt = l[1][jj];
      const Cd ur = x[0][jj], ut = x[1][jj];
      const Cd xp = ur + ci(ut), xm = ur - ci(ut);
      const Cd lp = lr + ci(lt), lm = lr - ci(lt);
      const Cd Lp = lp - (qp * qp * r2 + k2) * xp;
      const Cd Lm = lm - (qm * qm * r2 + k2) * xm;
      const Cd a = N(0, j), b = N(1, j);
      st(sf + ((size_t)0 * n + j) * P + md, idt * xp + ce * Lp + (a + ci(b)));
      st(sf + ((size_t)1 * n + j) * P + md, idt * xm + ce * Lm + (a - ci(b)));
    }
  } else {
    // u_z (operator L_m) or T (L_m / Pr)
    const int f = part + 1;
    Cd l[1][R], x[1][R];
    stencil_rows<R, 1>(g, PIPE ? g.lw + odd_off(g, m) : g.lw, n, j0, nrow, u + f * fs + md, fs, P,
                       l, x);
    const double cf = f == 3 ? ce / d.pr : ce;
#pragma unroll
    for (int jj = 0; jj < R; ++jj) {
      if (jj >= nrow) break;
      const int j = j0 + jj;
      const double ri = g.rinv[j];
      const double r2 = ri * ri;
      const Cd Lx = l[0][jj] - ((double)m * (double)m * r2 + k2) * x[0][jj];
      st(sf + ((size_t)f * n + j) * P + md, idt * x[0][jj] + cf * Lx + N(f, j));
    }
  }
}

// ---------------------------------------------------------------------------
// Batched sweeps: one lane per (mode, system), the system's right side given
// column-wise in global memory (rows strided by the mode count).  The
// intermediate y and the solution x stay in LDS (64 lanes x N_r complex) so
// the two recurrences issue no global stores and the factor / right-side
// loads of later rows can be scheduled ahead; the solution is copied out at
// the end.  Columns longer than the LDS budget keep y in the output array.
// ---------------------------------------------------------------------------
// Fourth word of a raw buffer resource on CDNA (gfx9 family): 32-bit data
// format, no swizzle; with stride 0 the record count is a byte count and
// loads past it return zero.
constexpr int kBufferWord3 = 0x00020000;

// Raw buffer resource over `bytes` bytes of factor data at base, for the
// fully unrolled sweeps (NR > 0), whose factor arrays the host keeps below
// 2^31 bytes; the other variants never read through it and get an empty one.
template <int NR>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t sweep_rsrc(const double *base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(base), 0,
                                           NR > 0 ? (int)bytes : 0, kBufferWord3);
}

struct SweepSys {
  Factors F;
  int qmode;   // 0: q = m, 1: q = m + 1, 2: q = |m - 1|
  int zero00;  // 1: mode (0,0) writes zeros (else its operator slot is used)
  const double2 *in;  // right side column base, rows strided by the mode count
  double2 *out;       // solution column base
};
struct SweepArgs {
  SweepSys s[3];
};
constexpr int kSweepLanes = 64;

// factor rows in flight per sweep: fully unrolled sweeps (issued in that
// order by scheduling barriers; 16 or 20 rows measure the same), and runtime
// row counts
constexpr int kPfUnrolled = 12;
constexpr int kPfRuntime = 16;
constexpr int kPc = 4;  // column entries read ahead per sweep (divides the ring depths)
static_assert(kPfUnrolled % kPc == 0 && kPfRuntime % kPc == 0,
              "the column ring follows the factor ring");

// FAMILY only names the launch (0: pressure/temperature, 1: velocity), so
// that profiles tell the two apart; the code is the same.
// NR > 0: the number of radial points as a compile-time constant, so that
// the row loops unroll completely and the memory-wait counters can track
// each prefetched factor row individually (with a rolled loop the waits at
// the loop head drain every outstanding load).
template <bool USE_LDS, int FAMILY, int NR>
__global__ void __launch_bounds__(kSweepLanes)
k_sweep(Dims d, SweepArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cd *col = reinterpret_cast<Cd *>(smem);
  const int lane = threadIdx.x;
  // logical (mode tile, system) after the XCD remap, system fastest: the
  // two halves of a tile row (m, +-k) use the same operators, and the
  // systems of neighbouring rows share them (q = m - 1, m, m + 1), so these
  // workgroups run next to each other on one XCD and read the factors from
  // its L2 instead of HBM
  const int L = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int sys = L % gridDim.y;
  const int md = (L / gridDim.y) * kSweepLanes + lane;
  if (md >= d.nmodes) return;
  const SweepSys &S = a.s[sys];
  const size_t P = d.nmodes;
  const int n = NR > 0 ? NR : d.nr;
  constexpr int kUnrollCol = NR > 0 ? NR : 8;   // column copy
  constexpr int kUnrollRows = NR > 0 ? NR : 1;  // row groups of the sweeps
  constexpr int kPf = NR > 0 ? kPfUnrolled : kPfRuntime;
  const int kp1 = d.kmax + 1;
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  const int ka = kk >= d.kmax ? kk - d.kmax : d.kmax - kk;
  const double2 *__restrict__ b = S.in + md;
  double2 *__restrict__ x = S.out + md;
  // one factor set for the whole workgroup (its base stays in scalar
  // registers); mode (0,0) of the pressure uses slot 0 of the same set,
  // which holds the mean pressure-head operator
  const Factors F = S.F;
  const int q = S.qmode == 0 ? m : (S.qmode == 1 ? m + 1 : (m >= 1 ? m - 1 : 1 - m));
  const int op = q * kp1 + ka;
  if (m == 0 && ka == 0 && S.zero00) {
    for (int j = 0; j < n; ++j) x[(size_t)j * P] = make_double2(0.0, 0.0);
    return;
  }
  if (!USE_LDS) {
    lu_solve<Cd>(F, op, n, [&](int j) { return ld(b + (size_t)j * P); },
                 [&](int j) -> Cd & { return *reinterpret_cast<Cd *>(x + (size_t)j * P); });
    return;
  }
  const size_t nops = F.nops;
  const double *__restrict__ vals = F.vals + op;
  const double *__restrict__ edge = F.edge + op;
  auto C = [&](int j) -> Cd & { return col[j * kSweepLanes + lane]; };
  // Everything a row needs is requested well before the row: the factor
  // rows and the right side kPf rows ahead (registers), the column entries
  // kPc ahead (LDS reads), and the edge rows of both ends at the start.  The
  // right side enters with the factor rows rather than in a bulk copy before
  // the sweeps.  (The solution leaves in one copy at the end: stored row by
  // row during the back substitution, its stores fall under the same wait
  // counter as the prefetched loads and slowed the velocity sweeps.)  One
  // wavefront per workgroup: registers are plentiful, and the distance of
  // these requests is what hides the memory latency of the recurrences.
  const int nm = n - 4;
  // Fully unrolled sweeps read the factor rows as raw buffer loads: the
  // lane's operator offset in one 32-bit register, the row and slot offset
  // in a scalar register, so no 64-bit address is formed per load and the
  // registers go to rows in flight (the host picks this variant only while
  // the factor array spans less than 2^31 bytes).
  const __amdgpu_buffer_rsrc_t frs =
      sweep_rsrc<NR>(F.vals, (size_t)n * kSlots * nops * sizeof(double));
  const int voff = op * (int)sizeof(double);
  auto row = [&](int j, int sl) -> double {
    if constexpr (NR > 0)
      return __builtin_bit_cast(
          double, __builtin_amdgcn_raw_buffer_load_b64(
                      frs, voff, (int)(((size_t)j * kSlots + sl) * nops * sizeof(double)), 0));
    else
      return vals[((size_t)j * kSlots + sl) * nops];
  };
  // The four L entries (part 0) or the four off-diagonal U entries (part 1)
  // of row j into o[0..3].  Unrolled: two 16-byte loads from the row-packed
  // copy, so that a row costs three memory instructions with its right side
  // or its diagonal instead of five.
  const __amdgpu_buffer_rsrc_t prs = sweep_rsrc<NR>(F.pk, (size_t)n * 8 * nops * sizeof(double));
  const int poff = op * (int)(4 * sizeof(double));
  auto quad = [&](int j, int part, double *o) {
    if constexpr (NR > 0) {
      const int so = (int)(((size_t)j * 2 + part) * nops * 4 * sizeof(double));
      const double2 a = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(prs, poff, so, 0));
      const double2 c = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(prs, poff + 16, so, 0));
      o[0] = a.x;
      o[1] = a.y;
      o[2] = c.x;
      o[3] = c.y;
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) o[t] = row(j, part ? 5 + t : t);
    }
  };
  // last four rows (forward) and first four rows (backward): band entries
  // and the extra envelope entries, requested kPf rows before their use so
  // that they do not hold registers through the bulk of the sweeps
  double lt[4][4], le[10], ut[4][5], ue[10];
  auto load_tail = [&] {
#pragma unroll
    for (int r = 0; r < 4; ++r) quad(nm + r, 0, lt[r]);
#pragma unroll
    for (int e = 0; e < 10; ++e) le[e] = edge[(size_t)(10 + e) * nops];
  };
  auto load_head = [&] {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      ut[r][0] = row(r, 4);
      quad(r, 1, ut[r] + 1);
    }
#pragma unroll
    for (int e = 0; e < 10; ++e) ue[e] = edge[(size_t)e * nops];
  };
  // (runtime row counts: at the start of each sweep)
  const int tail_at = NR > 0 && nm - kPf > 0 ? nm - kPf : 0;          // forward row
  const int head_at = NR > 0 && 4 + kPf < n - 1 ? 4 + kPf : n - 1;    // backward row
  if (tail_at == 0) load_tail();
  // right sides of the last four rows (after the ring's reach)
  Cd rt[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) rt[r] = ld(b + (size_t)(nm + r) * P);
  double fa[kPf][4];
  Cd rb[kPf];
#pragma unroll
  for (int r = 0; r < kPf; ++r) {
    const int jj = r < nm ? r : nm - 1;
    quad(jj, 0, fa[r]);
    rb[r] = ld(b + (size_t)jj * P);
  }
  Cd y1{0, 0}, y2{0, 0}, y3{0, 0}, y4{0, 0};
#pragma unroll kUnrollRows
  for (int j0 = 0; j0 < nm; j0 += kPf) {
#pragma unroll
    for (int r = 0; r < kPf; ++r) {
      const int j = j0 + r;
      if (j == tail_at && j > 0) load_tail();
      if (j < nm) {
        // oldest terms first: the newest value y1 enters last, so the
        // row-to-row dependency is a single fused multiply-add
        Cd y = rb[r];  // right side of row j (j0 is a multiple of kPf)
        y = y - fa[r][0] * y4;
        y = y - fa[r][1] * y3;
        y = y - fa[r][2] * y2;
        y = y - fa[r][3] * y1;
        y4 = y3;
        y3 = y2;
        y2 = y1;
        y1 = y;
        C(j) = y;
      }
      const int jn = j + kPf < nm ? j + kPf : nm - 1;
      quad(jn, 0, fa[r]);
      rb[r] = ld(b + (size_t)jn * P);
      // keep the source order: the loads of row jn go out now, not next to
      // their use kPf rows later
      if constexpr (NR > 0) __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int j = nm + r;
    Cd y = rt[r];
#pragma unroll
    for (int t = 1; t <= 4; ++t) y = y - lt[r][4 - t] * C(j - t);
    const int tt = n - 1 - j;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c <= r) y = y - le[edge_off(tt) + c] * C(n - 9 + c);
    C(j) = y;
  }
  // back substitution over rows N-1..4
  if (head_at == n - 1) load_head();
  double u[kPf][5];
#pragma unroll
  for (int r = 0; r < kPf; ++r) {
    const int jj = n - 1 - r >= 4 ? n - 1 - r : 4;
    u[r][0] = row(jj, 4);
    quad(jj, 1, u[r] + 1);
  }
  Cd cb[kPc];
#pragma unroll
  for (int r = 0; r < kPc; ++r) cb[r] = C(n - 1 - r >= 4 ? n - 1 - r : 4);
  Cd x1{0, 0}, x2{0, 0}, x3{0, 0}, x4{0, 0};
#pragma unroll kUnrollRows
  for (int j0 = n - 1; j0 >= 4; j0 -= kPf) {
#pragma unroll
    for (int r = 0; r < kPf; ++r) {
      const int j = j0 - r;
      if (j == head_at && j < n - 1) load_head();
      if (j >= 4) {
        const int i = r % kPc;  // = (n - 1 - j) mod kPc
        Cd xv = cb[i];
        xv = xv - u[r][4] * x4;
        xv = xv - u[r][3] * x3;
        xv = xv - u[r][2] * x2;
        xv = xv - u[r][1] * x1;
        xv = u[r][0] * xv;
        x4 = x3;
        x3 = x2;
        x2 = x1;
        x1 = xv;
        C(j) = xv;
        // row j - kPc still holds the forward result (written downwards)
        const int jc = j - kPc >= 4 ? j - kPc : 4;
        cb[i] = C(jc);
      }
      const int jn = j - kPf >= 4 ? j - kPf : 4;
      u[r][0] = row(jn, 4);
      quad(jn, 1, u[r] + 1);
      // keep the source order: the loads of row jn go out now, not next to
      // their use kPf rows later
      if constexpr (NR > 0) __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int r = 3; r >= 0; --r) {
    Cd xv = C(r);
#pragma unroll
    for (int t = 1; t <= 4; ++t) xv = xv - ut[r][t] * C(r + t);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < 4 - r) xv = xv - ue[edge_off(r) + c] * C(r + 5 + c);
    C(r) = ut[r][0] * xv;
  }
#pragma unroll kUnrollCol
  for (int j = 0; j < n; ++j) st(x + (size_t)j * P, C(j));
}


// Velocity right sides in place of f: f_X - (grad p0)_X inside, wall values
// on rows 0 and N-1; mode (0,0) solves u_theta directly (X+- = +-i u_theta).
// R consecutive rows per lane (blockIdx.y: the chunk).
template <int R, bool PIPE = false>
__global__ void __launch_bounds__(256)
k_vel_rhs(Dims d, Grid g, double2 *__restrict__ sf, const double2 *__restrict__ sp, int walls,
          int rows_first) {
  int bx, cy, unused;
  stencil_block(rows_first, bx, cy, unused);
  const int md = bx * blockDim.x + threadIdx.x;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const int n = d.nr;
  const int j0 = cy * R;
  const int nrow = n - j0 < R ? n - j0 : R;
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  const bool zero = (md == d.kmax);
  auto field = [&](int f, int j) { return sf + ((size_t)f * n + j) * P + md; };
  auto wall_row = [&](int j) {
    Cd wp = {0, 0};
    if (zero && walls) {
      const double re = j == 0 ? d.re_i : d.re_o;
      wp = {0.0, re};
    }
    st(field(0, j), wp);
    st(field(1, j), Cd{-wp.x, -wp.y});
    st(field(2, j), Cd{0, 0});
  };
  if (zero) {
    for (int jj = 0; jj < nrow; ++jj) {
      const int j = j0 + jj;
      if ((j == 0 && !PIPE) || j == n - 1) {
        wall_row(j);
        continue;
      }
      const Cd h = 0.5 * (ld(field(0, j)) - ld(field(1, j)));
      st(field(0, j), h);
      st(field(1, j), Cd{-h.x, -h.y});
      // pipe: the driving pressure gradient in the axial mean flow
      if (PIPE && walls) st(field(2, j), ld(field(2, j)) + Cd{d.gp, 0.0});
    }
    return;
  }
  const double kap = (double)(kk - d.kmax) * d.kz;
  Cd dp[1][R], pc[1][R];
  stencil_rows<R, 1>(g, PIPE ? g.d1 + odd_off(g, m) : g.d1, n, j0, nrow, sp + md, 0, P, dp, pc);
#pragma unroll
  for (int jj = 0; jj < R; ++jj) {
    if (jj >= nrow) break;
    const int j = j0 + jj;
    if ((j == 0 && !PIPE) || j == n - 1) {
      wall_row(j);
      continue;
    }
    const Cd pj = pc[0][jj];
    const Cd mp = (m * g.rinv[j]) * pj;
    double2 *fp = field(0, j), *fm = field(1, j), *fz = field(2, j);
    st(fp, ld(fp) - (dp[0][jj] - mp));
    st(fm, ld(fm) - (dp[0][jj] + mp));
    st(fz, ld(fz) - kap * ci(pj));
  }
}

// Poisson right side g = mask(div f) at one (mode, row) where no divergence
// is formed: every row of mode (0,0), which takes the mean-head right side
// (D1 + 1/r) F_r inside and F_r(r_o) at the outer wall (zeros if not
// requested), and the wall rows of the other modes (zero).  Heated: the wall
// rows of f_T are replaced by the wall values (+-1/2 in (0,0), zero
// elsewhere; all zero for walls = 0) in the same pass.
__device__ __forceinline__ void div_row(const Dims &d, const Grid &g, double2 *__restrict__ sf,
                                        double2 *__restrict__ sg, const double2 *__restrict__ nn,
                                        const double2 *__restrict__ nq, double cc, int want_p,
                                        int walls, int md, int j) {
  const size_t P = d.nmodes;
  const int n = d.nr;
  if (d.heated && (j == 0 || j == n - 1)) {
    const bool mean = (md == d.kmax) && walls;
    st(sf + ((size_t)3 * n + j) * P + md, Cd{mean ? (j == 0 ? 0.5 : -0.5) : 0.0, 0.0});
  }
  if (md == d.kmax) {
    // (pipe: every row but the wall's, where p = 0; F_r odd in r)
    Cd r = {0, 0};
    if (want_p && nn && (j > 0 || d.pipe) && !(d.pipe && j == n - 1)) {
      auto Fr = [&](int t) {
        return cc * ld(nq + (size_t)t * P + md) + (1.0 - cc) * ld(nn + (size_t)t * P + md);
      };
      if (j == n - 1) {
        r = Fr(n - 1);
      } else {
        const int s0 = g.s[j];
        const double *w = g.d1 + g.podd + j * kStencil;
        r = g.rinv[j] * Fr(j);
        for (int t = 0; t < kStencil; ++t) r = fmac(w[t], Fr(s0 + t), r);
      }
    }
    st(sg + (size_t)j * P + md, r);
    return;
  }
  st(sg + (size_t)j * P + md, Cd{0, 0});  // wall rows of the other modes
}

// Poisson right side g = mask(div f) = (D1 + (1+m)/r) F_+ / 2 + (D1 + (1-m)/r)
// F_- / 2 + i kappa F_z over R consecutive rows per lane: the rows of F_+
// and F_- that the rows' nine-point windows share are read once (R + 8 rows
// for R outputs inside, fewer at the walls) instead of nine times, and each
// derivative still sums its window from the left, as a single row would.
template <int R, bool PIPE = false>
__global__ void __launch_bounds__(256)
k_div2(Dims d, Grid g, double2 *__restrict__ sf, double2 *__restrict__ sg,
       const double2 *__restrict__ nn, const double2 *__restrict__ nq, double cc, int want_p,
       int walls, int rows_first) {
  int bx, cy, unused;
  stencil_block(rows_first, bx, cy, unused);
  const int md = bx * blockDim.x + threadIdx.x;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const int n = d.nr;
  const int j0 = cy * R;
  const int nrow = n - j0 < R ? n - j0 : R;
  if (md == d.kmax) {
    for (int jj = 0; jj < nrow; ++jj) div_row(d, g, sf, sg, nn, nq, cc, want_p, walls, md, j0 + jj);
    return;
  }
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  const double kap = (double)(kk - d.kmax) * d.kz;
  const double2 *fz = sf + (size_t)2 * n * P + md;
  // D1 of F_+ and F_- (fields 0 and 1 of f)
  Cd dv[2][R], v[2][R];
  stencil_rows<R, 2>(g, PIPE ? g.d1 + odd_off(g, m + 1) : g.d1, n, j0, nrow, sf + md,
                     (size_t)n * P, P, dv, v);
#pragma unroll
  for (int jj = 0; jj < R; ++jj) {
    const int j = j0 + jj;
    if (jj >= nrow) break;
    if ((j == 0 && !PIPE) || j == n - 1) {
      div_row(d, g, sf, sg, nn, nq, cc, want_p, walls, md, j);
      continue;
    }
    const double ri = g.rinv[j];
    const Cd vz = ld(fz + (size_t)j * P);
    const Cd dp = dv[0][jj], dm = dv[1][jj], vp = v[0][jj], vm = v[1][jj];
    st(sg + (size_t)j * P + md,
       0.5 * ((dp + ((1.0 + m) * ri) * vp) + (dm + ((1.0 - m) * ri) * vm)) + kap * ci(vz));
  }
}

// lambda = -A^-1 beta(X0), beta = divergence at the two walls.
// One lane per mode, 64-lane workgroups (more of the chip for a small
// grid); the wall windows start at 0 and N-9, so all 38 loads of a lane are
// independent and issue together.
template <bool PIPE = false>
__global__ void __launch_bounds__(64) k_influence(Dims d, Grid g, Influence I,
                                                  const double2 *__restrict__ sx,
                                                  double2 *__restrict__ lam) {
  const int md = blockIdx.x * blockDim.x + threadIdx.x;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const int n = d.nr;
  const int kp1 = d.kmax + 1;
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  const int ka = kk >= d.kmax ? kk - d.kmax : d.kmax - kk;
  if (m == 0 && ka == 0) {
    st(lam + 2 * (size_t)md, Cd{0, 0});
    st(lam + 2 * (size_t)md + 1, Cd{0, 0});
    return;
  }
  const double kap = (double)(kk - d.kmax) * d.kz;
  const double mm = (double)m;
  const double2 *xp = sx + md, *xm = sx + (size_t)n * P + md, *xz = sx + (size_t)2 * n * P + md;
  Cd beta[2] = {Cd{0, 0}, Cd{0, 0}};
#pragma unroll
  for (int w = PIPE ? 1 : 0; w < 2; ++w) {  // (pipe: one wall, beta[0] = 0)
    const int j = w == 0 ? 0 : n - 1;
    const int s0 = w == 0 ? 0 : n - kStencil;  // one-sided wall window
    const double *wd = g.d1 + j * kStencil;
    if constexpr (PIPE) wd += odd_off(g, m + 1);
    const double ri = g.rinv[j];
    Cd dp = {0.0, 0.0}, dm = {0.0, 0.0};
#pragma unroll
    for (int t = 0; t < kStencil; ++t) {
      dp = fmac(wd[t], ld(xp + (size_t)(s0 + t) * P), dp);
      dm = fmac(wd[t], ld(xm + (size_t)(s0 + t) * P), dm);
    }
    beta[w] = 0.5 * ((dp + ((1.0 + mm) * ri) * ld(xp + (size_t)j * P)) +
                     (dm + ((1.0 - mm) * ri) * ld(xm + (size_t)j * P))) +
              kap * ci(ld(xz + (size_t)j * P));
  }
  const int op = m * kp1 + ka;
  const size_t ns = I.nops;
  const double a00 = I.ainv[op], a01 = I.ainv[ns + op], a10 = I.ainv[2 * ns + op], a11 = I.ainv[3 * ns + op];
  const Cd l1 = {-(a00 * beta[0].x + a01 * beta[1].x), -(a00 * beta[0].y + a01 * beta[1].y)};
  const Cd l2 = {-(a10 * beta[0].x + a11 * beta[1].x), -(a10 * beta[0].y + a11 * beta[1].y)};
  st(lam + 2 * (size_t)md, l1);
  st(lam + 2 * (size_t)md + 1, l2);
}

struct Vals {
  Cd ur, ut, uz, T, p;
};

// WITH_P: also the pressure (the step itself does not need it)
template <bool WITH_P = true>
__device__ __forceinline__ Vals final_value(const Dims &d, const Influence &I,
                                            const double2 *__restrict__ sx,
                                            const double2 *__restrict__ sp,
                                            const double2 *__restrict__ lam, int j, int md) {
  const size_t P = d.nmodes;
  const int n = d.nr;
  const int kp1 = d.kmax + 1;
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  const int ka = kk >= d.kmax ? kk - d.kmax : d.kmax - kk;
  Cd xp = ld(sx + (size_t)j * P + md);
  Cd xm = ld(sx + ((size_t)n + j) * P + md);
  Cd xz = ld(sx + ((size_t)2 * n + j) * P + md);
  Cd p = WITH_P ? ld(sp + (size_t)j * P + md) : Cd{0.0, 0.0};
  Vals v;
  if (!(m == 0 && ka == 0)) {
    const double kap = (double)(kk - d.kmax) * d.kz;
    const Cd l1 = ld(lam + 2 * (size_t)md), l2 = ld(lam + 2 * (size_t)md + 1);
    const size_t ns = I.nops;
    const int op = m * kp1 + ka;
    auto Rv = [&](int s) { return I.resp[((size_t)s * n + j) * ns + op]; };
    if (WITH_P) p = p + Rv(0) * l1 + Rv(1) * l2;
    xp = xp + Rv(2) * l1 + Rv(3) * l2;
    xm = xm + Rv(4) * l1 + Rv(5) * l2;
    // X_z,j = -i kappa h_j
    const Cd hz = Rv(6) * l1 + Rv(7) * l2;
    xz = xz - kap * ci(hz);
  }
  v.ur = 0.5 * (xp + xm);
  const Cd dd = xp - xm;  // u_theta = (X+ - X-) / (2 i)
  v.ut = {0.5 * dd.y, -0.5 * dd.x};
  v.uz = xz;
  v.T = d.heated ? ld(sx + ((size_t)3 * n + j) * P + md) : Cd{0, 0};
  v.p = p;
  return v;
}

template <bool WITH_P>
__global__ void __launch_bounds__(256)
k_finalize(Dims d, Influence I, const double2 *__restrict__ sx, const double2 *__restrict__ sp,
           const double2 *__restrict__ lam, double2 *__restrict__ out,
           double2 *__restrict__ pout) {
  constexpr int NV = WITH_P ? 5 : 4;
  __shared__ Cd xch[NV][256];
  const int md = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const size_t P = d.nmodes;
  const int n = d.nr;
  Vals v{}, w{};
  if (d.mz <= (int)blockDim.x && blockIdx.x == 0) {
    // the whole m = 0 column lies in this workgroup: its lanes take their
    // mirror mode's values from the lane that computes them, instead of
    // computing them a second time
    if (md < d.nmodes) v = final_value<WITH_P>(d, I, sx, sp, lam, j, md);
    if (md < d.mz) {
      xch[0][md] = v.ur;
      xch[1][md] = v.ut;
      xch[2][md] = v.uz;
      xch[3][md] = v.T;
      if (WITH_P) xch[NV - 1][md] = v.p;
    }
    __syncthreads();
    if (md >= d.nmodes) return;
    if (md < d.mz) {
      const int mk = d.mz - 1 - md;
      w = Vals{xch[0][mk], xch[1][mk], xch[2][mk], xch[3][mk],
               WITH_P ? xch[NV - 1][mk] : Cd{0, 0}};
    }
  } else {
    if (md >= d.nmodes) return;
    v = final_value<WITH_P>(d, I, sx, sp, lam, j, md);
    if (md < d.mz) w = final_value<WITH_P>(d, I, sx, sp, lam, j, d.mz - 1 - md);
  }
  if (md < d.mz) {  // m = 0: Hermitian projection
    auto h = [](Cd a, Cd b) { return Cd{0.5 * (a.x + b.x), 0.5 * (a.y - b.y)}; };
    v.ur = h(v.ur, w.ur);
    v.ut = h(v.ut, w.ut);
    v.uz = h(v.uz, w.uz);
    v.T = h(v.T, w.T);
    v.p = h(v.p, w.p);
  }
  st(out + ((size_t)0 * n + j) * P + md, v.ur);
  st(out + ((size_t)1 * n + j) * P + md, v.ut);
  st(out + ((size_t)2 * n + j) * P + md, v.uz);
  if (d.heated) st(out + ((size_t)3 * n + j) * P + md, v.T);
  if (WITH_P) st(pout + (size_t)j * P + md, v.p);
}

// Perturbation energy partial sums: w_j r_j c_m |u - U_b|^2 per block.
__global__ void k_energy_part(Dims d, Grid g, const double2 *__restrict__ u, double *__restrict__ part) {
  __shared__ double red[16];
  const size_t P = d.nmodes;
  const size_t total = (size_t)d.nr * P;
  double acc = 0.0;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / P);
    const int md = (int)(idx - (size_t)j * P);
    const int m = md / d.mz;
    double s = 0.0;
    for (int f = 0; f < 3; ++f) {
      double2 v = u[((size_t)f * d.nr + j) * P + md];
      if (f == 1 && md == d.kmax) v.x -= d.a_cou * g.r[j] + d.b_cou * g.rinv[j];
      s += v.x * v.x + v.y * v.y;
    }
    acc += (m == 0 ? 1.0 : 2.0) * g.ccw[j] * g.r[j] * s;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += red[w];
    part[blockIdx.x] = r;
  }
}

__global__ void k_energy_final(const double *__restrict__ part, int n, double scale, double *out) {
  __shared__ double red[16];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += red[w];
    out[0] = r * scale;
  }
}

// u~ = herm(amps) * g(r), g = 16 (r - r_i)^2 (r_o - r)^2.
__global__ void k_seed(Dims d, Grid g, const double2 *__restrict__ amps, double2 *__restrict__ out) {
  const int md = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int f = blockIdx.z;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  Cd a = ld(amps + (size_t)f * P + md);
  if (md < d.mz) {
    const Cd b = ld(amps + (size_t)f * P + (d.mz - 1 - md));
    a = {0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
  }
  if (md == d.kmax) a = {0, 0};
  const double r = g.r[j];
  if (d.pipe) {
    // u_+- = (a_r +- i a_theta) g_{m+-1}, u_z = a_z g_m, g_q = r^q (1 - r^2)^2
    // at peak one (regular at the axis); this lane writes component f
    const int m = md / d.mz;
    auto gq = [&](int q) {
      const double w = 1.0 - r * r;
      const double peak = q > 0 ? pow(q / (q + 4.0), 0.5 * q) * (16.0 / ((q + 4.0) * (q + 4.0))) : 1.0;
      return pow(r, (double)q) * w * w / peak;
    };
    Cd v;
    if (f == 2) {
      v = gq(m) * a;
    } else {
      // both in-plane amplitudes, the m = 0 column made Hermitian
      Cd ar = ld(amps + md), at = ld(amps + P + md);
      if (md < d.mz) {
        const int mm = d.mz - 1 - md;
        const Cd br = ld(amps + mm), bt = ld(amps + P + mm);
        ar = {0.5 * (ar.x + br.x), 0.5 * (ar.y - br.y)};
        at = {0.5 * (at.x + bt.x), 0.5 * (at.y - bt.y)};
      }
      if (md == d.kmax) ar = at = Cd{0, 0};
      const Cd up = gq(m + 1) * (ar + ci(at));
      const Cd um = gq(m >= 1 ? m - 1 : 1 - m) * (ar - ci(at));
      v = f == 0 ? 0.5 * (up + um) : Cd{0.5 * (up.y - um.y), -0.5 * (up.x - um.x)};
    }
    st(out + ((size_t)f * d.nr + j) * P + md, v);
    return;
  }
  const double s = 16.0 * (r - d.r_i) * (r - d.r_i) * (d.r_o - r) * (d.r_o - r);
  st(out + ((size_t)f * d.nr + j) * P + md, s * a);
}

// out += basic state; T: out_T = T_c delta_00 + u~_T (unprojected).
__global__ void k_add_base(Dims d, Grid g, const double2 *__restrict__ pert, double2 *__restrict__ out) {
  const int md = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const double r = g.r[j];
  if (md == d.kmax && d.pipe) {  // Hagen--Poiseuille flow Re (1 - r^2), Re = gp / 4
    double2 *p = out + ((size_t)2 * d.nr + j) * P + md;
    p->x += 0.25 * d.gp * (1.0 - r * r);
  } else if (md == d.kmax) {
    double2 *p = out + ((size_t)1 * d.nr + j) * P + md;
    p->x += d.a_cou * r + d.b_cou * g.rinv[j];
  }
  if (d.heated) {
    Cd t = ld(pert + ((size_t)3 * d.nr + j) * P + md);
    if (md == d.kmax) t.x += 0.5 + log(r / d.r_i) / log(d.r_i / d.r_o);
    st(out + ((size_t)3 * d.nr + j) * P + md, t);
  }
}

// ---------------------------------------------------------------------------
// Vector--Jacobian product of the implicit stage (discrete adjoint).  The
// stage is affine in (X^n, N^n, N^q); its linear part per mode is, in order,
//   f = X^n/dt + (1-c) L X^n + c N^q + (1-c) N^n   (+- basis)
//   g = mask(div f), p0 = P^-1 g, X0 = H^-1 mask(f - grad p0),
//   lambda = -A^-1 beta(X0), X = X0 + sum lambda_j X_j, herm(output).
// The adjoint applies the transposes in reverse order; complex-linear maps
// are conjugate-transposed (real factors transpose, i -> -i).
// ---------------------------------------------------------------------------

// A^T x = b with A = L U in envelope storage: U^T y = b (forward), then
// L^T x = y (backward).  Rows 0..8 of the forward pass and N-9..N-1 of the
// backward pass carry the one-sided edge entries and are peeled.
template <typename V, typename RHS, typename COL>
__device__ __forceinline__ void lu_solve_t(const Factors &F, int op, int n, RHS rhs, COL col) {
  const size_t nops = F.nops;
  const double *__restrict__ vals = F.vals + op;
  const double *__restrict__ edge = F.edge + op;
  auto Vv = [&](int row, int slot) { return vals[((size_t)row * kSlots + slot) * nops]; };
  for (int j = 0; j < 9; ++j) {
    V y = rhs(j);
    for (int t = 1; t <= 4; ++t)
      if (j - t >= 0) y = y - Vv(j - t, 4 + t) * col(j - t);
    for (int c = 0; c <= 3; ++c)
      if (j - c >= 5) y = y - edge[(size_t)(edge_off(c) + j - c - 5) * nops] * col(c);
    col(j) = Vv(j, 4) * y;
  }
  V y1 = col(8), y2 = col(7), y3 = col(6), y4 = col(5);
#pragma unroll 4
  for (int j = 9; j < n; ++j) {
    const double a1 = Vv(j - 1, 5), a2 = Vv(j - 2, 6), a3 = Vv(j - 3, 7), a4 = Vv(j - 4, 8), di = Vv(j, 4);
    V y = rhs(j);
    y = y - a1 * y1;
    y = y - a2 * y2;
    y = y - a3 * y3;
    y = y - a4 * y4;
    y = di * y;
    y4 = y3;
    y3 = y2;
    y2 = y1;
    y1 = y;
    col(j) = y;
  }
  for (int j = n - 1; j >= n - 9; --j) {
    V x = col(j);
    for (int t = 1; t <= 4; ++t)
      if (j + t < n) x = x - Vv(j + t, 4 - t) * col(j + t);
    for (int c = n - 4; c <= n - 1; ++c)
      if (c - j >= 5) x = x - edge[(size_t)(10 + edge_off(n - 1 - c) + j - (n - 9)) * nops] * col(c);
    col(j) = x;
  }
  V x1 = col(n - 9), x2 = col(n - 8), x3 = col(n - 7), x4 = col(n - 6);
#pragma unroll 4
  for (int j = n - 10; j >= 0; --j) {
    const double a1 = Vv(j + 1, 3), a2 = Vv(j + 2, 2), a3 = Vv(j + 3, 1), a4 = Vv(j + 4, 0);
    V x = col(j);
    x = x - a1 * x1;
    x = x - a2 * x2;
    x = x - a3 * x3;
    x = x - a4 * x4;
    x4 = x3;
    x3 = x2;
    x2 = x1;
    x1 = x;
    col(j) = x;
  }
}

// (W^T v)_j = sum_i W[i][j - s_i] v_i over the rows i whose window holds j.
__device__ __forceinline__ Cd wt_rowc(const Grid &g, const double *w, int n, int j,
                                      const double2 *v, size_t stride, bool scale_rinv) {
  Cd acc = {0, 0};
  const int lo = j - 8 < 0 ? 0 : j - 8;
  const int hi = j + 8 > n - 1 ? n - 1 : j + 8;
  for (int i = lo; i <= hi; ++i) {
    const int s = g.s[i];
    const int t = j - s;
    if (t >= 0 && t < kStencil) {
      double c = w[i * kStencil + t];
      if (scale_rinv) c *= g.rinv[i];
      acc = fmac(c, ld(v + (size_t)i * stride), acc);
    }
  }
  return acc;
}

// Output adjoint: Hermitian projection of u_bar, then the +- basis:
// Xbar+- = (ubar_r +- i ubar_theta)/2, Xbar_z = ubar_z, Tbar.  Mode (0,0)
// keeps ubar_theta in slot 0 (its u_theta is solved directly).
__global__ void k_adj_out(Dims d, const double2 *__restrict__ ub, double2 *__restrict__ sx) {
  const int md = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const int n = d.nr;
  auto U = [&](int f, int m2) { return ld(ub + ((size_t)f * n + j) * P + m2); };
  Cd v[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {  // (constant trip count: v stays in registers)
    if (f >= d.f) {
      v[f] = Cd{0, 0};
      continue;
    }
    v[f] = U(f, md);
    if (md < d.mz) {
      const Cd w = U(f, d.mz - 1 - md);
      v[f] = {0.5 * (v[f].x + w.x), 0.5 * (v[f].y - w.y)};
    }
  }
  if (md == d.kmax) {
    st(sx + ((size_t)0 * n + j) * P + md, v[1]);
    st(sx + ((size_t)1 * n + j) * P + md, Cd{0, 0});
  } else {
    st(sx + ((size_t)0 * n + j) * P + md, 0.5 * (v[0] + ci(v[1])));
    st(sx + ((size_t)1 * n + j) * P + md, 0.5 * (v[0] - ci(v[1])));
  }
  st(sx + ((size_t)2 * n + j) * P + md, v[2]);
  if (d.heated) st(sx + ((size_t)3 * n + j) * P + md, v[3]);
}

// lambda_bar_j = sum_r (X_j+ Xbar+ + X_j- Xbar- + i kappa h_j Xbar_z);
// beta_bar = -A^-T lambda_bar.  Workgroup of 64 modes x 16 row parts (a few
// rows per lane, so each lane's loads go out in one round); the parts'
// partial sums meet in LDS (fixed order).
constexpr int kLamModes = 64, kLamParts = 16;

__global__ void __launch_bounds__(kLamModes * kLamParts)
k_adj_lambda(Dims d, Influence I, const double2 *__restrict__ sx, double2 *__restrict__ bbar) {
  __shared__ Cd part[kLamParts - 1][2][kLamModes];
  const int lane = threadIdx.x % kLamModes, q = threadIdx.x / kLamModes;
  const int md = blockIdx.x * kLamModes + lane;
  const bool live = md < d.nmodes;
  const size_t P = d.nmodes;
  const int n = d.nr;
  const int kp1 = d.kmax + 1;
  const int m = live ? md / d.mz : 0;
  const int kk = live ? md - m * d.mz : d.kmax;
  const int ka = kk >= d.kmax ? kk - d.kmax : d.kmax - kk;
  const double kap = (double)(kk - d.kmax) * d.kz;
  const int op = m * kp1 + ka;
  const size_t ns = I.nops;
  Cd l1 = {0, 0}, l2 = {0, 0};
  const int j0 = (n * q) / kLamParts, j1 = (n * (q + 1)) / kLamParts;
  if (live) {
#pragma unroll 4
    for (int j = j0; j < j1; ++j) {
      const Cd xp = ld(sx + (size_t)j * P + md);
      const Cd xm = ld(sx + ((size_t)n + j) * P + md);
      const Cd xz = kap * ci(ld(sx + ((size_t)2 * n + j) * P + md));  // i kappa Xbar_z
      auto Rv = [&](int s) { return I.resp[((size_t)s * n + j) * ns + op]; };
      l1 = l1 + (Rv(2) * xp + Rv(4) * xm + Rv(6) * xz);
      l2 = l2 + (Rv(3) * xp + Rv(5) * xm + Rv(7) * xz);
    }
  }
  if (q > 0) {
    part[q - 1][0][lane] = l1;
    part[q - 1][1][lane] = l2;
  }
  __syncthreads();
  if (q != 0 || !live) return;
#pragma unroll
  for (int t = 0; t < kLamParts - 1; ++t) {
    l1 = l1 + part[t][0][lane];
    l2 = l2 + part[t][1][lane];
  }
  if (m == 0 && ka == 0) {
    st(bbar + 2 * (size_t)md, Cd{0, 0});
    st(bbar + 2 * (size_t)md + 1, Cd{0, 0});
    return;
  }
  const double a00 = I.ainv[op], a01 = I.ainv[ns + op], a10 = I.ainv[2 * ns + op], a11 = I.ainv[3 * ns + op];
  st(bbar + 2 * (size_t)md, Cd{-(a00 * l1.x + a10 * l2.x), -(a00 * l1.y + a10 * l2.y)});
  st(bbar + 2 * (size_t)md + 1, Cd{-(a01 * l1.x + a11 * l2.x), -(a01 * l1.y + a11 * l2.y)});
}

// Transposed Helmholtz sweeps: comp 0/1/2 velocity (+, -, z), 3 temperature.
// rbar = mask(H^-T (Xbar + beta terms)) -> sf[comp]; mode (0,0) is the
// direct u_theta / u_z problem.
__global__ void __launch_bounds__(256)
k_adj_vel(Dims d, Grid g, Factors fv, Factors ft, const double2 *__restrict__ sx,
          const double2 *__restrict__ bbar, double2 *__restrict__ sf) {
  const int md = blockIdx.x * blockDim.x + threadIdx.x;
  if (md >= d.nmodes) return;
  const int comp = blockIdx.y;
  const size_t P = d.nmodes;
  const int n = d.nr;
  const int kp1 = d.kmax + 1;
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  const int ka = kk >= d.kmax ? kk - d.kmax : d.kmax - kk;
  const double kap = (double)(kk - d.kmax) * d.kz;
  const bool zero = (m == 0 && ka == 0);
  const double2 *xb = sx + (size_t)comp * n * P + md;
  double2 *out = sf + (size_t)comp * n * P + md;
  auto outr = [&](int j) -> Cd & { return *reinterpret_cast<Cd *>(out + (size_t)j * P); };
  if (comp == 3) {
    lu_solve_t<Cd>(ft, m * kp1 + ka, n, [&](int j) { return ld(xb + (size_t)j * P); }, outr);
    outr(0) = Cd{0, 0};
    outr(n - 1) = Cd{0, 0};
    return;
  }
  if (zero) {
    if (comp == 1) return;
    const int q = comp == 0 ? 1 : 0;
    lu_solve_t<Cd>(fv, q * kp1 + ka, n, [&](int j) { return ld(xb + (size_t)j * P); }, outr);
    outr(0) = Cd{0, 0};
    outr(n - 1) = Cd{0, 0};
    if (comp == 0) {  // fbar+ = (i/2) rbar_theta, fbar- = -(i/2) rbar_theta
      double2 *om = sf + (size_t)n * P + md;
      for (int j = 0; j < n; ++j) {
        const Cd r = outr(j);
        const Cd h = 0.5 * ci(r);
        outr(j) = h;
        st(om + (size_t)j * P, Cd{-h.x, -h.y});
      }
    }
    return;
  }
  const int q = comp == 0 ? m + 1 : (comp == 1 ? (m >= 1 ? m - 1 : 1 - m) : m);
  const Cd b0 = ld(bbar + 2 * (size_t)md), b1 = ld(bbar + 2 * (size_t)md + 1);
  const double sgn = comp == 0 ? 1.0 : -1.0;
  auto rhs = [&](int j) -> Cd {
    Cd v = ld(xb + (size_t)j * P);
    if (comp < 2) {
      // 1/2 (D1 + (1 +- m)/r)^T e_w beta_bar_w
      if (j <= 8) {
        double c = g.d1[0 * kStencil + j];
        if (j == 0) c += (1.0 + sgn * m) * g.rinv[0];
        v = v + (0.5 * c) * b0;
      }
      if (j >= n - 9) {
        double c = g.d1[(n - 1) * kStencil + (j - g.s[n - 1])];
        if (j == n - 1) c += (1.0 + sgn * m) * g.rinv[n - 1];
        v = v + (0.5 * c) * b1;
      }
    } else {
      if (j == 0) v = v - kap * ci(b0);
      if (j == n - 1) v = v - kap * ci(b1);
    }
    return v;
  };
  lu_solve_t<Cd>(fv, q * kp1 + ka, n, rhs, outr);
  outr(0) = Cd{0, 0};
  outr(n - 1) = Cd{0, 0};
}

// ---------------------------------------------------------------------------
// Transposed sweeps with the column in LDS (one lane per (mode, system), 64
// lanes per workgroup): A^T x = b with A = LU, i.e. U^T y = b upwards, then
// L^T x = y downwards, in place in the lane's LDS column.  The boundary rows
// (0..8 and N-9..N-1, with the envelope entries) read their factors up
// front; the bulk rows read theirs kPfT rows ahead.
// ---------------------------------------------------------------------------
constexpr int kPfT = 8;

template <int NR, class COL>
__device__ __forceinline__ void sweep_t_lds(const Factors &F, int op, int nrt, COL C) {
  const int n = NR > 0 ? NR : nrt;
  constexpr int kUnrollRows = NR > 0 ? NR : 1;
  const size_t nops = F.nops;
  const double *__restrict__ vals = F.vals + op;
  const double *__restrict__ edge = F.edge + op;
  auto V = [&](int row, int slot) { return vals[((size_t)row * kSlots + slot) * nops]; };
  // Unrolled: raw buffer loads (operator offset in one 32-bit register, row
  // offset in a scalar register) of the packed rows (part 0: L row, 1: U
  // row) and columns (2: L below the diagonal, 3: U above it), two 16-byte
  // loads per part; else the compact rows.
  const size_t n8 = (size_t)n * nops * sizeof(double);
  const __amdgpu_buffer_rsrc_t rv = sweep_rsrc<NR>(F.vals, n8 * kSlots);
  const __amdgpu_buffer_rsrc_t rk = sweep_rsrc<NR>(F.pk, n8 * 8);
  const __amdgpu_buffer_rsrc_t rc = sweep_rsrc<NR>(F.pc, n8 * 8);
  const int o8 = op * (int)sizeof(double);
  auto dg = [&](int j) -> double {  // 1/U_jj
    if constexpr (NR > 0)
      return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                            rv, o8, (j * kSlots + 4) * (int)nops * 8, 0));
    else
      return V(j, 4);
  };
  auto quad = [&](int j, int part, double *o) {
    if constexpr (NR > 0) {
      const int so = (j * 2 + (part & 1)) * (int)nops * 32;
      const __amdgpu_buffer_rsrc_t r = part < 2 ? rk : rc;
      const double2 a = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, 4 * o8, so, 0));
      const double2 b = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, 4 * o8 + 16, so, 0));
      o[0] = a.x;
      o[1] = a.y;
      o[2] = b.x;
      o[3] = b.y;
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        o[t] = part == 0 ? V(j, t)
             : part == 1 ? V(j, 5 + t)
             : part == 2 ? V(j + t + 1, 3 - t)   // L(j + t + 1, j)
                         : V(j - t - 1, 5 + t);  // U(j - t - 1, j)
    }
  };
  // U^T y = b: rows 0..8 with the top envelope entries
  {
    double hu[9][5], he[10];
#pragma unroll
    for (int j = 0; j < 9; ++j) {  // U(j, j + t), t = 0 the inverse diagonal
      hu[j][0] = dg(j);
      quad(j, 1, hu[j] + 1);
    }
#pragma unroll
    for (int e = 0; e < 10; ++e) he[e] = edge[(size_t)e * nops];
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      Cd y = C(j);
#pragma unroll
      for (int t = 1; t <= 4; ++t)
        if (j - t >= 0) y = y - hu[j - t][t] * C(j - t);
#pragma unroll
      for (int c = 0; c <= 3; ++c)
        if (j - c >= 5) y = y - he[edge_off(c) + j - c - 5] * C(c);
      C(j) = hu[j][0] * y;
    }
  }
  {
    // bulk rows 9..N-1: the U column above row j (U(j - t, j) at t) and
    // 1/U_jj at 0
    double fa[kPfT][5];
#pragma unroll
    for (int r = 0; r < kPfT; ++r) {
      const int j = 9 + r < n ? 9 + r : n - 1;
      quad(j, 3, fa[r] + 1);
      fa[r][0] = dg(j);
    }
    Cd y1 = C(8), y2 = C(7), y3 = C(6), y4 = C(5);
#pragma unroll kUnrollRows
    for (int j0 = 9; j0 < n; j0 += kPfT) {
#pragma unroll
      for (int r = 0; r < kPfT; ++r) {
        const int j = j0 + r;
        if (j < n) {
          Cd y = C(j);
          y = y - fa[r][4] * y4;
          y = y - fa[r][3] * y3;
          y = y - fa[r][2] * y2;
          y = y - fa[r][1] * y1;
          y = fa[r][0] * y;
          y4 = y3;
          y3 = y2;
          y2 = y1;
          y1 = y;
          C(j) = y;
        }
        const int jn = j + kPfT < n ? j + kPfT : n - 1;
        quad(jn, 3, fa[r] + 1);
        fa[r][0] = dg(jn);
      }
    }
  }
  // L^T x = y: rows N-1..N-9 with the bottom envelope entries
  {
    double tl[9][4], te[10];
#pragma unroll
    for (int i = 0; i < 9; ++i) quad(n - 9 + i, 0, tl[i]);  // L(row, row - 4 + t)
#pragma unroll
    for (int e = 0; e < 10; ++e) te[e] = edge[(size_t)(10 + e) * nops];
#pragma unroll
    for (int i = 8; i >= 0; --i) {
      const int j = n - 9 + i;
      Cd x = C(j);
#pragma unroll
      for (int t = 1; t <= 4; ++t)
        if (i + t <= 8) x = x - tl[i + t][4 - t] * C(j + t);  // L(j + t, j)
#pragma unroll
      for (int ci = 5; ci <= 8; ++ci) {
        const int c = n - 9 + ci;  // rows N-4..N-1
        if (ci - i >= 5) x = x - te[edge_off(n - 1 - c) + j - (n - 9)] * C(c);
      }
      C(j) = x;
    }
  }
  {
    // bulk rows N-10..0: the L column below row j (L(j + t, j) at t)
    double fl[kPfT][5];
#pragma unroll
    for (int r = 0; r < kPfT; ++r) {
      const int j = n - 10 - r >= 0 ? n - 10 - r : 0;
      quad(j, 2, fl[r] + 1);
    }
    Cd x1 = C(n - 9), x2 = C(n - 8), x3 = C(n - 7), x4 = C(n - 6);
#pragma unroll kUnrollRows
    for (int j0 = n - 10; j0 >= 0; j0 -= kPfT) {
#pragma unroll
      for (int r = 0; r < kPfT; ++r) {
        const int j = j0 - r;
        if (j >= 0) {
          Cd x = C(j);
          x = x - fl[r][4] * x4;
          x = x - fl[r][3] * x3;
          x = x - fl[r][2] * x2;
          x = x - fl[r][1] * x1;
          x4 = x3;
          x3 = x2;
          x2 = x1;
          x1 = x;
          C(j) = x;
        }
        const int jn = j - kPfT >= 0 ? j - kPfT : 0;
        quad(jn, 2, fl[r] + 1);
      }
    }
  }
}

// k_adj_vel and k_adj_poisson with the LDS sweep: kind 0 the transposed
// Helmholtz problems (blockIdx.y: 0/1/2 velocity +, -, z; 3 temperature),
// kind 1 the transposed Poisson problem.  Same right sides and masks.
template <int NR>
__global__ void __launch_bounds__(kSweepLanes)
k_adj_sweep(Dims d, Grid g, Factors fv, Factors ft, Factors fp, int kind,
            const double2 *__restrict__ src, const double2 *__restrict__ bbar,
            double2 *__restrict__ dst) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cd *col = reinterpret_cast<Cd *>(smem);
  const int lane = threadIdx.x;
  const int comp = blockIdx.y;
  // the factor family depends only on the launch and the system, so that its
  // base addresses stay uniform (scalar buffer resources)
  const Factors F = kind == 1 ? fp : (comp == 3 ? ft : fv);
  const int md = blockIdx.x * kSweepLanes + lane;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const int n = NR > 0 ? NR : d.nr;
  const int kp1 = d.kmax + 1;
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  const int ka = kk >= d.kmax ? kk - d.kmax : d.kmax - kk;
  const double kap = (double)(kk - d.kmax) * d.kz;
  const bool zero = (m == 0 && ka == 0);
  auto C = [&](int j) -> Cd & { return col[j * kSweepLanes + lane]; };
  const double2 *xb = src + (size_t)(kind == 0 ? comp : 0) * n * P + md;
  double2 *out = dst + (size_t)(kind == 0 ? comp : 0) * n * P + md;
  int op = 0;
  if (kind == 1) {
    if (zero) {
      for (int j = 0; j < n; ++j) st(out + (size_t)j * P, Cd{0, 0});
      return;
    }
    op = m * kp1 + ka;
    for (int j = 0; j < n; ++j) C(j) = ld(xb + (size_t)j * P);
  } else if (comp == 3) {
    op = m * kp1 + ka;
    for (int j = 0; j < n; ++j) C(j) = ld(xb + (size_t)j * P);
  } else if (zero) {
    if (comp == 1) return;
    op = (comp == 0 ? 1 : 0) * kp1 + ka;
    for (int j = 0; j < n; ++j) C(j) = ld(xb + (size_t)j * P);
  } else {
    const int q = comp == 0 ? m + 1 : (comp == 1 ? (m >= 1 ? m - 1 : 1 - m) : m);
    op = q * kp1 + ka;
    const Cd b0 = ld(bbar + 2 * (size_t)md), b1 = ld(bbar + 2 * (size_t)md + 1);
    const double sgn = comp == 0 ? 1.0 : -1.0;
    for (int j = 0; j < n; ++j) {
      Cd v = ld(xb + (size_t)j * P);
      if (comp < 2) {
        // 1/2 (D1 + (1 +- m)/r)^T e_w beta_bar_w
        if (j <= 8) {
          double c = g.d1[0 * kStencil + j];
          if (j == 0) c += (1.0 + sgn * m) * g.rinv[0];
          v = v + (0.5 * c) * b0;
        }
        if (j >= n - 9) {
          double c = g.d1[(n - 1) * kStencil + (j - g.s[n - 1])];
          if (j == n - 1) c += (1.0 + sgn * m) * g.rinv[n - 1];
          v = v + (0.5 * c) * b1;
        }
      } else {
        if (j == 0) v = v - kap * ci(b0);
        if (j == n - 1) v = v - kap * ci(b1);
      }
      C(j) = v;
    }
  }
  sweep_t_lds<NR>(F, op, n, C);
  C(0) = Cd{0, 0};
  C(n - 1) = Cd{0, 0};
  if (kind == 0 && zero && comp == 0) {  // fbar+ = (i/2) rbar_theta, fbar- = -(i/2) rbar_theta
    double2 *om = dst + (size_t)n * P + md;
    for (int j = 0; j < n; ++j) {
      const Cd h = 0.5 * ci(C(j));
      st(out + (size_t)j * P, h);
      st(om + (size_t)j * P, Cd{-h.x, -h.y});
    }
    return;
  }
  for (int j = 0; j < n; ++j) st(out + (size_t)j * P, C(j));
}

// pbar0 = -D1^T (rbar+ + rbar-) + (m/r)(rbar+ - rbar-) + i kappa rbar_z.
__global__ void k_adj_pbar(Dims d, Grid g, const double2 *__restrict__ sf, double2 *__restrict__ pb) {
  const int md = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const int n = d.nr;
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  if (md == d.kmax) {
    st(pb + (size_t)j * P + md, Cd{0, 0});
    return;
  }
  const double kap = (double)(kk - d.kmax) * d.kz;
  const double2 *rp = sf + md, *rm = sf + (size_t)n * P + md, *rz = sf + (size_t)2 * n * P + md;
  const Cd dp = wt_rowc(g, g.d1, n, j, rp, P, false);
  const Cd dm = wt_rowc(g, g.d1, n, j, rm, P, false);
  const Cd vp = ld(rp + (size_t)j * P), vm = ld(rm + (size_t)j * P), vz = ld(rz + (size_t)j * P);
  const Cd res = ((m * g.rinv[j]) * (vp - vm)) - (dp + dm) + kap * ci(vz);
  st(pb + (size_t)j * P + md, res);
}

// gbar = mask(P^-T pbar0).
__global__ void __launch_bounds__(256)
k_adj_poisson(Dims d, Factors fp, const double2 *__restrict__ pb, double2 *__restrict__ gb) {
  const int md = blockIdx.x * blockDim.x + threadIdx.x;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const int n = d.nr;
  const int kp1 = d.kmax + 1;
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  const int ka = kk >= d.kmax ? kk - d.kmax : d.kmax - kk;
  auto outr = [&](int j) -> Cd & { return *reinterpret_cast<Cd *>(gb + (size_t)j * P + md); };
  if (m == 0 && ka == 0) {
    for (int j = 0; j < n; ++j) outr(j) = Cd{0, 0};
    return;
  }
  lu_solve_t<Cd>(fp, m * kp1 + ka, n, [&](int j) { return ld(pb + (size_t)j * P + md); }, outr);
  outr(0) = Cd{0, 0};
  outr(n - 1) = Cd{0, 0};
}

// fbar+- = rbar+- + 1/2 (D1^T gbar + (1 +- m) gbar / r), fbar_z = rbar_z - i kappa gbar.
__global__ void k_adj_f(Dims d, Grid g, const double2 *__restrict__ sf, const double2 *__restrict__ gb,
                        double2 *__restrict__ fb) {
  const int md = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const int n = d.nr;
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  const double kap = (double)(kk - d.kmax) * d.kz;
  Cd fp = ld(sf + (size_t)j * P + md), fm = ld(sf + ((size_t)n + j) * P + md);
  Cd fz = ld(sf + ((size_t)2 * n + j) * P + md);
  if (md != d.kmax) {
    const Cd dg = wt_rowc(g, g.d1, n, j, gb + md, P, false);
    const Cd gv = ld(gb + (size_t)j * P + md);
    const double ri = g.rinv[j];
    fp = fp + 0.5 * (dg + ((1.0 + m) * ri) * gv);
    fm = fm + 0.5 * (dg + ((1.0 - m) * ri) * gv);
    fz = fz - kap * ci(gv);
  }
  st(fb + (size_t)j * P + md, fp);
  st(fb + ((size_t)n + j) * P + md, fm);
  st(fb + ((size_t)2 * n + j) * P + md, fz);
  if (d.heated) st(fb + ((size_t)3 * n + j) * P + md, ld(sf + ((size_t)3 * n + j) * P + md));
}

// Input adjoints: Xbar^n = fbar/dt + (1-c) L^T fbar; Nbar^q = c fbar,
// Nbar^n = (1-c) fbar; back to (r, theta, z, T) and accumulated.
__global__ void __launch_bounds__(256)
k_adj_in(Dims d, Grid g, const int *__restrict__ trow, const int *__restrict__ tcnt,
         const double *__restrict__ twt, const double2 *__restrict__ fb, double idt, double cc,
         double2 *__restrict__ ubn, double2 *__restrict__ nbn, double2 *__restrict__ nbq,
         int overwrite) {
  const int md = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const int n = d.nr;
  const int m = md / d.mz;
  const int kk = md - m * d.mz;
  const double kap = (double)(kk - d.kmax) * d.kz;
  const double ri = g.rinv[j], r2 = ri * ri, k2 = kap * kap;
  const double ce = 1.0 - cc;
  Cd xb[4], fv[4];
  const int nf = d.heated ? 4 : 3;
#pragma unroll
  for (int c = 0; c < 4; ++c) {  // (constant trip count: xb, fv stay in registers)
    if (c >= nf) {
      xb[c] = fv[c] = Cd{0, 0};
      continue;
    }
    const double2 *f = fb + (size_t)c * n * P + md;
    const double q = c == 0 ? (double)(m + 1) : (c == 1 ? (double)(m >= 1 ? m - 1 : 1 - m) : (double)m);
    const Cd v = ld(f + (size_t)j * P);
    // (D2 + D1/r)^T f at row j from the column's table (uniform per workgroup)
    Cd lt = {0, 0};
    const int cnt = tcnt[j];
    for (int e = 0; e < cnt; ++e)
      lt = fmac(twt[j * kTrans + e], ld(f + (size_t)trow[j * kTrans + e] * P), lt);
    const Cd LT = lt - (q * q * r2 + k2) * v;
    const double sc = c == 3 ? ce / d.pr : ce;
    xb[c] = idt * v + sc * LT;
    fv[c] = v;
  }
  auto acc = [&](double2 *base, int f, Cd v, int bit) {
    double2 *p = base + ((size_t)f * n + j) * P + md;
    if (overwrite & bit) {
      *p = make_double2(v.x, v.y);
    } else {
      p->x += v.x;
      p->y += v.y;
    }
  };
  // X+- = X_r +- i X_theta  =>  Xbar_r = Xbar+ + Xbar-, Xbar_theta = -i (Xbar+ - Xbar-)
  const Cd ur = xb[0] + xb[1];
  const Cd dd = xb[0] - xb[1];
  const Cd ut = {dd.y, -dd.x};
  acc(ubn, 0, ur, 1);
  acc(ubn, 1, ut, 1);
  acc(ubn, 2, xb[2], 1);
  if (d.heated) acc(ubn, 3, xb[3], 1);
  const Cd fr = fv[0] + fv[1];
  const Cd fdd = fv[0] - fv[1];
  const Cd ft = {fdd.y, -fdd.x};
  acc(nbq, 0, cc * fr, 4);
  acc(nbq, 1, cc * ft, 4);
  acc(nbq, 2, cc * fv[2], 4);
  acc(nbn, 0, ce * fr, 2);
  acc(nbn, 1, ce * ft, 2);
  acc(nbn, 2, ce * fv[2], 2);
  if (d.heated) {
    acc(nbq, 3, cc * fv[3], 4);
    acc(nbn, 3, ce * fv[3], 2);
  }
}

// dE/du = 2 pi L_z w_j r_j c_m (u - U_b) for the velocity, 0 for T.
__global__ void k_energy_grad(Dims d, Grid g, const double2 *__restrict__ u, double2 *__restrict__ gout) {
  const int md = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (md >= d.nmodes) return;
  const size_t P = d.nmodes;
  const int m = md / d.mz;
  const double s = 2.0 * M_PI * d.lz * g.ccw[j] * g.r[j] * (m == 0 ? 1.0 : 2.0);
  for (int f = 0; f < d.f; ++f) {
    double2 v = u[((size_t)f * d.nr + j) * P + md];
    if (f == 1 && md == d.kmax) v.x -= d.a_cou * g.r[j] + d.b_cou * g.rinv[j];
    if (f == 3) v = make_double2(0.0, 0.0);
    gout[((size_t)f * d.nr + j) * P + md] = make_double2(s * v.x, s * v.y);
  }
}

// Rows per lane of a stencil kernel with `parts` workgroups per (mode tile,
// row chunk): the longest chunk, up to four rows, that still leaves
// `min_waves` wavefronts per SIMD.  Longer chunks save reads of the shared
// window rows but cost occupancy.  Measured on 64 rows x 8128 modes and 128 x
// 130816: the kernels with two stencil fields per lane (divergence, the +-
// right sides) are fastest down to four wavefronts per SIMD (two and four
// rows on the first grid, four on the second); the velocity right sides, one
// stencil field beside six streamed ones, need eight (one row on the first
// grid, four on the second).
inline int chunk_rows(const nsc_ctx *c, int parts, int min_waves) {
  const long waves_row = (long)(c->d.nmodes + 255) / 256 * 4 * parts;
  const long simds = 4L * c->cu_count;
  for (int R = 4; R > 1; R /= 2)
    if (waves_row * ((c->d.nr + R - 1) / R) >= (long)min_waves * simds) return R;
  return 1;
}

inline dim3 mode_grid(const nsc_ctx *c, int y, int z = 1) {
  return dim3((c->d.nmodes + 255) / 256, y, z);
}

}  // namespace

hipError_t launch_factor(const nsc_ctx *c, Factors *f, int kind, double alpha, double beta) {
  hipLaunchKernelGGL(k_factor, dim3((f->nops + kFacThreads - 1) / kFacThreads), dim3(kFacThreads), 0,
                     c->stream, c->d, c->g, *f, *f, kind, alpha, beta, beta, 0);
  return hipGetLastError();
}

hipError_t launch_factor2(const nsc_ctx *c, Factors *f0, Factors *f1, int kind, double alpha,
                          double beta0, double beta1) {
  const int nmax = f0->nops > f1->nops ? f0->nops : f1->nops;
  hipLaunchKernelGGL(k_factor, dim3((nmax + kFacThreads - 1) / kFacThreads, 2),
                     dim3(kFacThreads), 0, c->stream, c->d, c->g, *f0, *f1, kind, alpha, beta0,
                     beta1, 0);
  return hipGetLastError();
}

hipError_t launch_influence_pressure(const nsc_ctx *c) {
  hipLaunchKernelGGL(k_influence_p, dim3((c->inf.nops + 63) / 64, 2), dim3(64), 0, c->stream, c->d,
                     c->fp, c->inf);
  return hipGetLastError();
}

hipError_t launch_influence_setup(const nsc_ctx *c) {
  const dim3 gx((c->inf.nops + 63) / 64, 2, 3);
  // LDS columns only while every workgroup is resident at once: the solves
  // are latency chains, and at larger sizes the LDS would cap the waves in
  // flight below what the global-memory variant keeps
  const size_t shm = (size_t)2 * c->d.nr * 64 * sizeof(double);
  const size_t resident = shm <= (size_t)c->lds_max ? (size_t)c->cu_count * (c->lds_cu / shm) : 0;
  if ((size_t)gx.x * gx.y * gx.z <= resident)
    hipLaunchKernelGGL(k_influence_x<true>, gx, dim3(64), shm, c->stream, c->d, c->g, c->fv, c->inf);
  else
    hipLaunchKernelGGL(k_influence_x<false>, gx, dim3(64), 0, c->stream, c->d, c->g, c->fv, c->inf);
  hipLaunchKernelGGL(k_influence_a, dim3((c->inf.nops + 63) / 64), dim3(64), 0, c->stream, c->d,
                     c->g, c->inf);
  return hipGetLastError();
}

hipError_t launch_rhs(const nsc_ctx *c, const double *u, const double *nn, const double *nq,
                      double dt, double cc) {
  const int parts = c->d.heated ? 3 : 2;
  auto rhs = [&](auto rows) {
    constexpr int R = decltype(rows)::value;
    auto kern = c->d.pipe ? k_rhs<R, true> : k_rhs<R, false>;
    hipLaunchKernelGGL(kern, mode_grid(c, (c->d.nr + R - 1) / R, parts), dim3(256), 0,
                       c->stream, c->d, c->g, reinterpret_cast<const double2 *>(u),
                       reinterpret_cast<const double2 *>(nn), reinterpret_cast<const double2 *>(nq),
                       reinterpret_cast<double2 *>(c->s_f), 1.0 / dt, cc, c->rows_first);
  };
  switch (chunk_rows(c, parts, 4)) {
    case 4: rhs(std::integral_constant<int, 4>{}); break;
    case 2: rhs(std::integral_constant<int, 2>{}); break;
    default: rhs(std::integral_constant<int, 1>{}); break;
  }
  return hipGetLastError();
}

hipError_t launch_influence(const nsc_ctx *c) {
  auto kern = c->d.pipe ? k_influence<true> : k_influence<false>;
  hipLaunchKernelGGL(kern, dim3((c->d.nmodes + 63) / 64), dim3(64), 0, c->stream, c->d, c->g, c->inf,
                     reinterpret_cast<const double2 *>(c->s_x), reinterpret_cast<double2 *>(c->s_lam));
  return hipGetLastError();
}

hipError_t launch_finalize(const nsc_ctx *c, double *out, double *p_out) {
  auto fin = p_out ? k_finalize<true> : k_finalize<false>;
  hipLaunchKernelGGL(fin, mode_grid(c, c->d.nr), dim3(256), 0, c->stream, c->d, c->inf,
                     reinterpret_cast<const double2 *>(c->s_x), reinterpret_cast<const double2 *>(c->s_p),
                     reinterpret_cast<const double2 *>(c->s_lam), reinterpret_cast<double2 *>(out),
                     reinterpret_cast<double2 *>(p_out));
  return hipGetLastError();
}

hipError_t launch_energy(const nsc_ctx *c, const double *u, double *e_dev) {
  hipLaunchKernelGGL(k_energy_part, dim3(c->e_nblk), dim3(256), 0, c->stream, c->d, c->g,
                     reinterpret_cast<const double2 *>(u), c->e_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, c->stream, c->e_part, c->e_nblk,
                     M_PI * c->d.lz, e_dev);
  return hipGetLastError();
}

hipError_t launch_seed(const nsc_ctx *c, const double *amps, double *out_pert) {
  hipLaunchKernelGGL(k_seed, mode_grid(c, c->d.nr, c->d.f), dim3(256), 0, c->stream, c->d, c->g,
                     reinterpret_cast<const double2 *>(amps), reinterpret_cast<double2 *>(out_pert));
  return hipGetLastError();
}

hipError_t launch_add_base(const nsc_ctx *c, const double *pert_tilde, double *out) {
  hipLaunchKernelGGL(k_add_base, mode_grid(c, c->d.nr), dim3(256), 0, c->stream, c->d, c->g,
                     reinterpret_cast<const double2 *>(pert_tilde), reinterpret_cast<double2 *>(out));
  return hipGetLastError();
}

hipError_t launch_solve_vjp(const nsc_ctx *c, const double *ubar_out, double *ubar_n,
                            double *nbar_n, double *nbar_q, double dt, double cc,
                            int overwrite) {
  const double2 *ub = reinterpret_cast<const double2 *>(ubar_out);
  double2 *sx = reinterpret_cast<double2 *>(c->s_x);
  double2 *sf = reinterpret_cast<double2 *>(c->s_f);
  double2 *sg = reinterpret_cast<double2 *>(c->s_g);
  double2 *sp = reinterpret_cast<double2 *>(c->s_p);
  double2 *lam = reinterpret_cast<double2 *>(c->s_lam);
  hipLaunchKernelGGL(k_adj_out, mode_grid(c, c->d.nr), dim3(256), 0, c->stream, c->d, ub, sx);
  hipLaunchKernelGGL(k_adj_lambda, dim3((c->d.nmodes + kLamModes - 1) / kLamModes), dim3(kLamModes * kLamParts),
                     0, c->stream, c->d, c->inf, sx, lam);
  const size_t col_bytes = (size_t)kSweepLanes * c->d.nr * sizeof(Cd);
  const bool lds = col_bytes <= 64 * 1024;
  const dim3 lg((c->d.nmodes + kSweepLanes - 1) / kSweepLanes, c->d.heated ? 4 : 3);
  const dim3 lg1((c->d.nmodes + kSweepLanes - 1) / kSweepLanes, 1);
  // the unrolled sweeps read the packed factors (present where they run)
  const bool unrolled = lds && c->fv.pc;
  auto adj_sweep = c->d.nr == 64 ? k_adj_sweep<64> : k_adj_sweep<32>;
  if (unrolled)
    hipLaunchKernelGGL(adj_sweep, lg, dim3(kSweepLanes), col_bytes, c->stream, c->d, c->g,
                       c->fv, c->ft, c->fp, 0, sx, lam, sf);
  else if (lds)
    hipLaunchKernelGGL(k_adj_sweep<0>, lg, dim3(kSweepLanes), col_bytes, c->stream, c->d, c->g,
                       c->fv, c->ft, c->fp, 0, sx, lam, sf);
  else
    hipLaunchKernelGGL(k_adj_vel, mode_grid(c, c->d.heated ? 4 : 3), dim3(256), 0, c->stream, c->d,
                       c->g, c->fv, c->ft, sx, lam, sf);
  hipLaunchKernelGGL(k_adj_pbar, mode_grid(c, c->d.nr), dim3(256), 0, c->stream, c->d, c->g, sf, sp);
  if (unrolled)
    hipLaunchKernelGGL(adj_sweep, lg1, dim3(kSweepLanes), col_bytes, c->stream, c->d, c->g,
                       c->fv, c->ft, c->fp, 1, sp, lam, sg);
  else if (lds)
    hipLaunchKernelGGL(k_adj_sweep<0>, lg1, dim3(kSweepLanes), col_bytes, c->stream, c->d, c->g,
                       c->fv, c->ft, c->fp, 1, sp, lam, sg);
  else
    hipLaunchKernelGGL(k_adj_poisson, mode_grid(c, 1), dim3(256), 0, c->stream, c->d, c->fp, sp, sg);
  hipLaunchKernelGGL(k_adj_f, mode_grid(c, c->d.nr), dim3(256), 0, c->stream, c->d, c->g, sf, sg, sx);
  hipLaunchKernelGGL(k_adj_in, mode_grid(c, c->d.nr), dim3(256), 0, c->stream, c->d, c->g,
                     c->t_row, c->t_cnt, c->t_wt, sx, 1.0 / dt, cc,
                     reinterpret_cast<double2 *>(ubar_n), reinterpret_cast<double2 *>(nbar_n),
                     reinterpret_cast<double2 *>(nbar_q), overwrite);
  return hipGetLastError();
}

__global__ void k_fill_zero(double *__restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_add(double *__restrict__ y, const double *__restrict__ x, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] += x[i];
}

// n doubles set to zero / y += x, in kernels (no memset node when captured)
hipError_t launch_fill_zero(const nsc_ctx *c, double *p, size_t n) {
  const size_t blocks = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, c->stream, p, n);
  return hipGetLastError();
}

hipError_t launch_add(const nsc_ctx *c, double *y, const double *x, size_t n) {
  const size_t blocks = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
  hipLaunchKernelGGL(k_add, dim3((unsigned)blocks), dim3(256), 0, c->stream, y, x, n);
  return hipGetLastError();
}

hipError_t launch_energy_grad(const nsc_ctx *c, const double *u, double *gout) {
  hipLaunchKernelGGL(k_energy_grad, mode_grid(c, c->d.nr), dim3(256), 0, c->stream, c->d, c->g,
                     reinterpret_cast<const double2 *>(u), reinterpret_cast<double2 *>(gout));
  return hipGetLastError();
}

// stage 0: Poisson right side (+ temperature wall rows); 1: pressure and
// temperature sweeps; 2: velocity right sides; 3: velocity sweeps.
hipError_t launch_solve_sweeps(const nsc_ctx *c, int stage, const double *nn, const double *nq,
                               double cc, int walls, int want_p) {
  const Dims &d = c->d;
  double2 *sf = reinterpret_cast<double2 *>(c->s_f);
  double2 *sg = reinterpret_cast<double2 *>(c->s_g);
  double2 *sp = reinterpret_cast<double2 *>(c->s_p);
  double2 *sx = reinterpret_cast<double2 *>(c->s_x);
  const int wp = (want_p && nn) ? 1 : 0;
  const size_t col_bytes = (size_t)kSweepLanes * d.nr * sizeof(Cd);
  const bool lds = col_bytes <= 64 * 1024;
  const size_t shm = lds ? col_bytes : 0;
  auto launch = [&](const SweepArgs &a, int nsys, auto family) {
    constexpr int FAM = decltype(family)::value;
    dim3 gr((d.nmodes + kSweepLanes - 1) / kSweepLanes, nsys);
    // the unrolled variant reads the row-packed factors with 32-bit buffer
    // offsets (allocated where sweeps_unrolled holds)
    if (lds && c->fv.pk && d.nr == 64)
      hipLaunchKernelGGL((k_sweep<true, FAM, 64>), gr, dim3(kSweepLanes), shm, c->stream, d, a);
    else if (lds && c->fv.pk)
      hipLaunchKernelGGL((k_sweep<true, FAM, 32>), gr, dim3(kSweepLanes), shm, c->stream, d, a);
    else if (lds)
      hipLaunchKernelGGL((k_sweep<true, FAM, 0>), gr, dim3(kSweepLanes), shm, c->stream, d, a);
    else
      hipLaunchKernelGGL((k_sweep<false, FAM, 0>), gr, dim3(kSweepLanes), 0, c->stream, d, a);
  };
  const size_t fld = (size_t)d.nr * d.nmodes;
  if (stage == 0) {
    auto div = [&](auto rows) {
      constexpr int R = decltype(rows)::value;
      auto kern = d.pipe ? k_div2<R, true> : k_div2<R, false>;
      hipLaunchKernelGGL(kern, mode_grid(c, (d.nr + R - 1) / R), dim3(256), 0, c->stream,
                         d, c->g, sf, sg, reinterpret_cast<const double2 *>(nn),
                         reinterpret_cast<const double2 *>(nq), cc, wp, walls, c->rows_first);
    };
    switch (chunk_rows(c, 1, 4)) {
      case 4: div(std::integral_constant<int, 4>{}); break;
      case 2: div(std::integral_constant<int, 2>{}); break;
      default: div(std::integral_constant<int, 1>{}); break;
    }
  } else if (stage == 1) {
    // pressure (s_g -> s_p) and temperature (s_f[3] -> s_x[3]) in one launch
    SweepArgs a{};
    a.s[0] = SweepSys{c->fp, 0, wp ? 0 : 1, sg, sp};
    if (d.heated) a.s[1] = SweepSys{c->ft, 0, 0, sf + 3 * fld, sx + 3 * fld};
    launch(a, d.heated ? 2 : 1, std::integral_constant<int, 0>{});
  } else if (stage == 2) {
    auto vel = [&](auto rows) {
      constexpr int R = decltype(rows)::value;
      auto kern = d.pipe ? k_vel_rhs<R, true> : k_vel_rhs<R, false>;
      hipLaunchKernelGGL(kern, mode_grid(c, (d.nr + R - 1) / R), dim3(256), 0,
                         c->stream, d, c->g, sf, sp, walls, c->rows_first);
    };
    switch (chunk_rows(c, 1, 8)) {
      case 4: vel(std::integral_constant<int, 4>{}); break;
      case 2: vel(std::integral_constant<int, 2>{}); break;
      default: vel(std::integral_constant<int, 1>{}); break;
    }
  } else {
    SweepArgs av{};
    av.s[0] = SweepSys{c->fv, 1, 0, sf, sx};
    av.s[1] = SweepSys{c->fv, 2, 0, sf + fld, sx + fld};
    av.s[2] = SweepSys{c->fv, 0, 0, sf + 2 * fld, sx + 2 * fld};
    launch(av, 3, std::integral_constant<int, 1>{});
  }
  return hipGetLastError();
}

}  // namespace nsc
