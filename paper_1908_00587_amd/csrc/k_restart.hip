// Restart with a change of resolution, and the state file it reads
// (section 2.1: at every restart the spatial resolution may change through
// interpolation and mode padding; section 2.4: the checkpoint-restart works
// on the spectral coefficients).
//
//   k_remap  one lane per (field, target mode), kRemapRows target rows per
//            lane: modes present at both resolutions take the radial
//            interpolation of their old profile, new modes are zero.  The
//            interpolation weights are uniform across a workgroup (scalar
//            loads); the source column streams once per row group.
//
// Interpolant: the polynomial through all points of the old
// Chebyshev--Gauss--Lobatto grid, in the barycentric form with the weights
// of those points ((-1)^j, halved at the two walls), which is the stable
// evaluation of that polynomial.  Both grids contain the walls, whose values
// are copied.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "nsc_internal.h"

namespace nsc {
namespace {

constexpr int kRemapLanes = 64;
constexpr int kRemapRows = 16;  // target rows accumulated per lane

__global__ void __launch_bounds__(kRemapLanes)
k_remap(const double2 *__restrict__ src, int n0, int mt0, int mz0, const double *__restrict__ W,
        double2 *__restrict__ dst, int n1, int mt1, int mz1) {
  const int md = blockIdx.x * kRemapLanes + threadIdx.x;
  const int nm1 = mt1 * mz1;
  if (md >= nm1) return;
  const int f = blockIdx.z;
  const int i0 = blockIdx.y * kRemapRows;
  const int m = md / mz1;
  const int k = md - m * mz1 - (mz1 - 1) / 2;
  const int K0 = (mz0 - 1) / 2;
  double2 acc[kRemapRows];
#pragma unroll
  for (int r = 0; r < kRemapRows; ++r) acc[r] = make_double2(0.0, 0.0);
  if (m < mt0 && k >= -K0 && k <= K0) {
    const size_t P0 = (size_t)mt0 * mz0;
    const double2 *s = src + (size_t)f * n0 * P0 + (size_t)m * mz0 + (k + K0);
    // rows past the end repeat the last row's weights (their sums are not stored)
    const double *w[kRemapRows];
#pragma unroll
    for (int r = 0; r < kRemapRows; ++r) w[r] = W + (size_t)min(i0 + r, n1 - 1) * n0;
#pragma unroll 4
    for (int j = 0; j < n0; ++j) {
      const double2 v = s[(size_t)j * P0];
#pragma unroll
      for (int r = 0; r < kRemapRows; ++r) {
        acc[r].x = fma(w[r][j], v.x, acc[r].x);
        acc[r].y = fma(w[r][j], v.y, acc[r].y);
      }
    }
  }
  double2 *o = dst + ((size_t)f * n1 + i0) * nm1 + md;
#pragma unroll
  for (int r = 0; r < kRemapRows; ++r)
    if (i0 + r < n1) o[(size_t)r * nm1] = acc[r];
}

// Radial grid of n points between the walls, as the context builds its own.
std::vector<double> cgl_grid(int n, double r_i, double r_o) {
  std::vector<double> r(n);
  for (int j = 0; j < n; ++j)
    r[j] = 0.5 * (r_i + r_o) + 0.5 * std::cos(M_PI * (double)(n - 1 - j) / (double)(n - 1));
  return r;
}

// W[i][j]: weight of old point j in the interpolant at new point i.
std::vector<double> remap_weights(const std::vector<double> &x0, const std::vector<double> &x1) {
  const int n0 = (int)x0.size(), n1 = (int)x1.size();
  std::vector<double> W((size_t)n1 * n0, 0.0);
  std::vector<double> bw(n0);
  for (int j = 0; j < n0; ++j) bw[j] = ((j & 1) ? -1.0 : 1.0) * ((j == 0 || j == n0 - 1) ? 0.5 : 1.0);
  for (int i = 0; i < n1; ++i) {
    double *row = W.data() + (size_t)i * n0;
    int hit = -1;
    for (int j = 0; j < n0; ++j)
      if (x1[i] == x0[j]) hit = j;
    if (hit >= 0) {
      row[hit] = 1.0;
      continue;
    }
    double den = 0.0;
    for (int j = 0; j < n0; ++j) {
      row[j] = bw[j] / (x1[i] - x0[j]);
      den += row[j];
    }
    for (int j = 0; j < n0; ++j) row[j] /= den;
  }
  return W;
}

// The grid limits of nsc_init: N_r <= 4096 and padded lengths 3 M_theta,
// 3 (M_z + 1) / 2 <= 4096.  They bound the payload (< 2^40 bytes), so a
// header's sizes cannot wrap the byte count.
bool valid_dims(int n_r, int m_theta, int m_z) {
  return n_r >= kStencil && n_r <= 4096 && m_theta >= 1 && 3 * (long)m_theta <= kMaxFFT &&
         m_z >= 1 && (m_z & 1) == 1 && 3 * (((long)m_z - 1) / 2 + 1) <= kMaxFFT;
}

// State file: a 128-byte little-endian header, then the coefficients
// [F][N_r][M_theta][M_z] as (re, im) FP64 pairs.
struct StateHeader {
  char magic[8];  // "NSCSTATE"
  uint32_t version;
  uint32_t fields;
  int32_t n_r, m_theta, m_z;
  uint32_t reserved0;
  double eta, re_i, re_o, ra, pr, l_z, time;
  uint8_t reserved[40];
};
static_assert(sizeof(StateHeader) == 128, "state file header is 128 bytes");
constexpr char kMagic[8] = {'N', 'S', 'C', 'S', 'T', 'A', 'T', 'E'};
constexpr uint32_t kVersion = 1;
constexpr size_t kStage = (size_t)32 << 20;  // pinned staging chunk

size_t payload_bytes(const StateHeader &h) {
  return (size_t)h.fields * h.n_r * h.m_theta * h.m_z * 2 * sizeof(double);
}

int read_header(FILE *fp, StateHeader *h) {
  if (std::fread(h, sizeof(StateHeader), 1, fp) != 1) return NSC_ERR_IO;
  if (std::memcmp(h->magic, kMagic, 8) != 0 || h->version != kVersion) return NSC_ERR_IO;
  if ((h->fields != 3 && h->fields != 4) || !valid_dims(h->n_r, h->m_theta, h->m_z))
    return NSC_ERR_IO;
  // the payload must be there in full
  const long here = std::ftell(fp);
  if (here < 0 || std::fseek(fp, 0, SEEK_END) != 0) return NSC_ERR_IO;
  const long end = std::ftell(fp);
  if (end < 0 || (size_t)(end - here) != payload_bytes(*h)) return NSC_ERR_IO;
  if (std::fseek(fp, here, SEEK_SET) != 0) return NSC_ERR_IO;
  return NSC_OK;
}

// bytes from the file into device memory through a pinned staging buffer
int upload(nsc_ctx *c, FILE *fp, double *dev, size_t bytes) {
  void *stage = nullptr;
  if (hipHostMalloc(&stage, kStage, hipHostMallocDefault) != hipSuccess) return NSC_ERR_OOM;
  int st = NSC_OK;
  for (size_t off = 0; off < bytes && st == NSC_OK; off += kStage) {
    const size_t n = bytes - off < kStage ? bytes - off : kStage;
    if (std::fread(stage, 1, n, fp) != n) {
      st = NSC_ERR_IO;
      break;
    }
    if (hipMemcpyAsync(reinterpret_cast<char *>(dev) + off, stage, n, hipMemcpyHostToDevice,
                       c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      st = NSC_ERR_DEVICE;
  }
  (void)hipHostFree(stage);
  return st;
}

}  // namespace

hipError_t launch_remap(const nsc_ctx *c, const double *src, int n0, int mt0, int mz0,
                        const double *W_dev, double *dst) {
  const nsc::Dims &d = c->d;
  const dim3 grid((d.nmodes + kRemapLanes - 1) / kRemapLanes, (d.nr + kRemapRows - 1) / kRemapRows,
                  d.f);
  hipLaunchKernelGGL(k_remap, grid, dim3(kRemapLanes), 0, c->stream,
                     reinterpret_cast<const double2 *>(src), n0, mt0, mz0, W_dev,
                     reinterpret_cast<double2 *>(dst), d.nr, d.mt, d.mz);
  return hipGetLastError();
}

}  // namespace nsc

using nsc::StateHeader;

int nsc_remap_state(nsc_ctx *c, const double *src, int N_r_src, int M_theta_src, int M_z_src,
                    double *dst) {
  if (!c || !src || !dst || !nsc::valid_dims(N_r_src, M_theta_src, M_z_src)) return NSC_ERR_ARG;
  if (c->d.pipe) return NSC_ERR_STATE;
  const size_t sbytes = (size_t)c->d.f * N_r_src * M_theta_src * M_z_src * 2 * sizeof(double);
  const size_t dbytes = (size_t)c->d.f * c->d.nr * c->d.nmodes * 2 * sizeof(double);
  const char *s0 = reinterpret_cast<const char *>(src), *d0 = reinterpret_cast<const char *>(dst);
  if (s0 < d0 + dbytes && d0 < s0 + sbytes) return NSC_ERR_ARG;  // overlap
  const std::vector<double> W = nsc::remap_weights(nsc::cgl_grid(N_r_src, c->d.r_i, c->d.r_o),
                                                   nsc::cgl_grid(c->d.nr, c->d.r_i, c->d.r_o));
  double *W_dev = nullptr;
  if (hipMalloc((void **)&W_dev, W.size() * sizeof(double)) != hipSuccess) return NSC_ERR_OOM;
  int st = NSC_OK;
  if (hipMemcpyAsync(W_dev, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice, c->stream) !=
      hipSuccess)
    st = NSC_ERR_DEVICE;
  if (st == NSC_OK) {
    nsc::StageTimer t(c, 3);
    if (nsc::launch_remap(c, src, N_r_src, M_theta_src, M_z_src, W_dev, dst) != hipSuccess)
      st = NSC_ERR_DEVICE;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess && st == NSC_OK) st = NSC_ERR_DEVICE;
  (void)hipFree(W_dev);
  return st;
}

int nsc_save_state(nsc_ctx *c, const double *u_hat, double time, const char *path) {
  if (!c || !u_hat || !path) return NSC_ERR_ARG;
  if (c->d.pipe) return NSC_ERR_STATE;
  StateHeader h{};
  std::memcpy(h.magic, nsc::kMagic, 8);
  h.version = nsc::kVersion;
  h.fields = (uint32_t)c->d.f;
  h.n_r = c->d.nr;
  h.m_theta = c->d.mt;
  h.m_z = c->d.mz;
  h.eta = c->eta;
  h.re_i = c->d.re_i;
  h.re_o = c->d.re_o;
  h.ra = c->ra;
  h.pr = c->d.pr;
  h.l_z = c->d.lz;
  h.time = time;
  FILE *fp = std::fopen(path, "wb");
  if (!fp) return NSC_ERR_IO;
  int st = std::fwrite(&h, sizeof h, 1, fp) == 1 ? NSC_OK : NSC_ERR_IO;
  void *stage = nullptr;
  if (st == NSC_OK && hipHostMalloc(&stage, nsc::kStage, hipHostMallocDefault) != hipSuccess)
    st = NSC_ERR_OOM;
  const size_t bytes = nsc::payload_bytes(h);
  for (size_t off = 0; off < bytes && st == NSC_OK; off += nsc::kStage) {
    const size_t n = bytes - off < nsc::kStage ? bytes - off : nsc::kStage;
    if (hipMemcpyAsync(stage, reinterpret_cast<const char *>(u_hat) + off, n, hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      st = NSC_ERR_DEVICE;
      break;
    }
    if (std::fwrite(stage, 1, n, fp) != n) st = NSC_ERR_IO;
  }
  if (stage) (void)hipHostFree(stage);
  if (std::fclose(fp) != 0 && st == NSC_OK) st = NSC_ERR_IO;
  if (st != NSC_OK) std::remove(path);  // no partial state file is left behind
  return st;
}

int nsc_read_state_header(const char *path, int *dims, double *params) {
  if (!path || !dims || !params) return NSC_ERR_ARG;
  FILE *fp = std::fopen(path, "rb");
  if (!fp) return NSC_ERR_IO;
  StateHeader h{};
  const int st = nsc::read_header(fp, &h);
  std::fclose(fp);
  if (st != NSC_OK) return st;
  dims[0] = (int)h.fields;
  dims[1] = h.n_r;
  dims[2] = h.m_theta;
  dims[3] = h.m_z;
  const double p[7] = {h.eta, h.re_i, h.re_o, h.ra, h.pr, h.l_z, h.time};
  std::memcpy(params, p, sizeof p);
  return NSC_OK;
}

int nsc_load_state(nsc_ctx *c, const char *path, double *u_hat, double *time_out) {
  if (!c || !path || !u_hat) return NSC_ERR_ARG;
  if (c->d.pipe) return NSC_ERR_STATE;
  FILE *fp = std::fopen(path, "rb");
  if (!fp) return NSC_ERR_IO;
  StateHeader h{};
  int st = nsc::read_header(fp, &h);
  // the geometry must be the context's; flow parameters may differ (a
  // restart may change them)
  if (st == NSC_OK &&
      ((int)h.fields != c->d.f || std::fabs(h.eta - c->eta) > 1e-12 * c->eta ||
       std::fabs(h.l_z - c->d.lz) > 1e-12 * c->d.lz))
    st = NSC_ERR_ARG;
  if (st == NSC_OK) {
    if (h.n_r == c->d.nr && h.m_theta == c->d.mt && h.m_z == c->d.mz) {
      st = nsc::upload(c, fp, u_hat, nsc::payload_bytes(h));
    } else {
      double *src = nullptr;
      if (hipMalloc((void **)&src, nsc::payload_bytes(h)) != hipSuccess) {
        st = NSC_ERR_OOM;
      } else {
        st = nsc::upload(c, fp, src, nsc::payload_bytes(h));
        if (st == NSC_OK) st = nsc_remap_state(c, src, h.n_r, h.m_theta, h.m_z, u_hat);
        (void)hipFree(src);
      }
    }
  }
  std::fclose(fp);
  if (st == NSC_OK && time_out) *time_out = h.time;
  return st;
}
