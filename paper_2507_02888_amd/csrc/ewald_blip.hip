// Batched blip-orbital evaluation for gfx950 (the paper's Sec. 2.4: orbitals
// re-represented in a blip (B-spline) basis; evaluating them after a move is a
// grid lookup, a few cubic polynomials, and the multiplication of the 64
// blip functions that are nonzero at the point by every orbital's
// coefficients, which the paper sends through 64-element BLAS calls one
// point at a time, Sec. 5.3).  Here one wave serves one point:
//   - lane p < 64 finds grid point p of the 4 x 4 x 4 window around the
//     point and forms its blip product, the product's Cartesian gradient and
//     its Laplacian (five weights), parked in LDS with the row index;
//   - every lane then streams the 64 coefficient rows (orbital index
//     fastest, so a wave reads 1 KiB of one row per 16-byte load) and
//     accumulates value, gradient and Laplacian of two orbitals per chunk of
//     128 orbitals.
// The work is a gather of 64 n_orb coefficients per point with 5 FMAs per
// coefficient: bound by memory (HBM, or the 256 MB last-level cache when the
// coefficient set fits it), not by arithmetic, and not a dense contraction
// (each point takes its own 64 rows).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>

#include "ewald.h"
#include "ewald_internal.h"

namespace ewald {
// thread-local message shared with the rest of the library
void set_last_error(const std::string& msg);
}  // namespace ewald

struct ewald_blip {
  int grid[3];
  int n_orb;
  double ainv[9];   // s = r Ainv (row vectors)
  double J[9];      // J[e][d] = d x_d / d r_e = Ainv[e][d] n_d
  double M[6];      // sum_e J[e][d] J[e][d'] for (d, d') = 00, 11, 22, 01, 02, 12
};

namespace ewald {
namespace {

struct BlipK {
  int n[3];
  int n_orb;
  double ainv[9];
  double J[9];
  double M[6];
};

// Blip function Th(x) = 1 - 3/2 x^2 + 3/4 |x|^3 (|x| <= 1), 1/4 (2 - |x|)^3
// (1 < |x| < 2), and its first two derivatives.
__device__ __forceinline__ void blip_fn(double x, double& f, double& f1, double& f2) {
  const double ax = fabs(x), sg = x < 0.0 ? -1.0 : 1.0;
  if (ax <= 1.0) {
    f = fma(0.75 * ax, x * x, fma(-1.5, x * x, 1.0));
    f1 = fma(2.25 * sg, x * x, -3.0 * x);
    f2 = fma(4.5, ax, -3.0);
  } else {
    const double t = ax < 2.0 ? 2.0 - ax : 0.0;
    f = 0.25 * t * t * t;
    f1 = -0.75 * sg * t * t;
    f2 = 1.5 * t;
  }
}

struct __align__(16) BlipW {
  double b, gx, gy, gz, l;
  long long row;  // coefficient row (grid point) index
};

constexpr int BLIP_WAVES = 4;  // points (waves) per workgroup

// VW = 2: orbital pairs read as 16-byte loads (n_orb even); 1: single loads.
template <int VW, bool DER>
__global__ __launch_bounds__(64 * BLIP_WAVES) void k_blip(BlipK K, const double* __restrict__ coef, int n_pts,
                                                            const double* __restrict__ pos, double* __restrict__ val,
                                                            double* __restrict__ grad, double* __restrict__ lap) {
  __shared__ BlipW wts[BLIP_WAVES][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = blockIdx.x * BLIP_WAVES + wave;
  if (p >= n_pts) return;  // uniform per wave; no block-level barrier below
  BlipW* W = wts[wave];
  {
    double x[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double s = 0.0;
#pragma unroll
      for (int e = 0; e < 3; ++e) s = fma(pos[size_t(p) * 3 + e], K.ainv[e * 3 + d], s);
      s -= floor(s);
      x[d] = s * K.n[d];
    }
    const int a[3] = {lane >> 4, (lane >> 2) & 3, lane & 3};
    double f[3], f1[3], f2[3];
    long long idx[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double fl = floor(x[d]);
      const long long g = (long long)fl - 1 + a[d];  // grid points floor(x) - 1 .. floor(x) + 2
      blip_fn(x[d] - double(g), f[d], f1[d], f2[d]);
      long long gw = g % K.n[d];
      idx[d] = gw < 0 ? gw + K.n[d] : gw;
    }
    BlipW w;
    w.b = f[0] * f[1] * f[2];
    if (DER) {
      const double dx[3] = {f1[0] * f[1] * f[2], f[0] * f1[1] * f[2], f[0] * f[1] * f1[2]};
      // second derivatives in x: diagonal and mixed
      const double h00 = f2[0] * f[1] * f[2], h11 = f[0] * f2[1] * f[2], h22 = f[0] * f[1] * f2[2];
      const double h01 = f1[0] * f1[1] * f[2], h02 = f1[0] * f[1] * f1[2], h12 = f[0] * f1[1] * f1[2];
      double g[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) g[e] = fma(K.J[e * 3 + 2], dx[2], fma(K.J[e * 3 + 1], dx[1], K.J[e * 3] * dx[0]));
      w.gx = g[0];
      w.gy = g[1];
      w.gz = g[2];
      w.l = fma(K.M[0], h00, fma(K.M[1], h11, fma(K.M[2], h22,
            2.0 * fma(K.M[3], h01, fma(K.M[4], h02, K.M[5] * h12)))));
    } else {
      w.gx = w.gy = w.gz = w.l = 0.0;
    }
    w.row = (idx[0] * K.n[1] + idx[1]) * K.n[2] + idx[2];
    W[lane] = w;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int n_orb = K.n_orb;
  const size_t out0 = size_t(p) * n_orb;
  for (int o = VW * lane; o < n_orb; o += 64 * VW) {
    double v[VW], gx[VW], gy[VW], gz[VW], l[VW];
#pragma unroll
    for (int c = 0; c < VW; ++c) v[c] = gx[c] = gy[c] = gz[c] = l[c] = 0.0;
#pragma unroll 8
    for (int r = 0; r < 64; ++r) {
      const BlipW w = W[r];
      const double* src = coef + size_t(w.row) * n_orb + o;
      double a[VW];
      if (VW == 2) {
        const double2 t = *reinterpret_cast<const double2*>(src);
        a[0] = t.x;
        a[VW - 1] = t.y;
      } else {
        a[0] = src[0];
      }
#pragma unroll
      for (int c = 0; c < VW; ++c) {
        v[c] = fma(w.b, a[c], v[c]);
        if (DER) {
          gx[c] = fma(w.gx, a[c], gx[c]);
          gy[c] = fma(w.gy, a[c], gy[c]);
          gz[c] = fma(w.gz, a[c], gz[c]);
          l[c] = fma(w.l, a[c], l[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < VW; ++c) {
      val[out0 + o + c] = v[c];
      if (DER) {
        grad[3 * out0 + o + c] = gx[c];
        grad[3 * out0 + n_orb + o + c] = gy[c];
        grad[3 * out0 + 2 * size_t(n_orb) + o + c] = gz[c];
        lap[out0 + o + c] = l[c];
      }
    }
  }
}

}  // namespace
}  // namespace ewald

extern "C" {

ewald_status ewald_blip_create(const double lattice[3][3], const int grid[3], int n_orb, ewald_blip** out) try {
  if (!out) {
    ewald::set_last_error("out is NULL");
    return EWALD_E_ARG;
  }
  *out = nullptr;
  if (!lattice || !grid) {
    ewald::set_last_error("lattice/grid is NULL");
    return EWALD_E_ARG;
  }
  if (n_orb < 1) {
    ewald::set_last_error("n_orb must be >= 1");
    return EWALD_E_ARG;
  }
  for (int d = 0; d < 3; ++d)
    if (grid[d] < 4 || grid[d] > 4096) {
      ewald::set_last_error("every grid dimension must be in [4, 4096]");
      return EWALD_E_ARG;
    }
  const double* A = &lattice[0][0];
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(A[i])) {
      ewald::set_last_error("non-finite lattice");
      return EWALD_E_LATTICE;
    }
  const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                     A[2] * (A[3] * A[7] - A[4] * A[6]);
  double norm = 1.0;
  for (int i = 0; i < 3; ++i) norm *= std::sqrt(A[3 * i] * A[3 * i] + A[3 * i + 1] * A[3 * i + 1] + A[3 * i + 2] * A[3 * i + 2]);
  if (!(std::fabs(det) > 1e-10 * norm)) {
    ewald::set_last_error("singular lattice");
    return EWALD_E_LATTICE;
  }
  ewald_blip* b = new ewald_blip();
  for (int d = 0; d < 3; ++d) b->grid[d] = grid[d];
  b->n_orb = n_orb;
  // inverse by cofactors: Ainv[e][d] with sum_e A[i][e] Ainv[e][d] = delta_id
  const double c[9] = {A[4] * A[8] - A[5] * A[7], A[2] * A[7] - A[1] * A[8], A[1] * A[5] - A[2] * A[4],
                       A[5] * A[6] - A[3] * A[8], A[0] * A[8] - A[2] * A[6], A[2] * A[3] - A[0] * A[5],
                       A[3] * A[7] - A[4] * A[6], A[1] * A[6] - A[0] * A[7], A[0] * A[4] - A[1] * A[3]};
  for (int i = 0; i < 9; ++i) b->ainv[i] = c[i] / det;
  for (int e = 0; e < 3; ++e)
    for (int d = 0; d < 3; ++d) b->J[e * 3 + d] = b->ainv[e * 3 + d] * grid[d];
  const int pd[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  for (int t = 0; t < 6; ++t) {
    double m = 0.0;
    for (int e = 0; e < 3; ++e) m += b->J[e * 3 + pd[t][0]] * b->J[e * 3 + pd[t][1]];
    b->M[t] = m;
  }
  *out = b;
  return EWALD_OK;
} catch (const std::bad_alloc&) {
  ewald::set_last_error("host allocation failed");
  return EWALD_E_NOMEM;
}

void ewald_blip_destroy(ewald_blip* b) { delete b; }

ewald_status ewald_blip_eval_batch(const ewald_blip* b, const double* coef, int n_points, const double* pos,
                                   double* val, double* grad, double* lap, void* stream) {
  ewald::CallTimer timer("ewald_blip_eval_batch", stream);
  if (!b) {
    ewald::set_last_error("blip handle is NULL");
    return EWALD_E_ARG;
  }
  if (n_points < 0) {
    ewald::set_last_error("n_points must be >= 0");
    return EWALD_E_ARG;
  }
  if (n_points == 0) return EWALD_OK;
  if (!coef || !pos || !val) {
    ewald::set_last_error("coef, pos and val must be non-NULL");
    return EWALD_E_ARG;
  }
  if ((grad == nullptr) != (lap == nullptr)) {
    ewald::set_last_error("grad and lap must be given together");
    return EWALD_E_ARG;
  }
  const bool vec = (b->n_orb % 2) == 0 && (reinterpret_cast<uintptr_t>(coef) % 16) == 0;
  ewald::BlipK K;
  for (int d = 0; d < 3; ++d) K.n[d] = b->grid[d];
  K.n_orb = b->n_orb;
  std::memcpy(K.ainv, b->ainv, sizeof K.ainv);
  std::memcpy(K.J, b->J, sizeof K.J);
  std::memcpy(K.M, b->M, sizeof K.M);
  const dim3 grid_dim((n_points + ewald::BLIP_WAVES - 1) / ewald::BLIP_WAVES);
  const dim3 block(64 * ewald::BLIP_WAVES);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool der = grad != nullptr;
  if (vec && der)
    hipLaunchKernelGGL((ewald::k_blip<2, true>), grid_dim, block, 0, s, K, coef, n_points, pos, val, grad, lap);
  else if (vec)
    hipLaunchKernelGGL((ewald::k_blip<2, false>), grid_dim, block, 0, s, K, coef, n_points, pos, val, grad, lap);
  else if (der)
    hipLaunchKernelGGL((ewald::k_blip<1, true>), grid_dim, block, 0, s, K, coef, n_points, pos, val, grad, lap);
  else
    hipLaunchKernelGGL((ewald::k_blip<1, false>), grid_dim, block, 0, s, K, coef, n_points, pos, val, grad, lap);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ewald::set_last_error(std::string("blip launch failed: ") + hipGetErrorString(e));
    return EWALD_E_HIP;
  }
  return EWALD_OK;
}

}  // extern "C"
