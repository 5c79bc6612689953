// Preprocess (forward and backward) and the workspace fill kernel.
//
// Forward, one lane per Gaussian, for every view:
//  * activations (Sec. 3.1): s = exp(log-scale), normalised quaternion -> R,
//    o = sigmoid(logit);
//  * the view rows of M T (Eq. T_matrix) and the window rows of T' = V P M T;
//  * cull, rho_c = 2 ln(o/tau_alpha) and the inversion-free screen box of
//    Sec. 3.2 (s, f, p_i, h_i), all in float64 so that the tile lists are
//    exact; pixel-centre rect -> tile rect -> instance count;
//  * the affine Pluecker record for the rasterizer and the SH colour.
// The same launch then scans the counts across workgroups (decoupled
// look-back over workgroup tickets), emits the (tile key, Gaussian index)
// instances with a load-balanced loop and adds the radix-sort digit
// histograms of those keys.
//
// Backward, one lane per Gaussian: sums the per-instance partials written by
// the raster backward, converts them from tile-local to camera coordinates
// and applies the chain rule back to means, log-scales, quaternions, opacity
// logits and SH coefficients.
#include <math.h>

#include "common.h"

namespace htgs {

// Orthonormal real spherical harmonics (no Condon-Shortley phase), l <= 3,
// as polynomials of the unit direction.
constexpr double kY00 = 0.28209479177387814;   // 1/(2 sqrt(pi))
constexpr double kY1 = 0.4886025119029199;     // sqrt(3/(4 pi))
constexpr double kY2a = 1.0925484305920792;    // sqrt(15/pi)/2
constexpr double kY2b = 0.31539156525252005;   // sqrt(5/pi)/4
constexpr double kY2c = 0.5462742152960396;    // sqrt(15/pi)/4
constexpr double kY3a = 0.5900435899266435;    // sqrt(35/(2 pi))/4
constexpr double kY3b = 2.890611442640554;     // sqrt(105/pi)/2
constexpr double kY3c = 0.4570457994644658;    // sqrt(21/(2 pi))/4
constexpr double kY3d = 0.3731763325901154;    // sqrt(7/pi)/4
constexpr double kY3e = 1.445305721320277;     // sqrt(105/pi)/4

template <typename T>
__device__ inline void sh_basis(T x, T y, T z, int deg, T *Y) {
  Y[0] = T(kY00);
  if (deg >= 1) {
    Y[1] = T(kY1) * y;
    Y[2] = T(kY1) * z;
    Y[3] = T(kY1) * x;
  }
  if (deg >= 2) {
    Y[4] = T(kY2a) * x * y;
    Y[5] = T(kY2a) * y * z;
    Y[6] = T(kY2b) * (T(3) * z * z - T(1));
    Y[7] = T(kY2a) * x * z;
    Y[8] = T(kY2c) * (x * x - y * y);
  }
  if (deg >= 3) {
    Y[9] = T(kY3a) * y * (T(3) * x * x - y * y);
    Y[10] = T(kY3b) * x * y * z;
    Y[11] = T(kY3c) * y * (T(5) * z * z - T(1));
    Y[12] = T(kY3d) * z * (T(5) * z * z - T(3));
    Y[13] = T(kY3c) * x * (T(5) * z * z - T(1));
    Y[14] = T(kY3e) * z * (x * x - y * y);
    Y[15] = T(kY3a) * x * (x * x - T(3) * y * y);
  }
}

// Gradient of each basis polynomial w.r.t. (x, y, z); only the part
// tangent to the sphere matters, and the caller projects it.
__device__ inline void sh_basis_grad(double x, double y, double z, int deg, double (*dY)[3]) {
  dY[0][0] = dY[0][1] = dY[0][2] = 0.0;
  if (deg >= 1) {
    dY[1][0] = 0; dY[1][1] = kY1; dY[1][2] = 0;
    dY[2][0] = 0; dY[2][1] = 0; dY[2][2] = kY1;
    dY[3][0] = kY1; dY[3][1] = 0; dY[3][2] = 0;
  }
  if (deg >= 2) {
    dY[4][0] = kY2a * y; dY[4][1] = kY2a * x; dY[4][2] = 0;
    dY[5][0] = 0; dY[5][1] = kY2a * z; dY[5][2] = kY2a * y;
    dY[6][0] = 0; dY[6][1] = 0; dY[6][2] = kY2b * 6.0 * z;
    dY[7][0] = kY2a * z; dY[7][1] = 0; dY[7][2] = kY2a * x;
    dY[8][0] = kY2c * 2.0 * x; dY[8][1] = -kY2c * 2.0 * y; dY[8][2] = 0;
  }
  if (deg >= 3) {
    dY[9][0] = kY3a * 6.0 * x * y; dY[9][1] = kY3a * 3.0 * (x * x - y * y); dY[9][2] = 0;
    dY[10][0] = kY3b * y * z; dY[10][1] = kY3b * x * z; dY[10][2] = kY3b * x * y;
    dY[11][0] = 0; dY[11][1] = kY3c * (5.0 * z * z - 1.0); dY[11][2] = kY3c * 10.0 * y * z;
    dY[12][0] = 0; dY[12][1] = 0; dY[12][2] = kY3d * (15.0 * z * z - 3.0);
    dY[13][0] = kY3c * (5.0 * z * z - 1.0); dY[13][1] = 0; dY[13][2] = kY3c * 10.0 * x * z;
    dY[14][0] = kY3e * 2.0 * x * z; dY[14][1] = -kY3e * 2.0 * y * z; dY[14][2] = kY3e * (x * x - y * y);
    dY[15][0] = kY3a * 3.0 * (x * x - y * y); dY[15][1] = -kY3a * 6.0 * x * y; dY[15][2] = 0;
  }
}

// Rotation of the normalised quaternion (w, x, y, z); columns are the
// splat's axes t_u, t_v, t_w.
__device__ inline void quat_to_rot(const double q[4], double R[3][3]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z); R[0][2] = 2 * (x * z + w * y);
  R[1][0] = 2 * (x * y + w * z); R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
  R[2][0] = 2 * (x * z - w * y); R[2][1] = 2 * (y * z + w * x); R[2][2] = 1 - 2 * (x * x + y * y);
}

struct Activated {
  double mu[3], s[3], q[4], qnorm, R[3][3], o;
};

__device__ inline void activate(const GaussPtrs &gp, int64_t g, Activated &a) {
  for (int k = 0; k < 3; ++k) {
    a.mu[k] = (double)gp.means[3 * g + k];
    a.s[k] = exp((double)gp.log_scales[3 * g + k]);
  }
  double qq = 0.0;
  for (int k = 0; k < 4; ++k) {
    a.q[k] = (double)gp.quats[4 * g + k];
    qq += a.q[k] * a.q[k];
  }
  a.qnorm = sqrt(qq);
  double qn[4];
  for (int k = 0; k < 4; ++k) qn[k] = a.q[k] / a.qnorm;
  quat_to_rot(qn, a.R);
  a.o = 1.0 / (1.0 + exp(-(double)gp.logits[g]));
}

// View rows of M T: Rv[k][j] = (W3 R diag(s))_{kj}, mv = W3 mu + t.
__device__ inline void view_rows(const ViewParams &V, const Activated &a, double Rv[3][3],
                                 double mv[3]) {
  for (int k = 0; k < 3; ++k) {
    const double w0 = V.w2c[4 * k + 0], w1 = V.w2c[4 * k + 1], w2 = V.w2c[4 * k + 2];
    mv[k] = w0 * a.mu[0] + w1 * a.mu[1] + w2 * a.mu[2] + (double)V.w2c[4 * k + 3];
    for (int j = 0; j < 3; ++j)
      Rv[k][j] = (w0 * a.R[0][j] + w1 * a.R[1][j] + w2 * a.R[2][j]) * a.s[j];
  }
}

__device__ inline void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ inline double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// One Gaussian in one view: cull, box, rect, record. Returns the instance
// count and writes the tile rect (and the record if the count is non-zero);
// *packed receives tx0 | ty0 << 10 | width << 20 of a non-empty rect.
__device__ inline uint32_t preprocess_view(const GaussPtrs &gp, const KCfg &cfg,
                                           const ViewParams &V, const Ws &w, int v,
                                           int64_t g, const Activated &a, uint32_t *packed) {
  double Rv[3][3], mv[3];
  view_rows(V, a, Rv, mv);
  const double fx = V.fx, fy = V.fy, cx = V.cx, cy = V.cy;
  bool vis = (a.o > (double)cfg.tau_alpha) && (mv[2] > (double)V.z_near);
  const double rc = 2.0 * log(a.o / (double)cfg.tau_alpha);
  // Window rows of T' (x, y and the homogeneous row).
  double T1[3], T2[3];
  for (int j = 0; j < 3; ++j) {
    T1[j] = fx * Rv[0][j] + cx * Rv[2][j];
    T2[j] = fy * Rv[1][j] + cy * Rv[2][j];
  }
  const double T10 = fx * mv[0] + cx * mv[2];
  const double T20 = fy * mv[1] + cy * mv[2];
  const double *T4 = Rv[2];
  const double T40 = mv[2];
  const double sq = rc * dot3(T4, T4) - T40 * T40;
  vis = vis && (sq < 0.0);
  const double p1 = (rc * dot3(T1, T4) - T10 * T40) / sq;
  const double p2 = (rc * dot3(T2, T4) - T20 * T40) / sq;
  const double q1 = (rc * dot3(T1, T1) - T10 * T10) / sq;
  const double q2 = (rc * dot3(T2, T2) - T20 * T20) / sq;
  const double h1 = sqrt(fmax(p1 * p1 - q1, 0.0));
  const double h2 = sqrt(fmax(p2 * p2 - q2, 0.0));
  vis = vis && isfinite(p1) && isfinite(p2) && isfinite(h1) && isfinite(h2);
  int4 rect = make_int4(1, 1, 0, 0);
  uint32_t count = 0;
  double x0 = 0, x1 = -1, y0 = 0, y1 = -1;
  if (vis) {
    x0 = fmax(ceil(p1 - h1 - 0.5), 0.0);
    x1 = fmin(floor(p1 + h1 - 0.5), (double)(V.width - 1));
    y0 = fmax(ceil(p2 - h2 - 0.5), 0.0);
    y1 = fmin(floor(p2 + h2 - 0.5), (double)(V.height - 1));
    if (x0 <= x1 && y0 <= y1) {
      rect.x = (int)x0 / cfg.tile_w;
      rect.y = (int)y0 / cfg.tile_h;
      rect.z = (int)x1 / cfg.tile_w;
      rect.w = (int)y1 / cfg.tile_h;
      count = (uint32_t)((rect.z - rect.x + 1) * (rect.w - rect.y + 1));
    }
  }
  w.rects[(int64_t)v * cfg.n + g] = rect;
  if (count == 0) return 0;
  *packed = (uint32_t)rect.x | ((uint32_t)rect.y << 10) | ((uint32_t)(rect.z - rect.x + 1) << 20);

  // Reference point: the centre of the covered pixel nearest the box centre.
  const double ixd = fmin(fmax(floor(p1), x0), x1);
  const double iyd = fmin(fmax(floor(p2), y0), y1);
  const double uc = (ixd + 0.5 - cx) / fx, vc = (iyd + 0.5 - cy) / fy;
  double D0[3], Du[3], Dv[3];
  cross3(Rv[0], Rv[1], D0);
  cross3(Rv[1], Rv[2], Du);
  cross3(Rv[2], Rv[0], Dv);
  float rec[kRecFloats];
  for (int k = 0; k < 3; ++k) {
    const double M0 = mv[0] * Rv[1][k] - mv[1] * Rv[0][k];
    const double Mu = mv[1] * Rv[2][k] - mv[2] * Rv[1][k];
    const double Mv = mv[2] * Rv[0][k] - mv[0] * Rv[2][k];
    rec[R_D0 + k] = (float)(D0[k] + uc * Du[k] + vc * Dv[k]);
    rec[R_DU + k] = (float)(Du[k] / fx);
    rec[R_DV + k] = (float)(Dv[k] / fy);
    rec[R_M0 + k] = (float)(M0 + uc * Mu + vc * Mv);
    rec[R_MU + k] = (float)(Mu / fx);
    rec[R_MV + k] = (float)(Mv / fy);
    rec[R_R3 + k] = (float)Rv[2][k];
  }
  rec[R_MUZ] = (float)mv[2];
  rec[R_O] = (float)a.o;
  rec[R_RC] = (float)rc;
  rec[R_IX] = __int_as_float((int)ixd);
  rec[R_IY] = __int_as_float((int)iyd);
  rec[R_BB0] = __uint_as_float((uint32_t)x0 | ((uint32_t)y0 << 16));
  rec[R_BB1] = __uint_as_float((uint32_t)x1 | ((uint32_t)y1 << 16));

  // View-dependent colour (Sec. 3.1; 3DGS convention).
  double dv[3] = {a.mu[0] - V.cam_pos[0], a.mu[1] - V.cam_pos[1], a.mu[2] - V.cam_pos[2]};
  const double dn = sqrt(dot3(dv, dv));
  float Y[16];
  sh_basis<float>((float)(dv[0] / dn), (float)(dv[1] / dn), (float)(dv[2] / dn), cfg.sh_degree,
                  Y);
  const int nb = (cfg.sh_degree + 1) * (cfg.sh_degree + 1);
  const float *sh = gp.sh + g * nb * 3;
  uint32_t flags = 0;
  for (int c = 0; c < 3; ++c) {
    float acc = 0.5f;
    for (int k = 0; k < nb; ++k) acc = fmaf(Y[k], sh[3 * k + c], acc);
    if (acc < 0.0f) {
      flags |= 1u << c;
      acc = 0.0f;
    }
    rec[R_RGB + c] = acc;
  }
  rec[R_FLAGS] = __uint_as_float(flags);
  float4 *dst = reinterpret_cast<float4 *>(w.records + ((int64_t)v * cfg.n + g) * kRecFloats);
#pragma unroll
  for (int k = 0; k < kRecFloats / 4; ++k)
    dst[k] = make_float4(rec[4 * k], rec[4 * k + 1], rec[4 * k + 2], rec[4 * k + 3]);
  return count;
}

__global__ void __launch_bounds__(256) k_fill_zero(uint4 *p, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void __launch_bounds__(kPreThreads) k_preprocess(GaussPtrs gp, KCfg cfg, ViewSet vs,
                                                             Ws w) {
  __shared__ uint32_t s_ticket;
  __shared__ uint32_t s_excl[kPreThreads + 1];
  __shared__ uint32_t s_vcnt[kMaxViews][kPreThreads];
  __shared__ uint32_t s_vrect[kMaxViews][kPreThreads];
  __shared__ uint32_t s_hist[4][256];
  __shared__ uint32_t s_wsum[kPreThreads / 64];
  __shared__ unsigned long long s_base;

  const int tid = threadIdx.x;
  if (tid == 0) s_ticket = atomicAdd(&w.status[1], 1u);
  for (int i = tid; i < 4 * 256; i += kPreThreads) (&s_hist[0][0])[i] = 0u;
  __syncthreads();
  const int64_t blk = s_ticket;
  const int64_t g = blk * kPreThreads + tid;

  uint32_t total = 0;
  if (g < cfg.n) {
    Activated a;
    activate(gp, g, a);
    for (int v = 0; v < vs.n; ++v) {
      uint32_t packed = 0;
      const uint32_t c = preprocess_view(gp, cfg, vs.v[v], w, v, g, a, &packed);
      s_vcnt[v][tid] = c;
      s_vrect[v][tid] = packed;
      total += c;
    }
  } else {
    for (int v = 0; v < vs.n; ++v) s_vcnt[v][tid] = 0u;
  }

  // Workgroup exclusive scan of the counts.
  const int lane = tid & 63, wave = tid >> 6;
  uint32_t x = total;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_wsum[wave] = x;
  __syncthreads();
  uint32_t woff = 0;
  for (int k = 0; k < wave; ++k) woff += s_wsum[k];
  const uint32_t incl = x + woff;
  s_excl[tid] = incl - total;
  if (tid == kPreThreads - 1) s_excl[kPreThreads] = incl;
  __syncthreads();
  const uint32_t block_total = s_excl[kPreThreads];

  // Decoupled look-back across workgroups (in ticket order).
  if (tid == 0) {
    unsigned long long excl = 0;
    if (blk == 0) {
      st_rel_u64(&w.pp_look[0], kFlagP64 | block_total);
    } else {
      st_rel_u64(&w.pp_look[blk], kFlagA64 | block_total);
      int64_t j = blk - 1;
      int spins = 0;
      while (true) {
        const unsigned long long s = ld_acq_u64(&w.pp_look[j]);
        const unsigned f = (unsigned)(s >> 62);
        if (f == 0) {
          if (++spins > kSpinLimit) {
            atomicOr(&w.status[0], (uint32_t)ST_SPIN);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += s & kMask64;
        if (f == 2) break;
        --j;
      }
      st_rel_u64(&w.pp_look[blk], kFlagP64 | (excl + block_total));
    }
    s_base = excl;
    if (blk == (int64_t)gridDim.x - 1) {
      const unsigned long long tot = excl + block_total;
      *w.total = tot;
      if (tot > (unsigned long long)w.capacity) atomicOr(&w.status[0], (uint32_t)ST_OVERFLOW);
    }
  }
  __syncthreads();
  const unsigned long long base = s_base;
  if (g < cfg.n) w.offsets[g] = (uint32_t)(base + s_excl[tid]);

  // Emit instances, one per loop iteration, balanced over the workgroup.
  uint16_t *k16 = reinterpret_cast<uint16_t *>(w.keys[0]);
  uint32_t *k32 = reinterpret_cast<uint32_t *>(w.keys[0]);
  for (uint32_t e = tid; e < block_total; e += kPreThreads) {
    int lo = 0, hi = kPreThreads;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_excl[mid] <= e) lo = mid; else hi = mid;
    }
    uint32_t rank = e - s_excl[lo];
    int v = 0;
    while (rank >= s_vcnt[v][lo]) {
      rank -= s_vcnt[v][lo];
      ++v;
    }
    const int64_t gi = blk * kPreThreads + lo;
    const uint32_t pr = s_vrect[v][lo];
    const uint32_t rw = pr >> 20;
    const uint32_t ty = ((pr >> 10) & 1023u) + rank / rw;
    const uint32_t tx = (pr & 1023u) + rank % rw;
    const uint32_t key = (uint32_t)vs.v[v].tile_base + ty * (uint32_t)vs.v[v].tiles_x + tx;
    const unsigned long long pos = base + e;
    if (pos < (unsigned long long)w.capacity) {
      if (w.key16) k16[pos] = (uint16_t)key; else k32[pos] = key;
      w.vals[0][pos] = (uint32_t)gi;
    }
    for (int p = 0; p < w.passes; ++p) atomicAdd(&s_hist[p][(key >> (8 * p)) & 255u], 1u);
  }
  __syncthreads();
  for (int p = 0; p < w.passes; ++p) {
    const uint32_t c = s_hist[p][tid];
    if (c) atomicAdd(&w.hist[p * 256 + tid], c);
  }
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------

__device__ inline void rot_grad_to_quat(const double qn[4], const double gR[3][3], double gq[4]) {
  const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  // d R / d(w, x, y, z) contracted with gR.
  gq[0] = 2 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] +
               x * gR[2][1]);
  gq[1] = 2 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2 * x * gR[1][1] - w * gR[1][2] +
               z * gR[2][0] + w * gR[2][1] - 2 * x * gR[2][2]);
  gq[2] = 2 * (-2 * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] -
               w * gR[2][0] + z * gR[2][1] - 2 * y * gR[2][2]);
  gq[3] = 2 * (-2 * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2 * z * gR[1][1] +
               y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
}

__global__ void __launch_bounds__(256) k_preprocess_bwd(GaussPtrs gp, GradPtrs gr, KCfg cfg,
                                                         ViewSet vs, Ws w) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= cfg.n) return;
  int4 rects[kMaxViews];
  uint32_t total = 0;
  for (int v = 0; v < vs.n; ++v) {
    rects[v] = w.rects[(int64_t)v * cfg.n + g];
    if (rects[v].x <= rects[v].z)
      total += (uint32_t)((rects[v].z - rects[v].x + 1) * (rects[v].w - rects[v].y + 1));
  }
  if (total == 0) return;
  const unsigned long long I = *w.total;
  const uint32_t first = w.offsets[g];
  if ((unsigned long long)first + total > (unsigned long long)w.capacity ||
      (unsigned long long)first + total > I)
    return;  // overflowed forward: status already reports it

  Activated a;
  activate(gp, g, a);
  const int nb = (cfg.sh_degree + 1) * (cfg.sh_degree + 1);
  double gA[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double gmu[3] = {0, 0, 0};
  double go = 0.0;
  double gsh[16][3];
  for (int k = 0; k < 16; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.0;

  uint32_t slot = first;
  for (int v = 0; v < vs.n; ++v) {
    const int4 r = rects[v];
    if (r.x > r.z) continue;
    const ViewParams &V = vs.v[v];
    const double fx = V.fx, fy = V.fy, cx = V.cx, cy = V.cy;
    double gD0[3] = {0, 0, 0}, gDu[3] = {0, 0, 0}, gDv[3] = {0, 0, 0};
    double gM0[3] = {0, 0, 0}, gMu[3] = {0, 0, 0}, gMv[3] = {0, 0, 0};
    double gc[3] = {0, 0, 0};
    for (int ty = r.y; ty <= r.w; ++ty) {
      const double vt = ((double)ty * cfg.tile_h + 0.5 - cy) / fy;
      for (int tx = r.x; tx <= r.z; ++tx, ++slot) {
        const double ut = ((double)tx * cfg.tile_w + 0.5 - cx) / fx;
        const float4 *P = reinterpret_cast<const float4 *>(w.partials + (int64_t)slot * kPartialFloats);
        float pf[kPartialFloats];
#pragma unroll
        for (int k = 0; k < kPartialFloats / 4; ++k) {
          const float4 t = P[k];
          pf[4 * k] = t.x; pf[4 * k + 1] = t.y; pf[4 * k + 2] = t.z; pf[4 * k + 3] = t.w;
        }
        for (int k = 0; k < 3; ++k) {
          const double s0 = pf[P_D0 + k], sx = pf[P_DX + k], sy = pf[P_DY + k];
          gD0[k] += s0;
          gDu[k] += ut * s0 + sx / fx;
          gDv[k] += vt * s0 + sy / fy;
          const double t0 = pf[P_M0 + k], tx_ = pf[P_MX + k], ty_ = pf[P_MY + k];
          gM0[k] += t0;
          gMu[k] += ut * t0 + tx_ / fx;
          gMv[k] += vt * t0 + ty_ / fy;
          gc[k] += pf[P_C + k];
        }
        go += pf[P_O];
      }
    }
    // Pluecker coefficients -> view rows of M T.
    double Rv[3][3], mv[3];
    view_rows(V, a, Rv, mv);
    double gR[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double gm[3] = {0, 0, 0};
    double t[3];
    // D0 = R1 x R2, Du = R2 x R3, Dv = R3 x R1 (rows R1..R3 of Rv)
    cross3(Rv[1], gD0, t); for (int k = 0; k < 3; ++k) gR[0][k] += t[k];
    cross3(gD0, Rv[0], t); for (int k = 0; k < 3; ++k) gR[1][k] += t[k];
    cross3(Rv[2], gDu, t); for (int k = 0; k < 3; ++k) gR[1][k] += t[k];
    cross3(gDu, Rv[1], t); for (int k = 0; k < 3; ++k) gR[2][k] += t[k];
    cross3(Rv[0], gDv, t); for (int k = 0; k < 3; ++k) gR[2][k] += t[k];
    cross3(gDv, Rv[2], t); for (int k = 0; k < 3; ++k) gR[0][k] += t[k];
    // M0 = m0 R2 - m1 R1, Mu = m1 R3 - m2 R2, Mv = m2 R1 - m0 R3
    for (int k = 0; k < 3; ++k) {
      gR[1][k] += mv[0] * gM0[k];
      gR[0][k] -= mv[1] * gM0[k];
      gR[2][k] += mv[1] * gMu[k];
      gR[1][k] -= mv[2] * gMu[k];
      gR[0][k] += mv[2] * gMv[k];
      gR[2][k] -= mv[0] * gMv[k];
    }
    gm[0] += dot3(gM0, Rv[1]) - dot3(gMv, Rv[2]);
    gm[1] += dot3(gMu, Rv[2]) - dot3(gM0, Rv[0]);
    gm[2] += dot3(gMv, Rv[0]) - dot3(gMu, Rv[1]);
    // Rv = W3 A (A = R diag(s)), mv = W3 mu + t
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += (double)V.w2c[4 * k + i] * gR[k][j];
        gA[i][j] += acc;
      }
      double accm = 0.0;
      for (int k = 0; k < 3; ++k) accm += (double)V.w2c[4 * k + i] * gm[k];
      gmu[i] += accm;
    }
    // Colour: SH coefficients and the viewing direction.
    const uint32_t flags =
        __float_as_uint(w.records[((int64_t)v * cfg.n + g) * kRecFloats + R_FLAGS]);
    for (int c = 0; c < 3; ++c)
      if (flags & (1u << c)) gc[c] = 0.0;
    double dv[3] = {a.mu[0] - V.cam_pos[0], a.mu[1] - V.cam_pos[1], a.mu[2] - V.cam_pos[2]};
    const double dn = sqrt(dot3(dv, dv));
    const double dir[3] = {dv[0] / dn, dv[1] / dn, dv[2] / dn};
    double Y[16], dY[16][3];
    sh_basis<double>(dir[0], dir[1], dir[2], cfg.sh_degree, Y);
    sh_basis_grad(dir[0], dir[1], dir[2], cfg.sh_degree, dY);
    const float *sh = gp.sh + g * nb * 3;
    double gdir[3] = {0, 0, 0};
    for (int k = 0; k < nb; ++k) {
      double wsum = 0.0;
      for (int c = 0; c < 3; ++c) {
        gsh[k][c] += Y[k] * gc[c];
        wsum += (double)sh[3 * k + c] * gc[c];
      }
      for (int j = 0; j < 3; ++j) gdir[j] += wsum * dY[k][j];
    }
    const double radial = dot3(gdir, dir);
    for (int j = 0; j < 3; ++j) gmu[j] += (gdir[j] - dir[j] * radial) / dn;
  }
  // A = R diag(s): to rotation, scales and quaternion.
  double gRot[3][3], gs[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      gRot[i][j] = gA[i][j] * a.s[j];
      gs[j] += gA[i][j] * a.R[i][j];
    }
  double qn[4];
  for (int k = 0; k < 4; ++k) qn[k] = a.q[k] / a.qnorm;
  double gqn[4];
  rot_grad_to_quat(qn, gRot, gqn);
  const double proj = qn[0] * gqn[0] + qn[1] * gqn[1] + qn[2] * gqn[2] + qn[3] * gqn[3];

  if (gr.means)
    for (int k = 0; k < 3; ++k) gr.means[3 * g + k] += (float)gmu[k];
  if (gr.log_scales)
    for (int k = 0; k < 3; ++k) gr.log_scales[3 * g + k] += (float)(gs[k] * a.s[k]);
  if (gr.quats)
    for (int k = 0; k < 4; ++k) gr.quats[4 * g + k] += (float)((gqn[k] - qn[k] * proj) / a.qnorm);
  if (gr.logits) gr.logits[g] += (float)(go * a.o * (1.0 - a.o));
  if (gr.sh)
    for (int k = 0; k < nb; ++k)
      for (int c = 0; c < 3; ++c) gr.sh[(g * nb + k) * 3 + c] += (float)gsh[k][c];
}

hipError_t launch_fill_zero(void *p, int64_t bytes, hipStream_t s) {
  const int64_t n16 = bytes / 16;
  if (n16 <= 0) return hipSuccess;
  int blocks = (int)((n16 + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, reinterpret_cast<uint4 *>(p), n16);
  return hipGetLastError();
}

hipError_t launch_preprocess(const GaussPtrs &gp, const KCfg &cfg, const ViewSet &vs, const Ws &w,
                             hipStream_t s) {
  if (cfg.n == 0) return hipSuccess;
  const int blocks = (int)((cfg.n + kPreThreads - 1) / kPreThreads);
  hipLaunchKernelGGL(k_preprocess, dim3(blocks), dim3(kPreThreads), 0, s, gp, cfg, vs, w);
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const GaussPtrs &gp, const GradPtrs &gr, const KCfg &cfg,
                                 const ViewSet &vs, const Ws &w, hipStream_t s) {
  if (cfg.n == 0) return hipSuccess;
  const int blocks = (int)((cfg.n + 255) / 256);
  hipLaunchKernelGGL(k_preprocess_bwd, dim3(blocks), dim3(256), 0, s, gp, gr, cfg, vs, w);
  return hipGetLastError();
}

}  // namespace htgs
