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
// A one-workgroup launch then scans the workgroups' instance totals, and an
// emit launch writes the (tile key, Gaussian index) instances with a
// load-balanced loop and adds the radix-sort digit histograms of those
// keys. No workgroup waits for another.
//
// Backward: a slot-parallel segmented reduction sums the per-instance
// partials of each (Gaussian, view); then one lane per Gaussian applies the
// chain rule back to means, log-scales, quaternions, opacity logits and SH
// coefficients.
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

// Unfiltered scale and opacity: the activations of Sec. 3.1, or the baked
// values themselves.
__device__ __forceinline__ double raw_scale(const GaussPtrs &gp, const KCfg &cfg, int64_t g,
                                            int k) {
  const double x = (double)gp.log_scales[3 * g + k];
  return cfg.baked ? x : exp(x);
}
__device__ __forceinline__ double raw_opacity(const GaussPtrs &gp, const KCfg &cfg, int64_t g) {
  const double x = (double)gp.logits[g];
  return cfg.baked ? x : 1.0 / (1.0 + exp(-x));
}

// s = exp(log-scale), R from the normalised quaternion, o = sigmoid(logit)
// (baked inputs: s, the unit quaternion and o as given). With the 3D filter
// (variance f per Gaussian, Mip-Splatting as used in Sec. 4.2) the
// covariance R diag(s^2) R^T gets f I added: s' = sqrt(s^2 + f) along the
// same axes, o' = o prod s/s' (the peak of the convolved density).
__device__ inline void activate(const GaussPtrs &gp, const KCfg &cfg, int64_t g, Activated &a) {
  for (int k = 0; k < 3; ++k) {
    a.mu[k] = (double)gp.means[3 * g + k];
    a.s[k] = raw_scale(gp, cfg, g, k);
  }
  double qq = 0.0;
  for (int k = 0; k < 4; ++k) {
    a.q[k] = (double)gp.quats[4 * g + k];
    qq += a.q[k] * a.q[k];
  }
  a.qnorm = cfg.baked ? 1.0 : sqrt(qq);
  const double iq = 1.0 / a.qnorm;
  double qn[4];
  for (int k = 0; k < 4; ++k) qn[k] = a.q[k] * iq;
  quat_to_rot(qn, a.R);
  a.o = raw_opacity(gp, cfg, g);
  if (gp.filter_var) {
    const double f = (double)gp.filter_var[g];
    for (int k = 0; k < 3; ++k) {
      const double sf = sqrt(a.s[k] * a.s[k] + f);
      a.o *= sf > 0.0 ? a.s[k] / sf : 1.0;
      a.s[k] = sf;
    }
  }
}

// What the backward's view loop needs of an activated Gaussian: the mean
// and A = R diag(s) (the rest is recomputed after the loop, which keeps
// fewer registers live while the partials are summed).
struct ViewAct {
  double mu[3], A[3][3];
};

__device__ inline void view_act(const Activated &a, ViewAct &va) {
  for (int k = 0; k < 3; ++k) {
    va.mu[k] = a.mu[k];
    for (int j = 0; j < 3; ++j) va.A[k][j] = a.R[k][j] * a.s[j];
  }
}

// View rows of M T from A = R diag(s): Rv = W3 A, mv = W3 mu + t.
__device__ inline void view_rows_va(const ViewParams &V, const ViewAct &va, double Rv[3][3],
                                    double mv[3]) {
  for (int k = 0; k < 3; ++k) {
    const double w0 = V.w2c[4 * k + 0], w1 = V.w2c[4 * k + 1], w2 = V.w2c[4 * k + 2];
    mv[k] = w0 * va.mu[0] + w1 * va.mu[1] + w2 * va.mu[2] + (double)V.w2c[4 * k + 3];
    for (int j = 0; j < 3; ++j) Rv[k][j] = w0 * va.A[0][j] + w1 * va.A[1][j] + w2 * va.A[2][j];
  }
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

// The NF = 3 (DEG+1)^2 SH coefficients of one Gaussian: 16-byte accesses
// where the row is a multiple of 16 bytes (degrees 1 and 3), so that a
// wave's loads cover whole cache lines instead of one line per lane.
template <int NF>
__device__ __forceinline__ void load_row(const float *__restrict__ src, float *dst) {
  if constexpr (NF % 4 == 0) {
    const float4 *s4 = reinterpret_cast<const float4 *>(src);
#pragma unroll
    for (int i = 0; i < NF / 4; ++i) {
      const float4 t = s4[i];
      dst[4 * i] = t.x; dst[4 * i + 1] = t.y; dst[4 * i + 2] = t.z; dst[4 * i + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < NF; ++i) dst[i] = src[i];
  }
}

template <int NF>
__device__ __forceinline__ void add_row(float *dst, const float *v) {
  if constexpr (NF % 4 == 0) {
    float4 *d4 = reinterpret_cast<float4 *>(dst);
#pragma unroll
    for (int i = 0; i < NF / 4; ++i) {
      float4 t = d4[i];
      t.x += v[4 * i]; t.y += v[4 * i + 1]; t.z += v[4 * i + 2]; t.w += v[4 * i + 3];
      d4[i] = t;
    }
  } else {
#pragma unroll
    for (int i = 0; i < NF; ++i) dst[i] += v[i];
  }
}

// Inclusive maximum and sum over the lanes of a wave by DPP moves (shifts
// by 1, 2, 4, 8 inside each row of 16 lanes, then the row ends broadcast
// to the rows after them); lanes whose source is outside receive 0. Every
// lane of the wave must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_move_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, false);
}
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x) {
  x = max(x, dpp_move_u32<0x111, 0xf>(x));
  x = max(x, dpp_move_u32<0x112, 0xf>(x));
  x = max(x, dpp_move_u32<0x114, 0xf>(x));
  x = max(x, dpp_move_u32<0x118, 0xf>(x));
  x = max(x, dpp_move_u32<0x142, 0xa>(x));
  x = max(x, dpp_move_u32<0x143, 0xc>(x));
  return x;
}
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
  x += dpp_move_u32<0x111, 0xf>(x);
  x += dpp_move_u32<0x112, 0xf>(x);
  x += dpp_move_u32<0x114, 0xf>(x);
  x += dpp_move_u32<0x118, 0xf>(x);
  x += dpp_move_u32<0x142, 0xa>(x);
  x += dpp_move_u32<0x143, 0xc>(x);
  return x;
}

// x / d for 0 <= x < 2^16 and 1 <= d <= 1024 (pixel index by tile size):
// x and d are exact in float32 and the product with the reciprocal is off
// by at most one, which one remainder test corrects (an integer division
// by a value not known at compile time is a sequence of ~15 instructions).
__device__ __forceinline__ int div_px(int x, int d) {
  int q = (int)((float)x * __builtin_amdgcn_rcpf((float)d));
  const int r = x - q * d;
  if (r < 0) --q;
  else if (r >= d) ++q;
  return q;
}

// Tiles of a screen box that the splat's rho_c-ellipse reaches. With the
// Pluecker vectors affine in the pixel offset (p, q) from the reference
// pixel, d = Dc + p Dx + q Dy and m = Mc + p Mx + q My, a pixel is a fragment
// iff Q(p, q) = |m|^2 - rho_c |d|^2 <= 0. Q is a quadratic in (p, q); for a
// splat in front of the camera its quadratic part is positive definite, so
// its minimum over a tile's rectangle of pixel centres is the free minimum
// if that lies inside, else the smallest of the four edge minima. A tile is
// kept if that minimum is <= 0 for rho_c enlarged by 0.1% (float32
// evaluation in the rasterizer cannot move a pixel across that margin).
// *valid is false (keep every tile) when the quadratic part is not clearly
// positive definite.
struct Conic {
  double A, B, C, Dpp, Epq, Fqq;  // Q = A + 2Bp + 2Cq + Dpp p^2 + 2Epq pq + Fqq q^2
};

__device__ inline Conic make_conic(const double Dc[3], const double Dx[3], const double Dy[3],
                                   const double Mc[3], const double Mx[3], const double My[3],
                                   double rc) {
  const double r = rc * 1.001;
  Conic c;
  c.A = dot3(Mc, Mc) - r * dot3(Dc, Dc);
  c.B = dot3(Mc, Mx) - r * dot3(Dc, Dx);
  c.C = dot3(Mc, My) - r * dot3(Dc, Dy);
  c.Dpp = dot3(Mx, Mx) - r * dot3(Dx, Dx);
  c.Epq = dot3(Mx, My) - r * dot3(Dx, Dy);
  c.Fqq = dot3(My, My) - r * dot3(Dy, Dy);
  return c;
}

__device__ __forceinline__ double conic_at(const Conic &c, double p, double q) {
  return c.A + 2.0 * (c.B * p + c.C * q) + c.Dpp * p * p + 2.0 * c.Epq * p * q + c.Fqq * q * q;
}

// Bits of the rect's tiles (row-major) that the ellipse Q <= 0 reaches.
// Tile rows are handled one at a time: over a row's band of pixel-centre
// rows q in [qa, qb] (offsets from the reference pixel, clipped to the
// covered pixel rect), the ellipse spans p from its left boundary's minimum
// to its right boundary's maximum; the left boundary is convex in q, so its
// minimum over the band is at the band point nearest the ellipse's
// leftmost point (likewise on the right). The pixel-centre columns in that
// span give the row's tiles. The conic is unusable (every tile stays) when
// its quadratic part is not clearly positive definite.
//
// The rows of a wave's Gaussians are tested by the whole wave: each lane
// puts its Gaussian's ellipse extent in LDS (cull_setup), then the (lane,
// tile row) pairs are dealt to the lanes in windows of 64 (wave_cull_rows).
// With each lane looping over its own rows, most lanes sat idle: in a 1080p
// frame a wave's Gaussians have ~2 tile rows on average and ~8 at most.
struct CullExt {                  // one lane's ellipse extent (104 bytes)
  double A, B, C, Dpp, Epq, Fqq;  // the conic
  double idp;                     // 1 / Dpp
  double qmin, qmax;              // q extent of the ellipse
  double qL, qR;                  // q of its leftmost and rightmost points
  uint32_t xs, ys;                // covered pixel rect: x0 | x1 << 16, y0 | y1 << 16
  uint32_t ref;                   // reference pixel ix | iy << 16
  uint32_t trect;                 // first tile column | first tile row << 16
};
struct CullLds {
  CullExt ext[64];
  unsigned long long mask[64];    // kept tiles
  uint32_t mark[64];              // see wave_cull_rows
};

// This lane's part of the cull: whether the conic is usable (*valid) and,
// if the ellipse is not empty, its extent in s; returns the number of tile
// rows to test (0: none; with a usable conic and an empty ellipse no tile
// is kept).
__device__ inline uint32_t cull_setup(const Conic &c, int4 rect, double x0, double x1,
                                      double y0, double y1, double ixd, double iyd, CullLds &s,
                                      int lane, bool *valid) {
  const double det = c.Dpp * c.Fqq - c.Epq * c.Epq;
  *valid = c.Dpp > 0.0 && c.Fqq > 0.0 && det > 1e-9 * c.Dpp * c.Fqq;
  if (!*valid) return 0u;
  const double idet = 1.0 / det;
  const double ps = (c.Epq * c.C - c.Fqq * c.B) * idet, qs = (c.Epq * c.B - c.Dpp * c.C) * idet;
  const double Q0 = conic_at(c, ps, qs);
  if (!(Q0 < 0.0)) return 0u;  // empty ellipse: no fragment anywhere
  const double hp = sqrt(-Q0 * c.Fqq * idet), hq = sqrt(-Q0 * c.Dpp * idet);
  const double eh = c.Epq * hp / c.Fqq;
  CullExt e;
  e.A = c.A; e.B = c.B; e.C = c.C; e.Dpp = c.Dpp; e.Epq = c.Epq; e.Fqq = c.Fqq;
  e.idp = 1.0 / c.Dpp;
  e.qmin = qs - hq;
  e.qmax = qs + hq;
  e.qL = qs + eh;
  e.qR = qs - eh;
  // (the covered rect and reference pixel are integers below 2^16)
  e.xs = (uint32_t)x0 | ((uint32_t)x1 << 16);
  e.ys = (uint32_t)y0 | ((uint32_t)y1 << 16);
  e.ref = (uint32_t)ixd | ((uint32_t)iyd << 16);
  e.trect = (uint32_t)rect.x | ((uint32_t)rect.y << 16);
  s.ext[lane] = e;
  return (uint32_t)(rect.w - rect.y + 1);
}

// Tile row k of a rect with extent e, w tiles wide: its kept tiles at
// their bits of the rect's mask.
__device__ inline unsigned long long cull_row(const CullExt &e, int k, int w, int tw, int th) {
  const double x0 = (double)(e.xs & 0xffffu), x1 = (double)(e.xs >> 16);
  const double y0 = (double)(e.ys & 0xffffu), y1 = (double)(e.ys >> 16);
  const double ixd = (double)(e.ref & 0xffffu), iyd = (double)(e.ref >> 16);
  const int rx = (int)(e.trect & 0xffffu), ty = (int)(e.trect >> 16) + k;
  const double a = fmax(fmax((double)(ty * th), y0) - iyd, e.qmin);
  const double b = fmin(fmin((double)(ty * th + th - 1), y1) - iyd, e.qmax);
  if (a > b) return 0ull;
  // p extent of the ellipse on the line q: pc(q) +- sqrt(disc(q)) / Dpp
  auto side = [&](double q, double sgn) {
    const double bq = e.B + e.Epq * q;
    const double disc = bq * bq - e.Dpp * (e.A + 2.0 * e.C * q + e.Fqq * q * q);
    return (-bq + sgn * sqrt(fmax(disc, 0.0))) * e.idp;
  };
  const double pl = side(fmin(fmax(e.qL, a), b), -1.0);
  const double pr = side(fmin(fmax(e.qR, a), b), 1.0);
  const double xlo = fmax(ceil(pl + ixd), x0), xhi = fmin(floor(pr + ixd), x1);
  if (xlo > xhi) return 0ull;
  const int t0 = div_px((int)xlo, tw) - rx, t1 = div_px((int)xhi, tw) - rx;
  const unsigned long long run = ((2ull << (t1 - t0)) - 1ull) << t0;
  return run << (k * w);
}

// The kept-tile mask of every lane's rect (rows: tile rows to test, 0 for
// lanes without a cull; w: the rect's width in tiles). All 64 lanes of the
// wave take part. Pair e of the wave (pairs in lane order, rows in order
// inside a lane) goes to lane e mod 64 of window e / 64. Its owner is the
// last lane whose first pair is at or before e: each lane whose first pair
// lies in the window marks that place with (first pair, width, lane + 1),
// and a max-scan over the window, seeded with the previous window's last
// owner, spreads the marks (the first pairs grow with the lane).
__device__ inline unsigned long long wave_cull_rows(CullLds &s, uint32_t rows, uint32_t w,
                                                   int tw, int th, int lane) {
  const uint32_t incl = wave_incl_sum(rows);
  const uint32_t first = incl - rows;   // < 4096
  const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  s.mask[lane] = 0ull;
  const uint32_t tag = (first << 14) | (w << 7) | ((uint32_t)lane + 1u);
  uint32_t carry = 0u;   // the previous window's last owner tag
  for (uint32_t e0 = 0; e0 < total; e0 += 64u) {
    s.mark[lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    if (rows && first >= e0 && first < e0 + 64u) s.mark[first - e0] = tag;
    __builtin_amdgcn_wave_barrier();
    uint32_t m = s.mark[lane];
    if (lane == 0) m = max(m, carry);
    const uint32_t own = wave_incl_max(m);
    carry = (uint32_t)__builtin_amdgcn_readlane((int)own, 63);
    const uint32_t e = e0 + (uint32_t)lane;
    if (e < total && (own & 127u) != 0u) {
      const int o = (int)(own & 127u) - 1;
      const int k = (int)(e - (own >> 14));
      const unsigned long long bits = cull_row(s.ext[o], k, (int)((own >> 7) & 127u), tw, th);
      if (bits) atomicOr(&s.mask[o], bits);
    }
    __builtin_amdgcn_wave_barrier();
  }
  return s.mask[lane];
}

// State of one (view, Gaussian) between its own work and the wave's cull.
struct ViewPending {
  int4 rect;        // tile rect
  uint32_t count;   // its tiles
  bool finish;      // visible: the rect, descriptor and count are still to be written
  bool cull;        // tiles to be culled with the wave's masks
  bool valid;       // the cull's conic is usable
  uint32_t rows;    // tile rows for the wave to test
  uint32_t width;   // the rect's width in tiles
};

// One Gaussian in one view: cull, box, rect, record, colour, and the
// lane's part of the tile cull (in cl). A Gaussian that is not visible
// gets its empty rect here (finish false); the others are finished by
// preprocess_view_end once the wave's cull masks are known.
template <int DEG, bool CULL>
__device__ inline ViewPending preprocess_view(const GaussPtrs &gp, const KCfg &cfg,
                                              const ViewParams &V, const Ws &w, int v,
                                              int64_t g, const Activated &a, CullLds &cl,
                                              int lane) {
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
      rect.x = div_px((int)x0, cfg.tile_w);
      rect.y = div_px((int)y0, cfg.tile_h);
      rect.z = div_px((int)x1, cfg.tile_w);
      rect.w = div_px((int)y1, cfg.tile_h);
      count = (uint32_t)((rect.z - rect.x + 1) * (rect.w - rect.y + 1));
    }
  }
  const int64_t vg = (int64_t)v * cfg.n + g;
  ViewPending pv{rect, count, false, false, false, 0u, (uint32_t)(rect.z - rect.x + 1)};
  if (count == 0) {
    w.rects[vg] = rect;
    w.cflags[vg] = 0u;   // not visible in this view
    return pv;
  }

  // Reference point: the centre of the covered pixel nearest the box centre.
  // (Divisions by the focal lengths are products with their reciprocals:
  // a float64 division is a sequence of about ten instructions at the
  // float64 rate, and these values are rounded to float32 or only decide
  // a conservative tile test.)
  const double ixd = fmin(fmax(floor(p1), x0), x1);
  const double iyd = fmin(fmax(floor(p2), y0), y1);
  const double ifx = 1.0 / fx, ify = 1.0 / fy;
  const double uc = (ixd + 0.5 - cx) * ifx, vc = (iyd + 0.5 - cy) * ify;
  // Pluecker vectors affine in the pixel offset: d = Dc + p Dx + q Dy,
  // m = Mc + p Mx + q My.
  double Dc[3], Dx[3], Dy[3], Mc[3], Mx[3], My[3];
  {
    double D0[3], Du[3], Dv[3];
    cross3(Rv[0], Rv[1], D0);
    cross3(Rv[1], Rv[2], Du);
    cross3(Rv[2], Rv[0], Dv);
    for (int k = 0; k < 3; ++k) {
      const double M0 = mv[0] * Rv[1][k] - mv[1] * Rv[0][k];
      const double Mu = mv[1] * Rv[2][k] - mv[2] * Rv[1][k];
      const double Mv = mv[2] * Rv[0][k] - mv[0] * Rv[2][k];
      Dc[k] = D0[k] + uc * Du[k] + vc * Dv[k];
      Dx[k] = Du[k] * ifx;
      Dy[k] = Dv[k] * ify;
      Mc[k] = M0 + uc * Mu + vc * Mv;
      Mx[k] = Mu * ifx;
      My[k] = Mv * ify;
    }
  }
  // Tile culling works on the float64 conic of the footprint; the tiles are
  // tested after the record is written, when few other values are live.
  const bool cull = CULL && count >= 2u && count <= 64u;
  Conic conic{};
  if (cull) conic = make_conic(Dc, Dx, Dy, Mc, Mx, My, rc);
  // The geometric part of the record is stored first so that its registers
  // are free before the colour is evaluated.
  float rec[24];
  for (int k = 0; k < 3; ++k) {
    rec[R_D0 + k] = (float)Dc[k];
    rec[R_DU + k] = (float)Dx[k];
    rec[R_DV + k] = (float)Dy[k];
    rec[R_M0 + k] = (float)Mc[k];
    rec[R_MU + k] = (float)Mx[k];
    rec[R_MV + k] = (float)My[k];
    rec[R_R3 + k] = (float)Rv[2][k];
  }
  rec[R_MUZ] = (float)mv[2];
  rec[R_O] = (float)a.o;
  rec[R_RC] = (float)rc;
  float4 *dst = reinterpret_cast<float4 *>(w.records + ((int64_t)v * cfg.n + g) * kRecFloats);
#pragma unroll
  for (int k = 0; k < 6; ++k)
    dst[k] = make_float4(rec[4 * k], rec[4 * k + 1], rec[4 * k + 2], rec[4 * k + 3]);
  w.refpix[vg] = (uint32_t)ixd | ((uint32_t)iyd << 16);
  dst[R_IX / 4] = make_float4(__int_as_float((int)ixd), __int_as_float((int)iyd),
                              __uint_as_float((uint32_t)x0 | ((uint32_t)y0 << 16)),
                              __uint_as_float((uint32_t)x1 | ((uint32_t)y1 << 16)));

  // View-dependent colour (Sec. 3.1; 3DGS convention).
  double dv[3] = {a.mu[0] - V.cam_pos[0], a.mu[1] - V.cam_pos[1], a.mu[2] - V.cam_pos[2]};
  const double idn = 1.0 / sqrt(dot3(dv, dv));
  constexpr int NB = (DEG + 1) * (DEG + 1), NF = 3 * NB;
  float Y[16];
  sh_basis<float>((float)(dv[0] * idn), (float)(dv[1] * idn), (float)(dv[2] * idn), DEG, Y);
  float coef[NF];
  load_row<NF>(gp.sh + g * NF, coef);
  uint32_t flags = 0;
  float col[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float acc = 0.5f;
#pragma unroll
    for (int k = 0; k < NB; ++k) acc = fmaf(Y[k], coef[3 * k + c], acc);
    if (acc < 0.0f) {
      flags |= 1u << c;
      acc = 0.0f;
    }
    col[c] = acc;
  }
  dst[R_RGB / 4] = make_float4(col[0], col[1], col[2], __uint_as_float(flags));
  w.cflags[(int64_t)v * cfg.n + g] = (uint8_t)(flags | kCflagVisible);

  pv.finish = true;
  pv.cull = cull;
  if (cull) pv.rows = cull_setup(conic, rect, x0, x1, y0, y1, ixd, iyd, cl, lane, &pv.valid);
  return pv;
}

// The rest of a visible (view, Gaussian) once the wave's cull masks are
// known (cmask: this lane's): returns the instance count and writes the
// tile rect; *packed receives tx0 | ty0 << 10 | width << 20 of a non-empty
// rect and *mask_out the surviving tiles of the rect (0 = all).
__device__ inline uint32_t preprocess_view_end(const Ws &w, int64_t vg, const ViewPending &pv,
                                               unsigned long long cmask, uint32_t *packed,
                                               unsigned long long *mask_out) {
  uint32_t count = pv.count;
  int4 rect = pv.rect;
  unsigned long long mask = 0ull;
  if (pv.cull && pv.valid) {
    mask = cmask;
    const uint32_t kept = (uint32_t)__popcll(mask);
    // every tile kept: no mask (the emit then skips the set-bit search)
    if (kept == count) mask = 0ull;
    count = kept;
  }
  if (count == 0) rect = make_int4(1, 1, 0, 0);
  w.rects[vg] = rect;
  *mask_out = mask;
  if (count) {
    *packed =
        (uint32_t)rect.x | ((uint32_t)rect.y << 10) | ((uint32_t)(rect.z - rect.x + 1) << 20);
  }
  return count;
}

__global__ void __launch_bounds__(256) k_fill_zero(uint4 *p, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Position pos of the list the front end walks holds Gaussian g: the index
// itself, or, for sorted blending, the Gaussian at that place of the
// front-to-back order (so instances are emitted in that order, and the
// stable tile sort keeps it inside each tile). False past the end.
__device__ __forceinline__ bool gaussian_at(const Ws &w, const KCfg &cfg, int64_t pos,
                                            int64_t &g) {
  g = pos;
  if (pos >= cfg.n) return false;
  if (w.perm) {
    const uint32_t x = w.perm[pos];
    if ((int64_t)x >= cfg.n) return false;
    g = (int64_t)x;
  }
  return true;
}

// Per Gaussian and view (MV: more than one view, which keeps more values
// live; CULL: tile culling of small boxes): the record, the rect, the
// colour flags and a tile-slot descriptor whose first word holds the
// instance count for now (the emit launch replaces it by the first slot);
// per workgroup the instance total, for the scan of the totals.
template <int DEG, bool MV, bool CULL>
__global__ void __launch_bounds__(kPreThreads) k_preprocess(GaussPtrs gp, KCfg cfg, ViewSet vs,
                                                             Ws w) {
  __shared__ unsigned long long s_wsum[kPreThreads / 64];
  __shared__ CullLds s_cull[CULL ? kPreThreads / 64 : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t blk = blockIdx.x;
  int64_t g;
  const bool live = gaussian_at(w, cfg, blk * kPreThreads + tid, g);
  const int nviews = MV ? vs.n : 1;
  unsigned long long total = 0;
  Activated a;
  if (live) activate(gp, cfg, g, a);
  CullLds &cl = s_cull[CULL ? wave : 0];
  for (int v = 0; v < nviews; ++v) {
    ViewPending pv{make_int4(1, 1, 0, 0), 0u, false, false, false, 0u, 0u};
    if (live) pv = preprocess_view<DEG, CULL>(gp, cfg, vs.v[v], w, v, g, a, cl, lane);
    // (every lane of the wave takes part in the cull, live or not)
    unsigned long long cmask = 0ull;
    if constexpr (CULL)
      cmask = wave_cull_rows(cl, pv.rows, pv.width, cfg.tile_w, cfg.tile_h, lane);
    if (live) {
      uint32_t c = 0, packed = 0;
      unsigned long long mk = 0ull;
      if (pv.finish) c = preprocess_view_end(w, (int64_t)v * cfg.n + g, pv, cmask, &packed, &mk);
      w.tslots[(int64_t)v * cfg.n + g] =
          c ? make_uint4(c, packed, (uint32_t)mk, (uint32_t)(mk >> 32)) : make_uint4(0u, 0u, 0u, 0u);
      total += c;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) total += __shfl_xor(total, off, 64);
  if (lane == 0) s_wsum[wave] = total;
  __syncthreads();
  if (tid == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int k = 0; k < kPreThreads / 64; ++k) t += s_wsum[k];
    w.pp_total[blk] = t;
  }
}

// Exclusive scan of the workgroup totals, in place, by one workgroup; the
// sum is the instance count, which raises the overflow flag when it
// exceeds the capacity.
constexpr int kTotScanThreads = 1024, kTotScanItems = 4;
__global__ void __launch_bounds__(kTotScanThreads) k_preprocess_scan(Ws w, int64_t nblk) {
  __shared__ unsigned long long s_wsum[kTotScanThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  unsigned long long carry = 0;
  for (int64_t b0 = 0; b0 < nblk; b0 += (int64_t)kTotScanThreads * kTotScanItems) {
    const int64_t bb = b0 + (int64_t)tid * kTotScanItems;
    unsigned long long v[kTotScanItems], sum = 0;
#pragma unroll
    for (int j = 0; j < kTotScanItems; ++j) {
      v[j] = bb + j < nblk ? w.pp_total[bb + j] : 0ull;
      sum += v[j];
    }
    unsigned long long inc = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned long long y = __shfl_up(inc, off, 64);
      if (lane >= off) inc += y;
    }
    __syncthreads();   // the previous round's readers of s_wsum are done
    if (lane == 63) s_wsum[wave] = inc;
    __syncthreads();
    unsigned long long run = carry + inc - sum;
    for (int k = 0; k < wave; ++k) run += s_wsum[k];
#pragma unroll
    for (int j = 0; j < kTotScanItems; ++j) {
      if (bb + j < nblk) w.pp_total[bb + j] = run;
      run += v[j];
    }
    for (int k = 0; k < kTotScanThreads / 64; ++k) carry += s_wsum[k];
  }
  if (tid == 0) {
    *w.total = carry;
    if (carry > (unsigned long long)w.capacity) atomicOr(&w.status[0], (uint32_t)ST_OVERFLOW);
  }
}

// The instances of the workgroup's Gaussians (the same 256 positions as the
// preprocess launch), written from its first slot on, and the radix-sort
// digit histograms of their keys. Slot layout: the workgroup's 64-Gaussian
// groups (one per wave) in order; inside a group view by view, inside a
// view Gaussian by Gaussian, inside a (view, Gaussian) tile by tile.
// s_start holds the workgroup-relative first slot of every (group, view,
// lane), in slot order, plus the workgroup total at the end; it first holds
// the counts. The tile-slot descriptors get their first slots here.
template <bool MV>
__global__ void __launch_bounds__(kPreThreads) k_emit(KCfg cfg, ViewSet vs, Ws w) {
  constexpr int NVL = MV ? kMaxViews : 1;
  __shared__ uint32_t s_start[NVL * kPreThreads + 1];
  __shared__ uint32_t s_vrect[NVL][kPreThreads];
  __shared__ unsigned long long s_vmask[NVL][kPreThreads];
  // (the batched form's per-view tables leave room for one copy)
  constexpr int HC = MV ? 1 : kHistLaneCopies;
  __shared__ uint32_t s_hist[4][HC * kHistPadWords];
  __shared__ uint32_t s_wsum[kPreThreads / 64];
  __shared__ uint32_t s_gidx[kPreThreads];
  __shared__ uint32_t s_mark[kPreThreads / 64][64];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t blk = blockIdx.x;
  for (int i = tid; i < 4 * HC * kHistPadWords; i += kPreThreads) (&s_hist[0][0])[i] = 0u;
  int64_t g;
  const bool live = gaussian_at(w, cfg, blk * kPreThreads + tid, g);
  s_gidx[tid] = (uint32_t)g;
  const int nviews = MV ? vs.n : 1;
  for (int v = 0; v < nviews; ++v) {
    const uint4 ts = live ? w.tslots[(int64_t)v * cfg.n + g] : make_uint4(0u, 0u, 0u, 0u);
    s_start[(wave * nviews + v) * 64 + lane] = ts.x;
    s_vrect[v][tid] = ts.y;
    s_vmask[v][tid] = (unsigned long long)ts.z | ((unsigned long long)ts.w << 32);
  }

  // Group-relative starts: a wave scan per view, the views one after
  // another (each lane reads and writes only its own entries).
  uint32_t gsum = 0;
  for (int v = 0; v < nviews; ++v) {
    uint32_t *e = &s_start[(wave * nviews + v) * 64 + lane];
    const uint32_t c = *e;
    uint32_t x = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    *e = gsum + x - c;
    gsum += (uint32_t)__shfl(x, 63, 64);
  }
  if (lane == 0) s_wsum[wave] = gsum;
  __syncthreads();
  uint32_t goff = 0, block_total = 0;
#pragma unroll
  for (int k = 0; k < kPreThreads / 64; ++k) {
    if (k < wave) goff += s_wsum[k];
    block_total += s_wsum[k];
  }
  for (int v = 0; v < nviews; ++v) s_start[(wave * nviews + v) * 64 + lane] += goff;
  const int nent = kPreThreads * nviews;
  if (tid == 0) s_start[nent] = block_total;
  __syncthreads();
  const unsigned long long base = w.pp_total[blk];

  if (live) {
    // First slot of each (view, Gaussian), clamped at 2^31 so that base +
    // rank cannot wrap (slots at or past the capacity are never written).
    for (int v = 0; v < nviews; ++v) {
      const int f = (wave * nviews + v) * 64 + lane;
      const unsigned long long m = s_vmask[v][tid];
      w.tslots[(int64_t)v * cfg.n + g] =
          make_uint4((uint32_t)min(base + s_start[f], 0x80000000ull), s_vrect[v][tid],
                     (uint32_t)m, (uint32_t)(m >> 32));
    }
  }

  // Instances to memory in windows of 64 consecutive instances, each wave
  // taking every fourth window. Instance e belongs to the last (group,
  // view, lane) entry starting at or before it. The owner of a window's
  // first instance comes from a 64-way search (two rounds of one LDS read
  // per lane and a ballot); every later entry that starts inside the window
  // marks the lane of its first instance with its distance from that owner,
  // and an inclusive max-scan of the marks gives each lane its owner.
  uint16_t *k16 = reinterpret_cast<uint16_t *>(w.keys[0]);
  uint32_t *k32 = reinterpret_cast<uint32_t *>(w.keys[0]);
  // instances e < room fit below the capacity
  const unsigned long long cap = (unsigned long long)w.capacity;
  const uint32_t room =
      base >= cap ? 0u : (uint32_t)min(cap - base, (unsigned long long)0xffffffffu);
  for (uint32_t e0 = (uint32_t)wave * 64u; e0 < block_total; e0 += kPreThreads) {
    int lo = 0, hi = nent;   // s_start[lo] <= e0 < s_start[hi]
    while (hi - lo > 1) {
      const int step = (hi - lo + 63) >> 6;
      const int idx = lo + lane * step;
      const bool t = idx < hi && s_start[idx] <= e0;
      const uint64_t bal = __ballot(t);
      const int last = 63 - (int)__builtin_clzll(bal);   // lane 0 always holds
      lo += last * step;
      hi = min(lo + step, hi);
    }
    s_mark[wave][lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    for (int jb = lo + 1; jb < nent; jb += 64) {
      const int j = jb + lane;
      const uint32_t st = j < nent ? s_start[j] : 0xffffffffu;
      if (st < e0 + 64u) atomicMax(&s_mark[wave][st - e0], (uint32_t)(j - lo));
      if (__ballot(st >= e0 + 64u)) break;   // later entries start later still
    }
    __builtin_amdgcn_wave_barrier();
    const int ent = lo + (int)wave_incl_max(s_mark[wave][lane]);
    const uint32_t e = e0 + (uint32_t)lane;
    const bool valid = e < block_total;
    uint32_t rank = valid ? e - s_start[ent] : 0u;
    const int grp = ent / (64 * nviews);
    const int v = MV ? (ent >> 6) - grp * nviews : 0;
    const int owner = grp * 64 + (ent & 63);
    const uint32_t gid = s_gidx[owner];
    const uint32_t pr = s_vrect[v][owner];
    const uint32_t rw = pr >> 20;
    // With a tile mask, the rank-th surviving tile is the rank-th set bit:
    // the half that holds it, then halving widths.
    const unsigned long long mk = s_vmask[v][owner];
    if (mk) {
      const uint32_t mlo = (uint32_t)mk, plo = (uint32_t)__popc(mlo);
      const bool in_lo = rank < plo;
      uint32_t m = in_lo ? mlo : (uint32_t)(mk >> 32);
      uint32_t k = in_lo ? rank : rank - plo;
      uint32_t pos = in_lo ? 0u : 32u;
#pragma unroll
      for (int wd = 16; wd >= 1; wd >>= 1) {
        const uint32_t c = (uint32_t)__popc(m & ((1u << wd) - 1u));
        if (k >= c) {
          k -= c;
          m >>= wd;
          pos += (uint32_t)wd;
        }
      }
      rank = pos;
    }
    // rank / rw and rank % rw; rank < 2^20 and rw <= 1024 are exact in
    // float32, and the quotient estimate is off by at most one
    int qy = (int)((float)rank * __builtin_amdgcn_rcpf((float)rw));
    int rx = (int)rank - qy * (int)rw;
    if (rx < 0) { --qy; rx += (int)rw; }
    if (rx >= (int)rw) { ++qy; rx -= (int)rw; }
    const uint32_t ty = ((pr >> 10) & 1023u) + (uint32_t)qy;
    const uint32_t tx = (pr & 1023u) + (uint32_t)rx;
    const uint32_t key = (uint32_t)vs.v[v].tile_base + ty * (uint32_t)vs.v[v].tiles_x + tx;
    // (one add per lane, spread over HC copies: the wave-level paths of
    // wave_hist_add cost the emit more than the conflicts they avoid)
    if (valid)
      for (int p = 0; p < w.passes; ++p)
        atomicAdd(&s_hist[p][(lane % HC) * kHistPadWords + ((key >> (8 * p)) & 255u)], 1u);
    if (valid && e < room) {
      if (w.key16) k16[base + e] = (uint16_t)key; else k32[base + e] = key;
      w.vals[0][base + e] = gid;
    }
  }
  __syncthreads();
  uint32_t *hist = hist_copy(w.hist);
  for (int p = 0; p < w.passes; ++p) {
    const uint32_t c = hist_total<HC>(s_hist[p], tid);
    if (c) atomicAdd(&hist[p * 256 + tid], c);
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

// One step of the wave-wide segmented inclusive scan of the partial
// values: lanes enabled by ROW_MASK take the DPP-moved value (CTRL) when
// the source lane holds the same segment id. Lanes with no source lane keep
// the complement of their own id, which never matches.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_scan_step(uint32_t seg, float *v) {
  const uint32_t src = (uint32_t)__builtin_amdgcn_update_dpp((int)~seg, (int)seg, CTRL, ROW_MASK,
                                                             0xf, false);
  const bool take = src == seg;
#pragma unroll
  for (int k = 0; k < kPartialFloats; ++k) {
    const float y = __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v[k]), CTRL, ROW_MASK, 0xf, false));
    v[k] += take ? y : 0.f;
  }
}

// ws[k] = sh_k . gc for the NB basis functions of one Gaussian, reading the
// coefficient row four basis functions (three 16-byte loads) at a time
// where the row allows it.
template <int NB>
__device__ __forceinline__ void sh_dots(const float *__restrict__ row, const double gcd[3],
                                        float *ws) {
  const float g0 = (float)gcd[0], g1 = (float)gcd[1], g2 = (float)gcd[2];
  if constexpr ((3 * NB) % 12 == 0) {
    const float4 *r4 = reinterpret_cast<const float4 *>(row);
#pragma unroll
    for (int j = 0; j < NB / 4; ++j) {
      const float4 a = r4[3 * j], b = r4[3 * j + 1], c = r4[3 * j + 2];
      const float t[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
#pragma unroll
      for (int q = 0; q < 4; ++q)
        ws[4 * j + q] = fmaf(t[3 * q + 2], g2, fmaf(t[3 * q + 1], g1, t[3 * q] * g0));
    }
  } else {
#pragma unroll
    for (int k = 0; k < NB; ++k)
      ws[k] = fmaf(row[3 * k + 2], g2, fmaf(row[3 * k + 1], g1, row[3 * k] * g0));
  }
}

// Writes (overwrite) or adds the gradients of Gaussian g.
template <int NB>
__device__ __forceinline__ void emit_grads(const GradPtrs &gr, int64_t g, const float gmu[3],
                                           const float gls[3], const float gq[4], float glogit,
                                           const float *gsh, bool overwrite) {
  if (overwrite) {
    if (gr.means)
      for (int k = 0; k < 3; ++k) gr.means[3 * g + k] = gmu[k];
    if (gr.log_scales)
      for (int k = 0; k < 3; ++k) gr.log_scales[3 * g + k] = gls[k];
    if (gr.quats)
      reinterpret_cast<float4 *>(gr.quats)[g] = make_float4(gq[0], gq[1], gq[2], gq[3]);
    if (gr.logits) gr.logits[g] = glogit;
    if (gr.sh) {
      float *dst = gr.sh + g * NB * 3;
      if constexpr ((3 * NB) % 4 == 0) {
        float4 *d4 = reinterpret_cast<float4 *>(dst);
#pragma unroll
        for (int i = 0; i < 3 * NB / 4; ++i)
          d4[i] = make_float4(gsh[4 * i], gsh[4 * i + 1], gsh[4 * i + 2], gsh[4 * i + 3]);
      } else {
#pragma unroll
        for (int i = 0; i < 3 * NB; ++i) dst[i] = gsh[i];
      }
    }
  } else {
    if (gr.means)
      for (int k = 0; k < 3; ++k) gr.means[3 * g + k] += gmu[k];
    if (gr.log_scales)
      for (int k = 0; k < 3; ++k) gr.log_scales[3 * g + k] += gls[k];
    if (gr.quats) {
      float4 t = reinterpret_cast<float4 *>(gr.quats)[g];
      t.x += gq[0]; t.y += gq[1]; t.z += gq[2]; t.w += gq[3];
      reinterpret_cast<float4 *>(gr.quats)[g] = t;
    }
    if (gr.logits) gr.logits[g] += glogit;
    if (gr.sh) add_row<3 * NB>(gr.sh + g * NB * 3, gsh);
  }
}

// SH backward for one view, straight-line for a fixed degree: adds
// Y_k(dir) * gc to gsh[k] and ws_k grad Y_k(dir) to gdir (ws_k = sh_k . gc).
template <int DEG>
__device__ __forceinline__ void sh_backward(const float *wsv, const double dir[3],
                                            const double gc[3], float *gsh, double gdir[3]) {
  const double x = dir[0], y = dir[1], z = dir[2];
#define HTGS_SH_TERM(k, Yv, gx, gy, gz)                                                     \
  {                                                                                         \
    const double Yk = (Yv);                                                                 \
    gsh[3 * (k)] += (float)(Yk * gc[0]);                                                    \
    gsh[3 * (k) + 1] += (float)(Yk * gc[1]);                                                \
    gsh[3 * (k) + 2] += (float)(Yk * gc[2]);                                                \
    const double ws = (double)wsv[k];                                                      \
    gdir[0] += ws * (gx);                                                                   \
    gdir[1] += ws * (gy);                                                                   \
    gdir[2] += ws * (gz);                                                                   \
  }
  HTGS_SH_TERM(0, kY00, 0.0, 0.0, 0.0)
  if constexpr (DEG >= 1) {
    HTGS_SH_TERM(1, kY1 * y, 0.0, kY1, 0.0)
    HTGS_SH_TERM(2, kY1 * z, 0.0, 0.0, kY1)
    HTGS_SH_TERM(3, kY1 * x, kY1, 0.0, 0.0)
  }
  if constexpr (DEG >= 2) {
    HTGS_SH_TERM(4, kY2a * x * y, kY2a * y, kY2a * x, 0.0)
    HTGS_SH_TERM(5, kY2a * y * z, 0.0, kY2a * z, kY2a * y)
    HTGS_SH_TERM(6, kY2b * (3.0 * z * z - 1.0), 0.0, 0.0, kY2b * 6.0 * z)
    HTGS_SH_TERM(7, kY2a * x * z, kY2a * z, 0.0, kY2a * x)
    HTGS_SH_TERM(8, kY2c * (x * x - y * y), kY2c * 2.0 * x, -kY2c * 2.0 * y, 0.0)
  }
  if constexpr (DEG >= 3) {
    HTGS_SH_TERM(9, kY3a * y * (3.0 * x * x - y * y), kY3a * 6.0 * x * y,
                 kY3a * 3.0 * (x * x - y * y), 0.0)
    HTGS_SH_TERM(10, kY3b * x * y * z, kY3b * y * z, kY3b * x * z, kY3b * x * y)
    HTGS_SH_TERM(11, kY3c * y * (5.0 * z * z - 1.0), 0.0, kY3c * (5.0 * z * z - 1.0),
                 kY3c * 10.0 * y * z)
    HTGS_SH_TERM(12, kY3d * z * (5.0 * z * z - 3.0), 0.0, 0.0, kY3d * (15.0 * z * z - 3.0))
    HTGS_SH_TERM(13, kY3c * x * (5.0 * z * z - 1.0), kY3c * (5.0 * z * z - 1.0), 0.0,
                 kY3c * 10.0 * x * z)
    HTGS_SH_TERM(14, kY3e * z * (x * x - y * y), kY3e * 2.0 * x * z, -kY3e * 2.0 * y * z,
                 kY3e * (x * x - y * y))
    HTGS_SH_TERM(15, kY3a * x * (x * x - 3.0 * y * y), kY3a * 3.0 * (x * x - y * y),
                 -kY3a * 6.0 * x * y, 0.0)
  }
#undef HTGS_SH_TERM
}


// Each wave owns 64 consecutive Gaussians (one slot group: their instance
// slots are one contiguous range, view by view). For each view the wave
// walks that view's part of the range 64 slots at a time with the
// segmented scan and adds each segment's sum into its owner's LDS column,
// so the partials are read once, coalesced. A slot's owner is the last
// Gaussian of the group whose first slot is at or before it (first slots
// increase with the Gaussian): each owner marks its first slot in LDS and
// a prefix maximum over the chunk fills the rest. Then every lane turns its
// Gaussian's summed moments for the view into gradients of the Pluecker
// coefficients (float64) and those into parameter gradients.
template <int DEG, bool MV>
__global__ void __launch_bounds__(256, MV ? 2 : 1) k_preprocess_bwd(GaussPtrs gp, GradPtrs gr, KCfg cfg,
                                                         ViewSet vs, Ws w) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  __shared__ float s_acc[4][kPartialFloats][64];
  __shared__ int s_own[4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pos0 = pos - lane;
  if (pos0 >= cfg.n) return;  // uniform over the wave
  const int nviews = MV ? vs.n : 1;
  const unsigned long long I = *w.total;
  // An overflowed forward (reported by the status word) leaves no usable
  // partials: zero gradient.
  const bool ok = I <= (unsigned long long)w.capacity && !front_failed(w);
  // Sorted blending emitted the instances in the depth order of its
  // Gaussians (position p holds Gaussian perm[p]), so a group of 64
  // positions owns one contiguous slot range; otherwise positions are
  // Gaussian indices. (Without usable partials the index order serves.)
  const bool by_perm = w.perm != nullptr && ok;
  auto gauss_at = [&](int64_t p) -> int64_t {
    if (!by_perm) return p;
    const uint32_t x = w.perm[p];
    return (int64_t)x < cfg.n ? (int64_t)x : p;
  };
  const bool live = pos < cfg.n;
  const int64_t g = live ? gauss_at(pos) : pos;
  uint32_t total = 0;
  if (live && ok)
    for (int v = 0; v < nviews; ++v)
      total += (uint32_t)tile_count(w.rects[(int64_t)v * cfg.n + g],
                                    tslot_mask(w.tslots[(int64_t)v * cfg.n + g]));

  ViewAct va;
  if (total) {
    Activated a0;
    activate(gp, cfg, g, a0);
    view_act(a0, va);
  }
  // per-view terms are formed in float64 and summed over the views in
  // float32 (at most 16 terms), which keeps fewer registers live
  float gA[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  float gmu[3] = {0, 0, 0};
  float go = 0.f;
  // densification statistic: sum over views of |dL_v/dmu| |mu - c_v| / 2
  float dstat = 0.f;
  const bool want_stat = gr.mean_grad_stat != nullptr;   // uniform
  float gsh[3 * NB];
#pragma unroll
  for (int k = 0; k < 3 * NB; ++k) gsh[k] = 0.f;
  const float *shrow = gp.sh + g * NB * 3;

  if (ok && __ballot(total != 0) != 0ull) {
    const int64_t gfirst = gauss_at(pos0);
    const uint64_t group_end =
        (pos0 + 64 < cfg.n) ? (uint64_t)w.tslots[gauss_at(pos0 + 64)].x : (uint64_t)I;
    for (int v = 0; v < nviews; ++v) {
      const uint64_t lo = w.tslots[(int64_t)v * cfg.n + gfirst].x;
      const uint64_t hi = min((v + 1 < nviews) ? (uint64_t)w.tslots[(int64_t)(v + 1) * cfg.n + gfirst].x
                                               : group_end, (uint64_t)I);
      if (lo >= hi) continue;  // no instance of this group in view v
#pragma unroll
      for (int k = 0; k < kPartialFloats; ++k) s_acc[wave][k][lane] = 0.f;
      // this lane's Gaussian in view v: first slot, instance count
      const uint4 myd = live ? w.tslots[(int64_t)v * cfg.n + g] : make_uint4(0u, 0u, 0u, 0u);
      const uint32_t mycnt =
          (live && total) ? (uint32_t)tile_count(w.rects[(int64_t)v * cfg.n + g], tslot_mask(myd)) : 0u;
      __builtin_amdgcn_wave_barrier();
      // Partials of slot sl (zeros past the range).
      auto load_partial = [&](uint64_t sl, float *pv) {
        if (sl < hi) {
          const float4 *P = reinterpret_cast<const float4 *>(w.partials + (int64_t)sl * kPartialFloats);
#pragma unroll
          for (int k = 0; k < kPartialFloats / 4; ++k) {
            const float4 t = P[k];
            pv[4 * k] = t.x; pv[4 * k + 1] = t.y; pv[4 * k + 2] = t.z; pv[4 * k + 3] = t.w;
          }
        } else {
#pragma unroll
          for (int k = 0; k < kPartialFloats; ++k) pv[k] = 0.f;
        }
      };
      // The next 64 slots are loaded while this chunk is scanned.
      float nv[kPartialFloats];
      load_partial(lo + lane, nv);
      int carry = -1;   // owner of the slot before the chunk
      for (uint64_t base = lo; base < hi; base += 64) {
        const uint64_t sl = base + lane;
        const bool valid = sl < hi;
        float pv[kPartialFloats];
#pragma unroll
        for (int k = 0; k < kPartialFloats; ++k) pv[k] = nv[k];
        if (base + 64 < hi) load_partial(base + 64 + lane, nv);
        // owners: marks at first slots, then a prefix maximum
        s_own[wave][lane] = -1;
        __builtin_amdgcn_wave_barrier();
        if (mycnt && (uint64_t)myd.x >= base && (uint64_t)myd.x < base + 64)
          s_own[wave][myd.x - base] = lane;
        __builtin_amdgcn_wave_barrier();
        int own = max(s_own[wave][lane], carry);
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const int y = __shfl_up(own, off, 64);
          if (lane >= off) own = max(own, y);
        }
        carry = __shfl(own, 63, 64);
        const uint32_t seg = valid ? (uint32_t)own : 0xffffffffu;
        // Inclusive segmented scan over the wave with DPP lane moves (no
        // LDS): shifts by 1, 2, 4, 8 inside each row of 16 lanes, then the
        // last lane of row 0 / row 2 into rows 1 / 3, then lane 31 into rows
        // 2 and 3. Segments are runs of consecutive slots, so equal owners
        // mean one run; the fixed tree makes the sums deterministic.
        seg_scan_step<0x111, 0xf>(seg, pv);   // row_shr:1
        seg_scan_step<0x112, 0xf>(seg, pv);   // row_shr:2
        seg_scan_step<0x114, 0xf>(seg, pv);   // row_shr:4
        seg_scan_step<0x118, 0xf>(seg, pv);   // row_shr:8
        seg_scan_step<0x142, 0xa>(seg, pv);   // row_bcast:15 into rows 1, 3
        seg_scan_step<0x143, 0xc>(seg, pv);   // row_bcast:31 into rows 2, 3
        const uint32_t sn = __shfl_down(seg, 1, 64);
        const bool end = valid && own >= 0 && (lane == 63 || sn != seg || sl + 1 == hi);
        if (end) {
#pragma unroll
          for (int k = 0; k < kPartialFloats; ++k) s_acc[wave][k][own] += pv[k];
        }
        __builtin_amdgcn_wave_barrier();
      }
      __builtin_amdgcn_wave_barrier();
      if (mycnt) {
        float acc[kPartialFloats];
#pragma unroll
        for (int k = 0; k < kPartialFloats; ++k) acc[k] = s_acc[wave][k][lane];
        const ViewParams &V = vs.v[v];
        // Pluecker coefficients in camera coordinates (d = D + u Du + v Dv,
        // u = (x + 1/2 - cx) / fx) and, from the summed moments about the
        // record's reference pixel (ox, oy), the loss gradients w.r.t. them.
        double Rv[3][3], mv[3];
        view_rows_va(V, va, Rv, mv);
        double D[3][3], M[3][3];   // [D or M][0: constant, 1: u, 2: v][xyz]
        cross3(Rv[0], Rv[1], D[0]);
        cross3(Rv[1], Rv[2], D[1]);
        cross3(Rv[2], Rv[0], D[2]);
        for (int k = 0; k < 3; ++k) {
          M[0][k] = mv[0] * Rv[1][k] - mv[1] * Rv[0][k];
          M[1][k] = mv[1] * Rv[2][k] - mv[2] * Rv[1][k];
          M[2][k] = mv[2] * Rv[0][k] - mv[0] * Rv[2][k];
        }
        const uint32_t rp = w.refpix[(int64_t)v * cfg.n + g];
        const double ox = (double)(rp & 0xffffu), oy = (double)(rp >> 16);
        const double ifx = 1.0 / (double)V.fx, ify = 1.0 / (double)V.fy;
        const double uo = (ox + 0.5 - (double)V.cx) * ifx, vo = (oy + 0.5 - (double)V.cy) * ify;
        double gD0[3], gDu[3], gDv[3], gM0[3], gMu[3], gMv[3], gc[3];
        for (int h = 0; h < 2; ++h) {
          const double(*C)[3] = h ? M : D;
          const float *m = acc + (h ? P_MM : P_MD);
          double *g0v = h ? gM0 : gD0, *guv = h ? gMu : gDu, *gvv = h ? gMv : gDv;
          for (int k = 0; k < 3; ++k) {
            // the vector at the origin pixel and its steps per pixel
            const double c0 = C[0][k] + uo * C[1][k] + vo * C[2][k];
            const double cx_ = C[1][k] * ifx, cy_ = C[2][k] * ify;
            const double s0 = c0 * m[0] + cx_ * m[1] + cy_ * m[2];
            const double sx = c0 * m[1] + cx_ * m[3] + cy_ * m[4];
            const double sy = c0 * m[2] + cx_ * m[4] + cy_ * m[5];
            g0v[k] = s0;
            guv[k] = uo * s0 + sx * ifx;
            gvv[k] = vo * s0 + sy * ify;
          }
        }
        for (int k = 0; k < 3; ++k) gc[k] = acc[P_C + k];
        go += acc[P_O];
        // Pluecker coefficients -> view rows of M T.
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
        double gmv[3];   // this view's dL/dmu
        // Rv = W3 A (A = R diag(s)), mv = W3 mu + t
        for (int i = 0; i < 3; ++i) {
          for (int j = 0; j < 3; ++j) {
            double s_ = 0.0;
            for (int k = 0; k < 3; ++k) s_ += (double)V.w2c[4 * k + i] * gR[k][j];
            gA[i][j] += (float)s_;
          }
          double sm = 0.0;
          for (int k = 0; k < 3; ++k) sm += (double)V.w2c[4 * k + i] * gm[k];
          gmv[i] = sm;
        }
        // Colour: SH coefficients and the viewing direction.
        const uint32_t flags = w.cflags[(int64_t)v * cfg.n + g];
        for (int c = 0; c < 3; ++c)
          if (flags & (1u << c)) gc[c] = 0.0;
        double dv[3] = {va.mu[0] - V.cam_pos[0], va.mu[1] - V.cam_pos[1],
                        va.mu[2] - V.cam_pos[2]};
        const double dn = sqrt(dot3(dv, dv));
        const double dir[3] = {dv[0] / dn, dv[1] / dn, dv[2] / dn};
        double gdir[3] = {0, 0, 0};
        float wsv[NB];
        sh_dots<NB>(shrow, gc, wsv);
        sh_backward<DEG>(wsv, dir, gc, gsh, gdir);
        const double radial = dot3(gdir, dir);
        for (int j = 0; j < 3; ++j) {
          gmv[j] += (gdir[j] - dir[j] * radial) / dn;
          gmu[j] += (float)gmv[j];
        }
        if (want_stat) dstat += (float)(sqrt(dot3(gmv, gmv)) * dn * 0.5);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (!live) return;
  if (ok) {
    // running sums for densification: always added to (they gather over
    // training steps), views counted where the screen box holds a pixel
    if (want_stat) gr.mean_grad_stat[g] += dstat;
    if (gr.visible_count) {
      float nvis = 0.f;
      for (int v = 0; v < nviews; ++v)
        nvis += (w.cflags[(int64_t)v * cfg.n + g] & kCflagVisible) ? 1.f : 0.f;
      gr.visible_count[g] += nvis;
    }
  }
  if (total == 0) {
    if (cfg.grad_overwrite) {
      const float z[4] = {0.f, 0.f, 0.f, 0.f};
      float zsh[3 * NB];
#pragma unroll
      for (int k = 0; k < 3 * NB; ++k) zsh[k] = 0.f;
      emit_grads<NB>(gr, g, z, z, z, 0.f, zsh, true);
    }
    return;
  }
  // A = R diag(s): to rotation, scales and quaternion.
  Activated a;
  activate(gp, cfg, g, a);
  double gRot[3][3], gs[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      gRot[i][j] = gA[i][j] * a.s[j];
      gs[j] += gA[i][j] * a.R[i][j];
    }
  // d(log-scale) and d(logit). Unfiltered: s = exp(l), o = sigmoid(x), so
  // dL/dl = s dL/ds and dL/dx = o (1 - o) dL/do. Through the 3D filter
  // (s' = sqrt(s^2 + f), o' = o0 prod s/s'): dL/dl_k = dL/ds'_k s_k^2 / s'_k
  // + dL/do' o' f / s'_k^2, and dL/dx = dL/do' o' (1 - o0).
  double gl[3], glogit;
  if (gp.filter_var) {
    const double f = (double)gp.filter_var[g];
    const double o0 = raw_opacity(gp, cfg, g);
    for (int k = 0; k < 3; ++k) {
      const double s0 = raw_scale(gp, cfg, g, k), sf = a.s[k];
      gl[k] = sf > 0.0 ? gs[k] * s0 * s0 / sf + (double)go * a.o * f / (sf * sf) : 0.0;
    }
    glogit = (double)go * a.o * (1.0 - o0);
  } else {
    for (int k = 0; k < 3; ++k) gl[k] = gs[k] * a.s[k];
    glogit = (double)go * a.o * (1.0 - a.o);
  }
  const double iq = 1.0 / a.qnorm;
  double qn[4];
  for (int k = 0; k < 4; ++k) qn[k] = a.q[k] * iq;
  double gqn[4];
  rot_grad_to_quat(qn, gRot, gqn);
  const double proj = qn[0] * gqn[0] + qn[1] * gqn[1] + qn[2] * gqn[2] + qn[3] * gqn[3];

  float fmu[3], fls[3], fq[4];
  for (int k = 0; k < 3; ++k) {
    fmu[k] = (float)gmu[k];
    fls[k] = (float)gl[k];
  }
  for (int k = 0; k < 4; ++k) fq[k] = (float)((gqn[k] - qn[k] * proj) * iq);
  emit_grads<NB>(gr, g, fmu, fls, fq, (float)glogit, gsh, cfg.grad_overwrite != 0);
}

// Opacity decay (Sec. 4.2): o <- lambda o on the logits, x' =
// logit(lambda sigmoid(x)), in float64 from the two exact rearrangements
// x' = log lambda - log(e^-x + 1 - lambda) (x >= 0) and
// x' = x + log lambda - log1p((1 - lambda) e^x) (x < 0), which stay finite
// for every finite x.
__global__ void __launch_bounds__(256) k_opacity_decay(float *x, int64_t n, double log_lam,
                                                        double one_minus_lam) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double v = (double)x[i];
    const double r = v >= 0.0 ? log_lam - log(exp(-v) + one_minus_lam)
                              : v + log_lam - log1p(one_minus_lam * exp(v));
    x[i] = (float)r;
  }
}

hipError_t launch_opacity_decay(float *x, int64_t n, double lambda, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_opacity_decay, dim3(blocks), dim3(256), 0, s, x, n, log(lambda),
                     1.0 - lambda);
  return hipGetLastError();
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
#define HTGS_PRE3(D, M, C)                                                                 \
  hipLaunchKernelGGL((k_preprocess<D, M, C>), dim3(blocks), dim3(kPreThreads), 0, s, gp, cfg, vs, w)
#define HTGS_PRE(D)                                                                        \
  do {                                                                                     \
    if (vs.n > 1) {                                                                        \
      if (cfg.tile_cull) HTGS_PRE3(D, true, true); else HTGS_PRE3(D, true, false);         \
    } else {                                                                               \
      if (cfg.tile_cull) HTGS_PRE3(D, false, true); else HTGS_PRE3(D, false, false);       \
    }                                                                                      \
  } while (0)
  switch (cfg.sh_degree) {
    case 0: HTGS_PRE(0); break;
    case 1: HTGS_PRE(1); break;
    case 2: HTGS_PRE(2); break;
    default: HTGS_PRE(3); break;
  }
#undef HTGS_PRE
#undef HTGS_PRE3
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_preprocess_scan, dim3(1), dim3(kTotScanThreads), 0, s, w, (int64_t)blocks);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (vs.n > 1)
    hipLaunchKernelGGL(k_emit<true>, dim3(blocks), dim3(kPreThreads), 0, s, cfg, vs, w);
  else
    hipLaunchKernelGGL(k_emit<false>, dim3(blocks), dim3(kPreThreads), 0, s, cfg, vs, w);
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const GaussPtrs &gp, const GradPtrs &gr, const KCfg &cfg,
                                 const ViewSet &vs, const Ws &w, hipStream_t s) {
  if (cfg.n == 0) return hipSuccess;
  const int blocks = (int)((cfg.n + 255) / 256);
  switch (cfg.sh_degree) {
#define HTGS_PREB(D)                                                                       \
  do {                                                                                     \
    if (vs.n > 1)                                                                          \
      hipLaunchKernelGGL((k_preprocess_bwd<D, true>), dim3(blocks), dim3(256), 0, s, gp, gr, \
                         cfg, vs, w);                                                      \
    else                                                                                   \
      hipLaunchKernelGGL((k_preprocess_bwd<D, false>), dim3(blocks), dim3(256), 0, s, gp, gr, \
                         cfg, vs, w);                                                      \
  } while (0)
    case 0: HTGS_PREB(0); break;
    case 1: HTGS_PREB(1); break;
    case 2: HTGS_PREB(2); break;
    default: HTGS_PREB(3); break;
  }
#undef HTGS_PREB
  return hipGetLastError();
}

}  // namespace htgs
