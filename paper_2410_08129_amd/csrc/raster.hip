// Tile rasterizer, forward and backward (Sec. 3.2 and Sec. 3.3).
//
// Forward: one workgroup per tile; each wave owns an 8x8 pixel block, one
// lane per pixel. The tile's instances are staged through LDS in batches of
// one record per lane; each wave then keeps only the staged splats whose
// covered pixel rect meets its block and walks them. For the Pluecker
// direction d and moment m of its pixel ray in splat space, rho^2 =
// |m|^2/|d|^2 (Eq. rho-pluecker), alpha = min(alpha_max, o exp(-rho^2/2)),
// and for fragments with alpha >= tau_K the view depth of the
// maximum-density point z = (M T [(d x m)/|d|^2; 1])_z (Sec. 3.3); since d
// and m are affine in the pixel offset, |d|^2, |m|^2 and R3 . (d x m) are
// quadratics in it, staged per (tile, splat) and evaluated per pixel. The
// fragments enter a register core of K (depth, list position) entries kept
// sorted by a median-of-three / select shift. Every fragment is
// added to running sums (sum alpha, sum alpha rgb, prod (1 - alpha)); at
// the end the core members are taken back out of them, which leaves the
// order-independent tail of everything that never entered the core or fell
// off its end. The composite is Eq. pixel_color_computation.
//
// Backward: one workgroup per tile. First each pixel's adjoint factors are
// built in LDS: the core terms T_i (c_i - B_i) . G and T_i by walking the
// stored core back to front, and the tail factors shared by every tail
// fragment of the pixel (Sec. 3.3, last paragraph). Then each wave takes 64
// of the tile's instances, one per lane, and loops over the tile's pixels
// (skipping 8x8 blocks no lane's rect touches), recomputing rho^2 and alpha
// (|d|^2 and |m|^2 as sums of squares along each pixel row, which round a
// little differently from the forward's per-tile forms: a fragment within
// rounding of the cutoff, whose alpha is tau_alpha, may be judged
// differently; core members, with alpha >= tau_K, never are). Because d
// and m are affine in the pixel offset (lx, ly), the gradient w.r.t. their
// 18 affine coefficients follows
// from six moments of dL/d(rho^2)-weights per vector (sum of w, w lx, w ly,
// w lx^2, w lx ly, w ly^2), accumulated in registers. Each lane writes one
// partial per instance (the moments about the pixel at the centre of the
// Gaussian's tile rect, opacity and colour terms): no floating-point
// atomics, deterministic results.
#include <float.h>

#include "common.h"

namespace htgs {

constexpr float kNegHalfLog2e = -0.72134752044448170368f;  // -1 / (2 ln 2)

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

// Forward staging. The forward needs, per pixel ray, only |d|^2 and |m|^2
// (the cutoff test and alpha) and R3 . (d x m) (the depth of the maximum
// point). With d and m affine in the pixel offset (X, Y) from the tile
// centre (|X|, |Y| <= (tile size - 1) / 2), |d|^2 and R3 . (d x m) are
// quadratics in (X, Y) whose coefficients (1, X, Y, X^2, XY, Y^2) are
// formed per (tile, splat); a pixel evaluates each with five FMAs. |m|^2
// vanishes at the splat's centre, where its expanded quadratic would lose
// precision to cancellation, so it is staged as a sum of squares instead:
// with an orthonormal basis (q1, q2) of a plane holding Mu and Mv (q1
// along Mu), m = s1 q1 + s2 q2 + r with s1 = R11 X + R12 Y + k1,
// s2 = R22 Y + k2 and r constant and orthogonal to both, so
// |m|^2 = s1^2 + s2^2 + |r|^2 (five FMAs, cancellation only inside s1, s2,
// as in the vector form).
enum FwdStage {
  F_QD = 0,           // |d|^2
  F_QM = 6,           // |m|^2: |r|^2, R11, R12, k1, R22, k2
  F_RC = 12, F_O = 13, F_MUZ = 14, F_R = 15,
  F_QZ = 16,          // R3 . (d x m)
  F_G = 22, F_B = 23,
  F_BB = 24,          // covered pixel rect relative to the tile's first pixel
  F_FLOATS = 28, F_TEST4 = 4   // float4s read for the cutoff test and alpha
};

__device__ __forceinline__ void cross_f(const float a[3], const float b[3], float c[3]) {
  c[0] = fmaf(a[1], b[2], -a[2] * b[1]);
  c[1] = fmaf(a[2], b[0], -a[0] * b[2]);
  c[2] = fmaf(a[0], b[1], -a[1] * b[0]);
}

__device__ __forceinline__ float dot_f(const float a[3], const float b[3]) {
  return fmaf(a[2], b[2], fmaf(a[1], b[1], a[0] * b[0]));
}

// R3 . (a x b + e x f)
__device__ __forceinline__ float triple2(const float r[3], const float a[3], const float b[3],
                                         const float e[3], const float f[3]) {
  float c[3], g[3];
  cross_f(a, b, c);
  cross_f(e, f, g);
  return fmaf(r[2], c[2] + g[2], fmaf(r[1], c[1] + g[1], r[0] * (c[0] + g[0])));
}

// (cx2, cy2): twice the tile centre in pixel-index units (an integer).
__device__ __forceinline__ void stage_fwd(const float *__restrict__ rec, int cx2, int cy2,
                                          float *q) {
  const float dx = 0.5f * (float)(cx2 - 2 * __float_as_int(rec[R_IX]));
  const float dy = 0.5f * (float)(cy2 - 2 * __float_as_int(rec[R_IY]));
  float D0[3], Du[3], Dv[3], M0[3], Mu[3], Mv[3], R3[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Du[k] = rec[R_DU + k]; Dv[k] = rec[R_DV + k];
    Mu[k] = rec[R_MU + k]; Mv[k] = rec[R_MV + k];
    D0[k] = fmaf(dy, Dv[k], fmaf(dx, Du[k], rec[R_D0 + k]));
    M0[k] = fmaf(dy, Mv[k], fmaf(dx, Mu[k], rec[R_M0 + k]));
    R3[k] = rec[R_R3 + k];
  }
  q[F_QD + 0] = dot_f(D0, D0);
  q[F_QD + 1] = 2.f * dot_f(D0, Du);
  q[F_QD + 2] = 2.f * dot_f(D0, Dv);
  q[F_QD + 3] = dot_f(Du, Du);
  q[F_QD + 4] = 2.f * dot_f(Du, Dv);
  q[F_QD + 5] = dot_f(Dv, Dv);
  {
    // Gram-Schmidt (q1 along Mu; other unit vectors where Mu, or the part of
    // Mv orthogonal to it, vanishes). Float rounding of the basis only
    // perturbs |m|^2 relatively, by ~1e-7.
    float q1[3], q2[3];
    const float na2 = dot_f(Mu, Mu), nb2 = dot_f(Mv, Mv);
    if (na2 > 0.f) {
      const float s = __builtin_amdgcn_rsqf(na2);
      for (int k = 0; k < 3; ++k) q1[k] = Mu[k] * s;
    } else if (nb2 > 0.f) {
      const float s = __builtin_amdgcn_rsqf(nb2);
      for (int k = 0; k < 3; ++k) q1[k] = Mv[k] * s;
    } else {
      q1[0] = 1.f; q1[1] = 0.f; q1[2] = 0.f;
    }
    const float r12 = dot_f(q1, Mv);
    float v[3];
    for (int k = 0; k < 3; ++k) v[k] = fmaf(-r12, q1[k], Mv[k]);
    const float nv2 = dot_f(v, v);
    if (nv2 > 1e-12f * nb2 && nv2 > 0.f) {
      const float s = __builtin_amdgcn_rsqf(nv2);
      for (int k = 0; k < 3; ++k) q2[k] = v[k] * s;
    } else {
      // q1 x (the axis q1 is least along), normalised
      const float a0 = fabsf(q1[0]), a1 = fabsf(q1[1]), a2 = fabsf(q1[2]);
      float e[3] = {0.f, 0.f, 0.f};
      e[(a0 <= a1 && a0 <= a2) ? 0 : (a1 <= a2 ? 1 : 2)] = 1.f;
      cross_f(q1, e, q2);
      const float s = __builtin_amdgcn_rsqf(dot_f(q2, q2));
      for (int k = 0; k < 3; ++k) q2[k] *= s;
    }
    const float k1 = dot_f(q1, M0), k2 = dot_f(q2, M0);
    float r[3];
    for (int k = 0; k < 3; ++k) r[k] = fmaf(-k2, q2[k], fmaf(-k1, q1[k], M0[k]));
    q[F_QM + 0] = dot_f(r, r);
    q[F_QM + 1] = dot_f(q1, Mu);
    q[F_QM + 2] = r12;
    q[F_QM + 3] = k1;
    q[F_QM + 4] = dot_f(q2, Mv);
    q[F_QM + 5] = k2;
  }
  // d x m = D0xM0 + X (D0xMu + DuxM0) + Y (D0xMv + DvxM0) + X^2 DuxMu
  //         + XY (DuxMv + DvxMu) + Y^2 DvxMv
  float c[3];
  cross_f(D0, M0, c);
  q[F_QZ + 0] = dot_f(R3, c);
  q[F_QZ + 1] = triple2(R3, D0, Mu, Du, M0);
  q[F_QZ + 2] = triple2(R3, D0, Mv, Dv, M0);
  cross_f(Du, Mu, c);
  q[F_QZ + 3] = dot_f(R3, c);
  q[F_QZ + 4] = triple2(R3, Du, Mv, Dv, Mu);
  cross_f(Dv, Mv, c);
  q[F_QZ + 5] = dot_f(R3, c);
  q[F_RC] = rec[R_RC];
  q[F_O] = rec[R_O];
  q[F_MUZ] = rec[R_MUZ];
  q[F_R] = rec[R_RGB];
  q[F_G] = rec[R_RGB + 1];
  q[F_B] = rec[R_RGB + 2];
}

// Per-pixel constants of the quadratics: X, Y, X^2, XY, Y^2.
struct PixQ {
  float x, y, xx, xy, yy;
};

__device__ __forceinline__ float eval_q(const float *c, const PixQ &u) {
  return fmaf(u.yy, c[5], fmaf(u.xy, c[4], fmaf(u.xx, c[3], fmaf(u.y, c[2], fmaf(u.x, c[1], c[0])))));
}

// |d|^2 from its staged quadratic, the Y terms first (a pixel row shares
// them) and then the X terms: c0 + Y c2 + Y^2 c5 + X^2 c3 + X (c1 + Y c4).
// The backward evaluates it in the same order, row part once per row, so
// both passes get the same bits.
__device__ __forceinline__ float eval_dd(const float *c, const PixQ &u) {
  return fmaf(u.x, fmaf(u.y, c[4], c[1]), fmaf(u.xx, c[3], fmaf(u.yy, c[5], fmaf(u.y, c[2], c[0]))));
}

// |m|^2 = s1^2 + s2^2 + |r|^2 (see FwdStage).
__device__ __forceinline__ float eval_mm(const float *c, const PixQ &u) {
  const float s1 = fmaf(c[1], u.x, fmaf(c[2], u.y, c[3]));
  const float s2 = fmaf(c[4], u.y, c[5]);
  return fmaf(s1, s1, fmaf(s2, s2, c[0]));
}

// min(x, a) as a compare and a select (fminf canonicalizes its operands
// first, which costs an instruction per call in the raster loops).
__device__ __forceinline__ float min_sel(float x, float a) {
  return x <= a ? x : a;
}

// alpha = min(alpha_max, o exp(-rho^2 / 2)) with rho^2 = mm / dd.
__device__ __forceinline__ float frag_alpha(float o, float mm, float inv, float amax) {
  return min_sel(o * exp2_fast((mm * inv) * kNegHalfLog2e), amax);
}

__device__ __forceinline__ bool is_fragment(float dd, float mm, float rc) {
  return (dd >= FLT_MIN) && (mm <= rc * dd);
}


__device__ __forceinline__ void load_record(const float *__restrict__ recs, uint32_t gid, float *rec) {
  const float4 *r4 = reinterpret_cast<const float4 *>(recs + (int64_t)gid * kRecFloats);
#pragma unroll
  for (int k = 0; k < kRecFloats / 4; ++k) {
    const float4 t = r4[k];
    rec[4 * k] = t.x; rec[4 * k + 1] = t.y; rec[4 * k + 2] = t.z; rec[4 * k + 3] = t.w;
  }
}

struct TileInfo {
  int t, v, tx, ty;
};

// Float offset of a tile's forward state (tile-major layout: nval values
// of nt pixels per tile, tiles row-major inside their view).
__device__ __forceinline__ int64_t tile_state_off(const ViewParams &V, const TileInfo &ti,
                                                  int nval, int nt) {
  return V.state_off + ((int64_t)ti.ty * V.tiles_x + ti.tx) * nval * nt;
}

__device__ __forceinline__ bool tile_info(const ViewSet &vs, const KCfg &cfg, const Ws &w,
                                          TileInfo &ti) {
  if (cfg.cost_order) {
    if ((int)blockIdx.x >= vs.total_tiles) return false;
    ti.t = (int)w.order[blockIdx.x];
  } else {
    ti.t = xcd_tile(blockIdx.x, vs.total_tiles);
    if (ti.t >= vs.total_tiles) return false;
  }
  ti.v = view_of_tile(vs, ti.t);
  const int lt = ti.t - vs.v[ti.v].tile_base;
  ti.tx = lt % vs.v[ti.v].tiles_x;
  ti.ty = lt / vs.v[ti.v].tiles_x;
  return true;
}

// Tile of queue slot q in persistent mode: descending-cost order when the
// cost order is on, else row-major.
__device__ __forceinline__ void tile_of_slot(const ViewSet &vs, const KCfg &cfg, const Ws &w, int q,
                                             TileInfo &ti) {
  ti.t = cfg.cost_order ? (int)w.order[q] : q;
  ti.v = view_of_tile(vs, ti.t);
  const int lt = ti.t - vs.v[ti.v].tile_base;
  ti.tx = lt % vs.v[ti.v].tiles_x;
  ti.ty = lt / vs.v[ti.v].tiles_x;
}

// Runs BODY(ti) for the workgroup's tile, or, in persistent mode, for tiles
// taken from the atomic queue w.status[QSLOT] until it is exhausted (every
// workgroup leaves when the queue passes the tile count). PERSIST is a
// compile-time choice: the queue loop and its LDS word would otherwise cost
// the one-tile kernels registers and, for 8x8 backward tiles, a workgroup
// per CU (16 KiB of LDS plus that word).
#define HTGS_FOR_TILES(PERSIST, QSLOT, BODY)                                     \
  do {                                                                           \
    if constexpr (!(PERSIST)) {                                                  \
      TileInfo ti_;                                                              \
      if (tile_info(vs, cfg, w, ti_)) BODY(ti_);                                 \
    } else {                                                                     \
      __shared__ int s_next_;                                                    \
      for (;;) {                                                                 \
        __syncthreads();                                                         \
        if (threadIdx.x == 0) s_next_ = (int)atomicAdd(&w.status[QSLOT], 1u);    \
        __syncthreads();                                                         \
        const int q_ = s_next_;                                                  \
        if (q_ >= vs.total_tiles) break;                                         \
        TileInfo ti_;                                                            \
        tile_of_slot(vs, cfg, w, q_, ti_);                                       \
        BODY(ti_);                                                               \
      }                                                                          \
    }                                                                            \
  } while (0)

__device__ __forceinline__ bool rect_meets_block(const float *bb, int bx, int by) {
  return (__float_as_int(bb[2]) >= bx) && (__float_as_int(bb[0]) <= bx + 7) &&
         (__float_as_int(bb[3]) >= by) && (__float_as_int(bb[1]) <= by + 7);
}

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------
// One tile. EXACT: K == KMAX, known at compile time.
template <int KMAX, int TW, int TH, int BM, bool EXACT>
__device__ __forceinline__ void fwd_tile(const TileInfo &ti, const Ws &w, const ViewSet &vs,
                                         const KCfg &cfg, float *__restrict__ state,
                                         const uint32_t *__restrict__ vals) {
  constexpr int NT = TW * TH;
  constexpr int NBATCH = NT * BM;   // records staged per batch
  constexpr int NW = NT / 64;       // waves, one 8x8 block each
  constexpr int BX = TW / 8;
  constexpr int SV = F_FLOATS / 4;
  __shared__ float4 s_stage[NBATCH * SV];
  __shared__ uint16_t s_list[NW][NBATCH];
  __shared__ uint32_t s_nfrag;

  const ViewParams &V = vs.v[ti.v];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bx = (wave % BX) * 8, by = (wave / BX) * 8;
  const int lx = bx + (lane & 7), ly = by + (lane >> 3);
  const int px0 = ti.tx * TW, py0 = ti.ty * TH;
  const int px = px0 + lx, py = py0 + ly;
  const bool inside = (px < V.width) && (py < V.height);
  // a failed front end (overflow) leaves every
  // tile empty: background, and no list or record is read
  const uint2 rg = front_failed(w) ? make_uint2(0u, 0u) : w.ranges[ti.t];
  PixQ u;
  u.x = (float)lx - 0.5f * (float)(TW - 1);
  u.y = (float)ly - 0.5f * (float)(TH - 1);
  u.xx = u.x * u.x; u.xy = u.x * u.y; u.yy = u.y * u.y;   // exact (half-integers)
  const int cx2 = 2 * px0 + TW - 1, cy2 = 2 * py0 + TH - 1;
  const int K = EXACT ? KMAX : cfg.K;
  const float tau_core = cfg.tau_core, amax = cfg.alpha_max;
  const bool no_tail = cfg.no_tail != 0;
  const float *recs = w.records + (int64_t)ti.v * cfg.n * kRecFloats;
  const uint64_t lanemask_lt = (1ull << lane) - 1ull;

  // Core: depth, list position and (CARRY) alpha of up to K fragments,
  // sorted by depth (ties keep list order). Every fragment is added to the
  // running sums (alpha, alpha rgb, prod 1 - alpha); once the list is done
  // the core members are taken back out of them with the same alphas, which
  // leaves exactly the tail sums. Cores of up to 8 entries carry the alphas
  // through the insertion; larger ones recompute them from the records at
  // the end (same staging and arithmetic, so the same values), which keeps
  // 16 registers free for occupancy.
  constexpr bool CARRY = KMAX <= 8;
  float cz[KMAX], ca[KMAX];
  int cp[KMAX];
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    cz[i] = INFINITY; ca[i] = 0.f; cp[i] = -1;
  }
  float zlast = INFINITY;
  float A = 0.f, S0 = 0.f, S1 = 0.f, S2 = 0.f, P = 1.f;
  uint32_t nfrag = 0;
  if (tid == 0) s_nfrag = 0u;

  for (uint32_t base = rg.x; base < rg.y; base += NBATCH) {
    const int cnt = (int)min((uint32_t)NBATCH, rg.y - base);
    __syncthreads();
#pragma unroll
    for (int r0 = 0; r0 < NBATCH; r0 += NT) {
      const int r = r0 + tid;
      if (r < cnt) {
        const uint32_t gid = vals[base + r];
        float rec[kRecFloats];
        load_record(recs, gid, rec);
        float st[F_FLOATS];
        stage_fwd(rec, cx2, cy2, st);
        const uint32_t b0 = __float_as_uint(rec[R_BB0]), b1 = __float_as_uint(rec[R_BB1]);
        st[F_BB + 0] = __int_as_float((int)(b0 & 0xffffu) - px0);
        st[F_BB + 1] = __int_as_float((int)(b0 >> 16) - py0);
        st[F_BB + 2] = __int_as_float((int)(b1 & 0xffffu) - px0);
        st[F_BB + 3] = __int_as_float((int)(b1 >> 16) - py0);
#pragma unroll
        for (int k = 0; k < SV; ++k)
          s_stage[r * SV + k] = make_float4(st[4 * k], st[4 * k + 1], st[4 * k + 2], st[4 * k + 3]);
      }
    }
    __syncthreads();
    // This wave's list: the staged splats whose pixel rect meets its block.
    int nlist = cnt;
    if constexpr (NW > 1) {
      nlist = 0;
      for (int j0 = 0; j0 < cnt; j0 += 64) {
        const int j = j0 + lane;
        bool hit = false;
        if (j < cnt) {
          const float4 b = s_stage[j * SV + F_BB / 4];
          const float bb[4] = {b.x, b.y, b.z, b.w};
          hit = rect_meets_block(bb, bx, by);
        }
        const uint64_t mk = __ballot(hit);
        if (hit) s_list[wave][nlist + __popcll(mk & lanemask_lt)] = (uint16_t)j;
        nlist += __popcll(mk);
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (!inside) continue;
    auto stage_index = [&](int q) -> int {
      if constexpr (NW > 1) return s_list[wave][q];
      else return q;
    };
    auto fetch = [&](int j, float *e) {
#pragma unroll
      for (int k = 0; k < F_TEST4; ++k) {
        const float4 t = s_stage[j * SV + k];
        e[4 * k] = t.x; e[4 * k + 1] = t.y; e[4 * k + 2] = t.z; e[4 * k + 3] = t.w;
      }
    };
    auto step = [&](int j, const float *e) {
      const float dd = eval_dd(e + F_QD, u);
      const float mm = eval_mm(e + F_QM, u);
      if (!is_fragment(dd, mm, e[F_RC])) return;
      ++nfrag;
      const float inv = rcp_fast(dd);
      const float alpha = frag_alpha(e[F_O], mm, inv, amax);
      const float4 f5 = s_stage[j * SV + F_QZ / 4 + 1];   // qz4, qz5, g, b
      if (!no_tail) {   // uniform: a kernel argument
        A += alpha;
        S0 = fmaf(alpha, e[F_R], S0);
        S1 = fmaf(alpha, f5.z, S1);
        S2 = fmaf(alpha, f5.w, S2);
        P *= 1.f - alpha;
      }
      if (alpha >= tau_core && K > 0) {
        const float4 f4 = s_stage[j * SV + F_QZ / 4];     // qz0..qz3
        const float qz[6] = {f4.x, f4.y, f4.z, f4.w, f5.x, f5.y};
        const float z = fmaf(eval_q(qz, u), inv, e[F_MUZ]);
        if (z < zlast) {
          // Insert at the first entry deeper than z; the entries from there
          // on move back by one and the last one drops out of the core. On
          // the sorted depths that is new[i] = median(old[i-1], old[i], z)
          // (one instruction); the positions follow the comparisons.
          const int pos = (int)(base - rg.x) + j;
          bool c[KMAX];
#pragma unroll
          for (int i = 0; i < KMAX; ++i) c[i] = z < cz[i];
          // (Entries at K and beyond, if K < KMAX, are shifted too but never
          // read.)
#pragma unroll
          for (int i = KMAX - 1; i >= 1; --i) {
            cp[i] = c[i - 1] ? cp[i - 1] : (c[i] ? pos : cp[i]);
            if constexpr (CARRY) ca[i] = c[i - 1] ? ca[i - 1] : (c[i] ? alpha : ca[i]);
            cz[i] = __builtin_amdgcn_fmed3f(cz[i - 1], cz[i], z);
          }
          cp[0] = c[0] ? pos : cp[0];
          if constexpr (CARRY) ca[0] = c[0] ? alpha : ca[0];
          cz[0] = c[0] ? z : cz[0];
          if (K == KMAX) {
            zlast = cz[KMAX - 1];
          } else {
#pragma unroll
            for (int i = 0; i < KMAX; ++i)
              if (i == K - 1) zlast = cz[i];
          }
        }
      }
    };
    // One staged splat per step, its ray-test values read from LDS just
    // before use: without a second register buffer for the next splat the
    // 8x8 forward stays under 96 VGPRs (5 waves per SIMD), and the extra
    // wave hides the LDS latency better than the buffer did.
    for (int q = 0; q < nlist; ++q) {
      const int ja = stage_index(q);
      float ea[4 * F_TEST4];
      fetch(ja, ea);
      step(ja, ea);
    }
  }
  __syncthreads();
  if (nfrag) atomicAdd(&s_nfrag, nfrag);
  __syncthreads();
  if (tid == 0 && s_nfrag) count_add(w.frags, (unsigned long long)s_nfrag);
  if (!inside) return;

  // Composite (Eq. pixel_color_computation): the core front to back, then
  // the tail behind it.
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  float Ac = 0.f, Sc0 = 0.f, Sc1 = 0.f, Sc2 = 0.f;
  uint32_t ncore = 0;
  // tile-major state: this tile's values, value by value, each over the
  // tile's 8x8 blocks (this wave's block is block number `wave`)
  float *sp = state ? state + tile_state_off(V, ti, state_values(K), NT) + wave * 64 + lane
                    : nullptr;
  // One core member: composite, take it out of the sums, store it.
  auto core_entry = [&](int i, int gid, float a, float r, float g, float b) {
    if (gid >= 0) {
      const float wgt = a * T;
      C0 = fmaf(wgt, r, C0);
      C1 = fmaf(wgt, g, C1);
      C2 = fmaf(wgt, b, C2);
      T *= 1.f - a;
      Ac += a;
      Sc0 = fmaf(a, r, Sc0);
      Sc1 = fmaf(a, g, Sc1);
      Sc2 = fmaf(a, b, Sc2);
      ++ncore;
    }
    if (sp) {
      sp[(int64_t)i * NT] = __int_as_float(gid);
      sp[(int64_t)(K + i) * NT] = a;
      sp[(int64_t)(2 * K + i) * NT] = __int_as_float(cp[i]);
      sp[(int64_t)(3 * K + 3 * i) * NT] = r;
      sp[(int64_t)(3 * K + 3 * i + 1) * NT] = g;
      sp[(int64_t)(3 * K + 3 * i + 2) * NT] = b;
    }
  };
  if constexpr (CARRY) {
    // ids, then colours: every entry's loads are independent of the others'
    int gids[KMAX];
    float crgb[KMAX][3];
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
      gids[i] = (i < K && cp[i] >= 0) ? (int)vals[rg.x + (uint32_t)cp[i]] : -1;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gids[i] >= 0)
        c = reinterpret_cast<const float4 *>(recs + (int64_t)gids[i] * kRecFloats)[R_RGB / 4];
      crgb[i][0] = c.x; crgb[i][1] = c.y; crgb[i][2] = c.z;
    }
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
      if (i < K)
        core_entry(i, gids[i], gids[i] >= 0 ? ca[i] : 0.f, crgb[i][0], crgb[i][1], crgb[i][2]);
  } else {
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      if (i < K) {
        int gid = -1;
        float a = 0.f, r = 0.f, g = 0.f, b = 0.f;
        if (cp[i] >= 0) {
          gid = (int)vals[rg.x + (uint32_t)cp[i]];
          float rec[kRecFloats];
          load_record(recs, gid, rec);
          // the same staging and arithmetic as in the list walk: the same alpha
          float st[F_FLOATS];
          stage_fwd(rec, cx2, cy2, st);
          const float dd = eval_dd(st + F_QD, u), mm = eval_mm(st + F_QM, u);
          a = frag_alpha(st[F_O], mm, rcp_fast(dd), amax);
          r = st[F_R]; g = st[F_G]; b = st[F_B];
        }
        core_entry(i, gid, a, r, g, b);
      }
    }
  }
  // Tail sums: everything minus the core; exactly empty when no fragment
  // is left over, or when the tail is left out (inference without the
  // tail, Sec. 4.3: the background lies right behind the core).
  if (no_tail || nfrag == ncore) {
    A = 0.f; S0 = S1 = S2 = 0.f; P = 1.f;
  } else {
    A = fmaxf(A - Ac, 0.f);
    S0 = fmaxf(S0 - Sc0, 0.f);
    S1 = fmaxf(S1 - Sc1, 0.f);
    S2 = fmaxf(S2 - Sc2, 0.f);
    P = T > 0.f ? fminf(P / T, 1.f) : 0.f;
  }
  float X0 = P * cfg.bg[0], X1 = P * cfg.bg[1], X2 = P * cfg.bg[2];
  if (A > 0.f) {
    const float k = (1.f - P) / A;
    X0 = fmaf(k, S0, X0);
    X1 = fmaf(k, S1, X1);
    X2 = fmaf(k, S2, X2);
  }
  const int64_t npix = (int64_t)V.width * V.height;
  const int64_t pix = (int64_t)py * V.width + px;
  V.out_rgb[pix] = fmaf(T, X0, C0);
  V.out_rgb[npix + pix] = fmaf(T, X1, C1);
  V.out_rgb[2 * npix + pix] = fmaf(T, X2, C2);
  if (sp) {
    sp[(int64_t)(6 * K) * NT] = T;
    sp[(int64_t)(6 * K + 1) * NT] = A;
    sp[(int64_t)(6 * K + 2) * NT] = S0;
    sp[(int64_t)(6 * K + 3) * NT] = S1;
    sp[(int64_t)(6 * K + 4) * NT] = S2;
    sp[(int64_t)(6 * K + 5) * NT] = P;
  }
}

// ---------------------------------------------------------------------------
// Forward, sorted blending
// ---------------------------------------------------------------------------
// The paper's "w/o per-pixel HT" configuration (Sec. 4.3, Table splat_eval):
// the per-pixel evaluation of Sec. 3.2 with plain alpha blending (Eq.
// alpha_blending) in the order of the tile's list, which the front end has
// sorted front to back by the view depth of the Gaussians' means. A pixel
// stops before the fragment that would take its transmittance below tau_T
// (the early stop plain alpha blending allows, Sec. 5), and the workgroup
// stops staging batches once every pixel of its tile has stopped.
template <int TW, int TH>
__device__ __forceinline__ void fwd_tile_sorted(const TileInfo &ti, const Ws &w,
                                                const ViewSet &vs, const KCfg &cfg,
                                                float *__restrict__ state,
                                                const uint32_t *__restrict__ vals) {
  constexpr int NT = TW * TH;
  constexpr int NW = NT / 64;
  constexpr int BX = TW / 8;
  constexpr int SV = F_FLOATS / 4;
  __shared__ float4 s_stage[NT * SV];
  __shared__ uint16_t s_list[NW][NT];
  __shared__ uint32_t s_nfrag;

  const ViewParams &V = vs.v[ti.v];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bx = (wave % BX) * 8, by = (wave / BX) * 8;
  const int lx = bx + (lane & 7), ly = by + (lane >> 3);
  const int px0 = ti.tx * TW, py0 = ti.ty * TH;
  const int px = px0 + lx, py = py0 + ly;
  const bool inside = (px < V.width) && (py < V.height);
  const uint2 rg = front_failed(w) ? make_uint2(0u, 0u) : w.ranges[ti.t];
  PixQ u;
  u.x = (float)lx - 0.5f * (float)(TW - 1);
  u.y = (float)ly - 0.5f * (float)(TH - 1);
  u.xx = u.x * u.x; u.xy = u.x * u.y; u.yy = u.y * u.y;
  const int cx2 = 2 * px0 + TW - 1, cy2 = 2 * py0 + TH - 1;
  const float amax = cfg.alpha_max, tau_T = cfg.tau_T;
  const float *recs = w.records + (int64_t)ti.v * cfg.n * kRecFloats;
  const uint64_t lanemask_lt = (1ull << lane) - 1ull;

  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  bool done = !inside;
  int nb = 0, end_pos = 0, stop_pos = -1;
  if (tid == 0) s_nfrag = 0u;

  for (uint32_t base = rg.x; base < rg.y; base += NT) {
    // (also the barrier before the stage is overwritten)
    if (__syncthreads_and(done)) break;
    const int cnt = (int)min((uint32_t)NT, rg.y - base);
    if (tid < cnt) {
      const uint32_t gid = vals[base + tid];
      float rec[kRecFloats];
      load_record(recs, gid, rec);
      float st[F_FLOATS];
      stage_fwd(rec, cx2, cy2, st);
      const uint32_t b0 = __float_as_uint(rec[R_BB0]), b1 = __float_as_uint(rec[R_BB1]);
      st[F_BB + 0] = __int_as_float((int)(b0 & 0xffffu) - px0);
      st[F_BB + 1] = __int_as_float((int)(b0 >> 16) - py0);
      st[F_BB + 2] = __int_as_float((int)(b1 & 0xffffu) - px0);
      st[F_BB + 3] = __int_as_float((int)(b1 >> 16) - py0);
#pragma unroll
      for (int k = 0; k < SV; ++k)
        s_stage[tid * SV + k] = make_float4(st[4 * k], st[4 * k + 1], st[4 * k + 2], st[4 * k + 3]);
    }
    __syncthreads();
    int nlist = cnt;
    if constexpr (NW > 1) {
      nlist = 0;
      for (int j0 = 0; j0 < cnt; j0 += 64) {
        const int j = j0 + lane;
        bool hit = false;
        if (j < cnt) {
          const float4 b = s_stage[j * SV + F_BB / 4];
          const float bb[4] = {b.x, b.y, b.z, b.w};
          hit = rect_meets_block(bb, bx, by);
        }
        const uint64_t mk = __ballot(hit);
        if (hit) s_list[wave][nlist + __popcll(mk & lanemask_lt)] = (uint16_t)j;
        nlist += __popcll(mk);
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (done) continue;
    for (int q = 0; q < nlist; ++q) {
      int j = q;
      if constexpr (NW > 1) j = s_list[wave][q];
      float e[4 * F_TEST4];
#pragma unroll
      for (int k = 0; k < F_TEST4; ++k) {
        const float4 t = s_stage[j * SV + k];
        e[4 * k] = t.x; e[4 * k + 1] = t.y; e[4 * k + 2] = t.z; e[4 * k + 3] = t.w;
      }
      const float dd = eval_dd(e + F_QD, u);
      const float mm = eval_mm(e + F_QM, u);
      if (!is_fragment(dd, mm, e[F_RC])) continue;
      const float alpha = frag_alpha(e[F_O], mm, rcp_fast(dd), amax);
      const float tn = T * (1.f - alpha);
      const int pos = (int)(base - rg.x) + j;
      if (tn < tau_T) {
        done = true;
        stop_pos = pos;
        break;
      }
      const float4 f5 = s_stage[j * SV + F_QZ / 4 + 1];   // qz4, qz5, g, b
      const float wgt = alpha * T;
      C0 = fmaf(wgt, e[F_R], C0);
      C1 = fmaf(wgt, f5.z, C1);
      C2 = fmaf(wgt, f5.w, C2);
      T = tn;
      ++nb;
      end_pos = pos + 1;
    }
  }
  __syncthreads();
  if (nb) atomicAdd(&s_nfrag, (uint32_t)nb);
  __syncthreads();
  if (tid == 0 && s_nfrag) count_add(w.frags, (unsigned long long)s_nfrag);
  if (!inside) return;
  const int64_t npix = (int64_t)V.width * V.height;
  const int64_t pix = (int64_t)py * V.width + px;
  V.out_rgb[pix] = fmaf(T, cfg.bg[0], C0);
  V.out_rgb[npix + pix] = fmaf(T, cfg.bg[1], C1);
  V.out_rgb[2 * npix + pix] = fmaf(T, cfg.bg[2], C2);
  if (state) {
    float *sp = state + tile_state_off(V, ti, kSortedStateValues, NT) + wave * 64 + lane;
    sp[0] = T;
    sp[NT] = C0;
    sp[2 * NT] = C1;
    sp[3 * NT] = C2;
    sp[4 * NT] = __int_as_float(end_pos);
    sp[5 * NT] = __int_as_float(nb);
    sp[6 * NT] = __int_as_float(stop_pos >= 0 ? (int)vals[rg.x + (uint32_t)stop_pos] : -1);
  }
}

template <int TW, int TH, bool PERSIST>
__global__ void __launch_bounds__(TW * TH)
    k_raster_fwd_sorted(Ws w, ViewSet vs, KCfg cfg, float *__restrict__ state,
                        const uint32_t *__restrict__ vals) {
#define HTGS_FWDS_BODY(T) fwd_tile_sorted<TW, TH>(T, w, vs, cfg, state, vals)
  HTGS_FOR_TILES(PERSIST, kQueueFwd, HTGS_FWDS_BODY);
#undef HTGS_FWDS_BODY
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------
// Per-pixel adjoint factors of the hybrid backward in LDS (the core's list
// positions are read from the forward state when a chunk's core table is
// built, which keeps the row at 24 floats for K = 8).
template <int KMAX>
struct PixLayout {
  // G(3), w1, q1, q2, pad(2), dL/dalpha_i[KMAX], T_i[KMAX]
  static constexpr int kCoef = 8;
  static constexpr int kT = 8 + KMAX;
  static constexpr int kStride = ((8 + 2 * KMAX) + 3) / 4 * 4;
};

// Gradient contribution of one fragment (lane's splat at pixel Pp, column c
// of its 8x8 block; c is a constant after unrolling) to the lane's
// accumulators. cslot is the fragment's core index at this pixel, or -1 for
// a tail fragment. rs holds this row's sums of the d and m weights times
// (1, c, c^2).
template <int KMAX>
__device__ __forceinline__ void bwd_fragment(float op, const float *rgb, const float *Pp, int c,
                                             float dd, float mm, int cslot, float amax,
                                             float *rs, float *acc) {
  using L = PixLayout<KMAX>;
  // alpha exactly as the forward's frag_alpha forms it
  const float inv = rcp_fast(dd);
  const float r2 = mm * inv;
  const float e = exp2_fast(r2 * kNegHalfLog2e);
  const float araw = op * e;
  const bool unclamped = araw <= amax;
  const float alpha = unclamped ? araw : amax;
  const float G0 = Pp[0], G1 = Pp[1], G2 = Pp[2], w1 = Pp[3];
  // tail: dC/dalpha = w1 (c - c_tail) - T P (c_bg - c_tail) / (1 - alpha),
  // dC/dc = w1 alpha; core: the pixel's precomputed T_i (c_i - B_i) and T_i
  const float gdc = fmaf(G2, rgb[2], fmaf(G1, rgb[1], G0 * rgb[0]));
  const float tail = fmaf(w1, gdc, -Pp[4]) - Pp[5] * rcp_fast(1.f - alpha);
  // Branch-free: every lane reads a core entry (entry 0 for tail
  // fragments) and selects.
  const bool core = cslot >= 0;
  const int ci = core ? cslot : 0;
  const float cf = Pp[L::kCoef + ci], cT = Pp[L::kT + ci];
  const float dLda = core ? cf : tail;
  const float wc = alpha * (core ? cT : w1);
  acc[13] = fmaf(wc, G0, acc[13]);
  acc[14] = fmaf(wc, G1, acc[14]);
  acc[15] = fmaf(wc, G2, acc[15]);
  // Where alpha is clamped, o and rho^2 receive no gradient.
  const float g = unclamped ? dLda : 0.f;
  {
    acc[12] = fmaf(g, e, acc[12]);
    const float s1 = -alpha * g * inv;      // weight of m: 2 dL/drho^2 / |d|^2
    const float s2 = -s1 * r2;              // weight of d
    rs[0] += s2;
    rs[3] += s1;
    if (c == 1) {
      rs[1] += s2; rs[2] += s2;
      rs[4] += s1; rs[5] += s1;
    } else if (c > 1) {
      const float fc = (float)c, fc2 = (float)(c * c);
      rs[1] = fmaf(fc, s2, rs[1]);
      rs[2] = fmaf(fc2, s2, rs[2]);
      rs[4] = fmaf(fc, s1, rs[4]);
      rs[5] = fmaf(fc2, s1, rs[5]);
    }
  }
}

// Writes one instance partial: the lane's moments about the tile's first
// pixel (acc[0..5] for the d weights, acc[6..11] for the m weights) moved to
// an origin (a, b) pixels before it (dx = lx + a: sum w dx = S_x + a S,
// sum w dx^2 = S_xx + 2 a S_x + a^2 S, ...), then dL/do and dL/d(rgb).
__device__ __forceinline__ void write_partial(const float *acc, float a, float b, float *dstf) {
  float out[kPartialFloats];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float *S = acc + 6 * h;
    float *M = out + (h ? P_MM : P_MD);
    M[0] = S[0];
    M[1] = fmaf(a, S[0], S[1]);
    M[2] = fmaf(b, S[0], S[2]);
    M[3] = fmaf(a, fmaf(a, S[0], 2.f * S[1]), S[3]);
    M[4] = fmaf(a, fmaf(b, S[0], S[2]), fmaf(b, S[1], S[4]));
    M[5] = fmaf(b, fmaf(b, S[0], 2.f * S[2]), S[5]);
  }
  out[P_O] = acc[12];
  out[P_C] = acc[13];
  out[P_C + 1] = acc[14];
  out[P_C + 2] = acc[15];
  float4 *dst = reinterpret_cast<float4 *>(dstf);
#pragma unroll
  for (int k = 0; k < kPartialFloats / 4; ++k)
    dst[k] = make_float4(out[4 * k], out[4 * k + 1], out[4 * k + 2], out[4 * k + 3]);
}

// Byte swizzle of the backward's core table rows (see bwd_tile).
__device__ __forceinline__ constexpr int slot_swz(int q) { return ((q >> 1) & 15) << 2; }

// Waves per backward workgroup. A tile's 64-instance chunks are dealt to
// its waves round-robin, so waves whose share ends early idle until the
// tile is done: with four waves ~25% of the wave time at 1080p; fewer waves
// idle less but stage the tile's per-pixel factors for fewer waves.
#ifndef HTGS_BWD_WAVES_SMALL
#define HTGS_BWD_WAVES_SMALL 2
#endif
#ifndef HTGS_BWD_WAVES_MID
#define HTGS_BWD_WAVES_MID 4
#endif
template <int TW, int TH>
constexpr int bwd_waves() {
  return TW * TH <= 64 ? HTGS_BWD_WAVES_SMALL : (TW * TH <= 128 ? HTGS_BWD_WAVES_MID : 4);
}

// Target waves per SIMD of the backward (register budget; HIP's second
// launch-bounds argument is a minimum number of waves per execution unit).
template <int KMAX, int TW>
constexpr int bwd_simd_waves() {
  return (TW == 8 && KMAX <= 8) ? 5 : ((TW == 8 && KMAX <= 16) ? 4 : 1);
}

template <int KMAX, int TW, int TH, bool EXACT>
__device__ __forceinline__ void bwd_tile(const TileInfo &ti, const Ws &w, const ViewSet &vs,
                                         const KCfg &cfg, const float *__restrict__ state,
                                         const uint32_t *__restrict__ vals, uint32_t &nfr) {
  constexpr int NT = TW * TH;
  constexpr int NB = NT / 64;
  constexpr int BX = TW / 8;
  using L = PixLayout<KMAX>;
  __shared__ float4 s_pix[NT * L::kStride / 4];
  constexpr int BW = bwd_waves<TW, TH>();
  constexpr int BT = 64 * BW;
  // per wave, for the 8x8 block being walked: [block pixel][lane ^ swz(pixel)]
  // = core index + 1 of the lane's instance at that pixel, 0 if not in the
  // core. The byte swizzle swz(q) = ((q >> 1) & 15) << 2 spreads the fill
  // (each lane writes its own pixel's 64-byte row) over the banks; the
  // reads (one row, one byte per lane) stay conflict-free.
  // With a core of at most 8 entries the table holds core index + 1 in
  // nibbles (two lanes per byte; a pixel's row is 32 bytes): half the LDS of
  // byte rows, 10 KiB in all for an 8x8 tile, which made the 8x8 backward
  // ~4% faster. Paired waves keep byte rows, which double as the buffer
  // through which they hand over their sums.
  constexpr bool NIB = KMAX <= 8 && !(NB == 2 && BW == 4);
  constexpr int SB = NIB ? 32 : 64;
  __shared__ uint8_t s_slot[BW][64][SB];
  // core index (or -1) of table row entry idx
  auto core_of = [](const uint8_t *row, int idx) -> int {
    if constexpr (NIB) return (int)((row[idx >> 1] >> ((idx & 1) * 4)) & 15u) - 1;
    else return (int)row[idx] - 1;
  };

  const ViewParams &V = vs.v[ti.v];
  const int tid = threadIdx.x;
  const int px0 = ti.tx * TW, py0 = ti.ty * TH;
  const int K = EXACT ? KMAX : cfg.K;
  const float *recs = w.records + (int64_t)ti.v * cfg.n * kRecFloats;
  const int64_t npix = (int64_t)V.width * V.height;
  float *sp_all = reinterpret_cast<float *>(s_pix);

  // Per-pixel adjoint factors. Threads walk the pixels in the state's
  // order (8x8 blocks, row-major inside), so consecutive threads read
  // consecutive state words.
  const float *tstate = state + tile_state_off(V, ti, state_values(K), NT);
  for (int ps = tid; ps < NT; ps += BT) {
    const int lxp = ((ps >> 6) % BX) * 8 + (ps & 7), lyp = ((ps >> 6) / BX) * 8 + ((ps >> 3) & 7);
    const int p = lyp * TW + lxp;
    const int px = px0 + lxp, py = py0 + lyp;
    float *Pp = sp_all + p * L::kStride;
    float G[3] = {0.f, 0.f, 0.f}, w1 = 0.f, q1 = 0.f, q2 = 0.f;
    int pos[KMAX];
    float coef[KMAX], Ti[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) { pos[i] = -1; coef[i] = 0.f; Ti[i] = 0.f; }
    if (px < V.width && py < V.height) {
      const int64_t pix = (int64_t)py * V.width + px;
      for (int c = 0; c < 3; ++c) G[c] = V.grad_rgb[c * npix + pix];
      const float *sp = tstate + ps;
      float ca[KMAX], cc[KMAX][3];
#pragma unroll
      for (int i = 0; i < KMAX; ++i) {
        ca[i] = 0.f; cc[i][0] = cc[i][1] = cc[i][2] = 0.f;
        if (i < K) {
          // all loads independent of each other (one round trip); empty
          // entries (position -1) get alpha and colour 0 from the forward
          ca[i] = sp[(int64_t)(K + i) * NT];
          pos[i] = __float_as_int(sp[(int64_t)(2 * K + i) * NT]);
          cc[i][0] = sp[(int64_t)(3 * K + 3 * i) * NT];
          cc[i][1] = sp[(int64_t)(3 * K + 3 * i + 1) * NT];
          cc[i][2] = sp[(int64_t)(3 * K + 3 * i + 2) * NT];
        }
      }
      const float A = sp[(int64_t)(6 * K + 1) * NT];
      const float S[3] = {sp[(int64_t)(6 * K + 2) * NT], sp[(int64_t)(6 * K + 3) * NT],
                          sp[(int64_t)(6 * K + 4) * NT]};
      const float Pt = sp[(int64_t)(6 * K + 5) * NT];
      float T = 1.f;
#pragma unroll
      for (int i = 0; i < KMAX; ++i) {
        if (i < K && pos[i] >= 0) {
          Ti[i] = T;
          T *= 1.f - ca[i];
        }
      }
      float X[3], ct[3] = {0.f, 0.f, 0.f};
      const bool has_tail = A > 0.f;
      for (int c = 0; c < 3; ++c) {
        X[c] = Pt * cfg.bg[c];
        if (has_tail) {
          ct[c] = S[c] / A;
          X[c] = fmaf(1.f - Pt, ct[c], X[c]);
        }
      }
      float B[3] = {X[0], X[1], X[2]};
#pragma unroll
      for (int i = KMAX - 1; i >= 0; --i) {
        if (i < K && pos[i] >= 0) {
          coef[i] = Ti[i] * (G[0] * (cc[i][0] - B[0]) + G[1] * (cc[i][1] - B[1]) +
                             G[2] * (cc[i][2] - B[2]));
          for (int c = 0; c < 3; ++c) B[c] = fmaf(ca[i], cc[i][c] - B[c], B[c]);
        }
      }
      if (has_tail) {
        w1 = T * (1.f - Pt) / A;
        q1 = w1 * (G[0] * ct[0] + G[1] * ct[1] + G[2] * ct[2]);
        q2 = T * Pt *
             (G[0] * (cfg.bg[0] - ct[0]) + G[1] * (cfg.bg[1] - ct[1]) + G[2] * (cfg.bg[2] - ct[2]));
      }
    }
    Pp[0] = G[0]; Pp[1] = G[1]; Pp[2] = G[2];
    Pp[3] = w1; Pp[4] = q1; Pp[5] = q2; Pp[6] = 0.f; Pp[7] = 0.f;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      Pp[L::kCoef + i] = coef[i];
      Pp[L::kT + i] = Ti[i];
    }
  }
  __syncthreads();

  const uint2 rg = w.ranges[ti.t];
  const int wave = tid >> 6, lane = tid & 63;
  const uint32_t count = rg.y - rg.x;
  const uint32_t nch = (count + 63u) >> 6;
  const float amax = cfg.alpha_max;
  // Chunk schedule. In general a wave takes every BW-th chunk over all of
  // the tile's 8x8 blocks. With two blocks and four waves (16x8, 8x16
  // tiles) a pair of waves shares each chunk instead, one block each, and
  // the pairs alternate chunks; the block-1 wave hands its sums to the
  // block-0 wave, which writes the partial. A tile whose chunk count is not
  // a multiple of the wave count then leaves fewer waves idle.
  constexpr bool PAIRS = (NB == 2 && BW == 4);
  const int myblk = PAIRS ? (wave >> 1) : -1;
  const uint32_t c_end = PAIRS ? 2u * ((nch + 1u) >> 1) : nch;  // uniform per block when PAIRS
  const uint32_t c_step = PAIRS ? 2u : (uint32_t)BW;
  const int cx2 = 2 * px0 + TW - 1, cy2 = 2 * py0 + TH - 1;
  const float hx = 0.5f * (float)(TW - 1), hy = 0.5f * (float)(TH - 1);
  for (uint32_t c = PAIRS ? (uint32_t)(wave & 1) : (uint32_t)wave; c < c_end; c += c_step) {
    const uint32_t j = rg.x + c * 64u + lane;
    const bool active = c < nch && j < rg.y;
    // The forward's staged forms of |d|^2 and |m|^2 for this (tile, splat)
    // (stage_fwd, same arithmetic), so that every pixel's |d|^2, |m|^2,
    // fragment test and alpha are bit-identical to the forward's: the
    // backward differentiates exactly the fragments the image blended.
    float qd[6], qm[6], rc = -1.f, op = 0.f, rgb[3] = {0.f, 0.f, 0.f};
    int bb[4] = {1 << 20, 1 << 20, -1, -1};
#pragma unroll
    for (int k = 0; k < 6; ++k) { qd[k] = 0.f; qm[k] = 0.f; }
    uint32_t slot = 0, gid = 0;
    int ox = 0, oy = 0;   // moment origin: the record's reference pixel
    if (active) {
      gid = vals[j];
      float rec[kRecFloats];
      load_record(recs, gid, rec);
      float sf[F_FLOATS];
      stage_fwd(rec, cx2, cy2, sf);
#pragma unroll
      for (int k = 0; k < 6; ++k) { qd[k] = sf[F_QD + k]; qm[k] = sf[F_QM + k]; }
      rc = sf[F_RC];
      op = sf[F_O];
      rgb[0] = sf[F_R]; rgb[1] = sf[F_G]; rgb[2] = sf[F_B];
      const uint32_t b0 = __float_as_uint(rec[R_BB0]), b1 = __float_as_uint(rec[R_BB1]);
      bb[0] = (int)(b0 & 0xffffu) - px0;
      bb[1] = (int)(b0 >> 16) - py0;
      bb[2] = (int)(b1 & 0xffffu) - px0;
      bb[3] = (int)(b1 >> 16) - py0;
      if (myblk <= 0) {
        slot = tslot_slot(w.tslots[(int64_t)ti.v * cfg.n + gid], ti.tx, ti.ty);
        ox = __float_as_int(rec[R_IX]);
        oy = __float_as_int(rec[R_IY]);
      }
    }
    const float bbf[4] = {__int_as_float(bb[0]), __int_as_float(bb[1]), __int_as_float(bb[2]),
                          __int_as_float(bb[3])};
    // acc: d-moments (6), m-moments (6), dL/do, dL/drgb (3)
    float acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.f;
    for (int blk = 0; blk < NB; ++blk) {
      if (PAIRS && blk != myblk) continue;
      const int bx = (blk % BX) * 8, by = (blk / BX) * 8;
      const bool hitb = active && rect_meets_block(bbf, bx, by);
      if (__ballot(hitb) == 0ull) continue;
      // Core table of this block for this chunk: lane = block pixel.
      {
        // list positions of the pixel's core from the forward state
        const float *tst = tstate + blk * 64 + lane;
        int cps[KMAX];
#pragma unroll
        for (int i = 0; i < KMAX; ++i) cps[i] = i < K ? __float_as_int(tst[(int64_t)(2 * K + i) * NT]) : -1;
        // cleared with consecutive lanes on consecutive words (no bank
        // conflicts), then each lane fills its own pixel's row
        uint32_t *tab = reinterpret_cast<uint32_t *>(&s_slot[wave][0][0]);
#pragma unroll
        for (int k = 0; k < SB / 4; ++k) tab[k * 64 + lane] = 0u;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
          if (i < K) {
            const int ps = cps[i];
            const uint32_t dl = (uint32_t)(ps - (int)(c * 64u));
            if (ps >= 0 && dl < 64u) {
              if constexpr (NIB) {
                uint8_t *b = &s_slot[wave][lane][(dl ^ slot_swz(lane)) >> 1];
                *b = (uint8_t)(*b | ((i + 1) << ((dl & 1u) * 4u)));
              } else {
                s_slot[wave][lane][dl ^ slot_swz(lane)] = (uint8_t)(i + 1);
              }
            }
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
      // Pixels of the block inside the image (the forward skips the rest).
      const int cols_in = V.width - (px0 + bx), rows_in = V.height - (py0 + by);
      // A row at a time: the row's parts of the two staged forms (Y, the
      // pixel's offset from the tile centre, fixed), then two FMAs per pixel
      // for each; the columns are unrolled, so for one-block tiles X is a
      // constant. The moments (1, lx, ly, lx^2, lx ly, ly^2) of the weights
      // follow from per-row sums over (1, c, c^2).
      const float fbx = (float)bx;
      for (int row = 0; row < 8; ++row) {
        const float ly = (float)(by + row);
        const float Y = ly - hy, YY = Y * Y;
        const float rd0 = fmaf(YY, qd[5], fmaf(Y, qd[2], qd[0]));
        const float rd1 = fmaf(Y, qd[4], qd[1]);
        const float s2 = fmaf(qm[4], Y, qm[5]);
        const float rm0 = fmaf(s2, s2, qm[0]);
        const float rm1 = fmaf(qm[2], Y, qm[3]);
        // (bitwise ands: both pixels of a column pair are tested before
        // either fragment path branches, and no test branches on its own)
        const bool row_in = hitb & (row < rows_in);
        float rs[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int col = 0; col < 8; col += 2) {
          const float X0 = (fbx + (float)col) - hx, X1 = X0 + 1.f;
          const float dd0 = fmaf(X0, rd1, fmaf(X0 * X0, qd[3], rd0));
          const float dd1 = fmaf(X1, rd1, fmaf(X1 * X1, qd[3], rd0));
          const float s10 = fmaf(qm[1], X0, rm1), s11 = fmaf(qm[1], X1, rm1);
          const float mm0 = fmaf(s10, s10, rm0), mm1 = fmaf(s11, s11, rm0);
          const bool f0 = row_in & (col < cols_in) & (dd0 >= FLT_MIN) & (mm0 <= rc * dd0);
          const bool f1 = row_in & (col + 1 < cols_in) & (dd1 >= FLT_MIN) & (mm1 <= rc * dd1);
          const int q = row * 8 + col;
          const float *P0 = sp_all + ((by + row) * TW + bx + col) * L::kStride;
          if (f0) {
            ++nfr;
            bwd_fragment<KMAX>(op, rgb, P0, col, dd0, mm0, core_of(s_slot[wave][q], lane ^ slot_swz(q)), amax,
                               rs, acc);
          }
          if (f1) {
            ++nfr;
            bwd_fragment<KMAX>(op, rgb, P0 + L::kStride, col + 1, dd1, mm1,
                               core_of(s_slot[wave][q + 1], lane ^ slot_swz(q + 1)), amax, rs, acc);
          }
        }
        if constexpr (BX > 1) {
          // sums over (1, c, c^2) -> over (1, lx, lx^2), lx = bx + c
          rs[2] = fmaf(fbx, fmaf(fbx, rs[0], 2.f * rs[1]), rs[2]);
          rs[1] = fmaf(fbx, rs[0], rs[1]);
          rs[5] = fmaf(fbx, fmaf(fbx, rs[3], 2.f * rs[4]), rs[5]);
          rs[4] = fmaf(fbx, rs[3], rs[4]);
        }
        const float ly2 = ly * ly;
        acc[0] += rs[0];
        acc[1] += rs[1];
        acc[2] = fmaf(ly, rs[0], acc[2]);
        acc[3] += rs[2];
        acc[4] = fmaf(ly, rs[1], acc[4]);
        acc[5] = fmaf(ly2, rs[0], acc[5]);
        acc[6] += rs[3];
        acc[7] += rs[4];
        acc[8] = fmaf(ly, rs[3], acc[8]);
        acc[9] += rs[5];
        acc[10] = fmaf(ly, rs[4], acc[10]);
        acc[11] = fmaf(ly2, rs[3], acc[11]);
      }
      __builtin_amdgcn_wave_barrier();
    }
    if constexpr (PAIRS) {
      // The block-1 wave's core table is free now: it carries the sums.
      float *xch = reinterpret_cast<float *>(&s_slot[2 + (wave & 1)][0][0]);
      if (myblk == 1) {
#pragma unroll
        for (int k = 0; k < 16; ++k) xch[k * 64 + lane] = acc[k];
      }
      __syncthreads();
      if (myblk == 0) {
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] += xch[k * 64 + lane];
      }
      __syncthreads();  // before the block-1 waves rebuild their tables
    }
    if (myblk <= 0 && active && (uint64_t)slot < (uint64_t)w.capacity) {
      // The tile's moments (about its first pixel) moved to the record's
      // reference pixel, (a, b) pixels from it (near the splat's centre,
      // which keeps the moments small): with dx = lx + a,
      // sum w dx = S_x + a S, sum w dx^2 = S_xx + 2 a S_x + a^2 S, ...
      const float a = (float)(px0 - ox);
      const float b = (float)(py0 - oy);
      write_partial(acc, a, b, w.partials + (int64_t)slot * kPartialFloats);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Minimum waves per SIMD asked of the compiler for the forward (HIP's
// second launch bound): 4 keeps up to 128 VGPRs per lane, which the
// forward with a core of up to 8 entries fits in without spilling (8x8
// tiles stay under 96, 5 waves). The macros let a build try other bounds.
#ifndef HTGS_FWD_WAVES_NARROW
#define HTGS_FWD_WAVES_NARROW 4
#endif
#ifndef HTGS_FWD_WAVES_WIDE
#define HTGS_FWD_WAVES_WIDE 4
#endif
template <int KMAX, int TW, int BM>
constexpr int fwd_simd_waves() {
  // (a doubled LDS batch holds the forward at 3 workgroups per SIMD anyway)
  return (KMAX > 8 || BM > 1) ? 1 : (TW == 8 ? HTGS_FWD_WAVES_NARROW : HTGS_FWD_WAVES_WIDE);
}

template <int KMAX, int TW, int TH, int BM, bool EXACT, bool PERSIST>
__global__ void __launch_bounds__((TW * TH), (fwd_simd_waves<KMAX, TW, BM>()))
    k_raster_fwd(Ws w, ViewSet vs, KCfg cfg, float *__restrict__ state,
                 const uint32_t *__restrict__ vals) {
#define HTGS_FWD_BODY(T) fwd_tile<KMAX, TW, TH, BM, EXACT>(T, w, vs, cfg, state, vals)
  HTGS_FOR_TILES(PERSIST, kQueueFwd, HTGS_FWD_BODY);
#undef HTGS_FWD_BODY
}

template <int KMAX, int TW, int TH, bool EXACT, bool PERSIST>
__global__ void __launch_bounds__((64 * bwd_waves<TW, TH>()), (bwd_simd_waves<KMAX, TW>()))
    k_raster_bwd(Ws w, ViewSet vs, KCfg cfg, const float *__restrict__ state,
                 const uint32_t *__restrict__ vals) {
  // the forward of a failed front end rendered empty tiles: nothing to do
  if (front_failed(w)) return;
  uint32_t nfr = 0;   // fragments this thread differentiated
#define HTGS_BWD_BODY(T) bwd_tile<KMAX, TW, TH, EXACT>(T, w, vs, cfg, state, vals, nfr)
  HTGS_FOR_TILES(PERSIST, kQueueBwd, HTGS_BWD_BODY);
#undef HTGS_BWD_BODY
  // one atomic per wave (a word of LDS would take the 8x8 and 16x8 kernels
  // past 16 and 32 KiB, one workgroup per CU fewer)
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) nfr += (uint32_t)__shfl_xor((int)nfr, off, 64);
  if ((threadIdx.x & 63) == 0 && nfr) count_add(w.frags_bwd, (unsigned long long)nfr);
}

// ---------------------------------------------------------------------------
// Backward, sorted blending
// ---------------------------------------------------------------------------
// Inclusive scans over the 64 lanes of a wave with DPP lane moves: shifts
// by 1, 2, 4, 8 inside each row of 16 lanes, then lane 15 into rows 1 and 3
// and lane 31 into rows 2 and 3. Lanes without a source take the identity.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float x, float identity) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(identity), __float_as_int(x),
                                                    CTRL, ROW_MASK, 0xf, false));
}
__device__ __forceinline__ float wave_scan_mul(float x) {
  x *= dpp_move<0x111, 0xf>(x, 1.f);
  x *= dpp_move<0x112, 0xf>(x, 1.f);
  x *= dpp_move<0x114, 0xf>(x, 1.f);
  x *= dpp_move<0x118, 0xf>(x, 1.f);
  x *= dpp_move<0x142, 0xa>(x, 1.f);
  x *= dpp_move<0x143, 0xc>(x, 1.f);
  return x;
}
__device__ __forceinline__ float wave_scan_add(float x) {
  x += dpp_move<0x111, 0xf>(x, 0.f);
  x += dpp_move<0x112, 0xf>(x, 0.f);
  x += dpp_move<0x114, 0xf>(x, 0.f);
  x += dpp_move<0x118, 0xf>(x, 0.f);
  x += dpp_move<0x142, 0xa>(x, 0.f);
  x += dpp_move<0x143, 0xc>(x, 0.f);
  return x;
}

// Adjoint of sorted blending. With the fragments of a pixel blended front
// to back, C = sum_i alpha_i T_i c_i + T c_bg, T_i = prod_{k<i} (1 -
// alpha_k):
//   dC/dc_i = alpha_i T_i,
//   dC/dalpha_i = T_i c_i - R_i / (1 - alpha_i),  R_i = sum_{k>i} alpha_k T_k
//                 c_k + T c_bg = C - (sum_{k<=i} alpha_k T_k c_k).
// The lanes of a wave hold 64 consecutive list entries (splats) of the tile
// and walk the pixels of their 8x8 block; at a pixel a wave scan over the
// lanes gives each lane T_i (product of 1 - alpha) and the dot product with
// G = dL/dC of the prefix colour sum, starting from the pixel's carry of the
// earlier chunks (kept in LDS), so the chunks of a tile run in list order.
// A lane's fragment is differentiated iff the forward blended it: its list
// position lies before the pixel's end position stored by the forward (the
// same staged forms and arithmetic give the same fragment test and alpha).
// Partials as in the hybrid backward: moments of the d and m weights, opacity
// and colour terms, one per instance. One wave per 8x8 block; with several
// blocks the waves add their sums in LDS and wave 0 writes the partial.
template <int TW, int TH>
__device__ __forceinline__ void bwd_tile_sorted(const TileInfo &ti, const Ws &w,
                                                const ViewSet &vs, const KCfg &cfg,
                                                const float *__restrict__ state,
                                                const uint32_t *__restrict__ vals, uint32_t &nfr) {
  constexpr int NT = TW * TH;
  constexpr int NB = NT / 64;
  constexpr int BX = TW / 8;
  // per pixel: G (3), G . C, then end position, T carry, (G . prefix) carry
  __shared__ float4 s_pg[NT], s_pc[NT];
  __shared__ float s_red[NB > 1 ? NB * 16 * 64 : 1];   // [block][value][lane]
  __shared__ int s_maxend;

  const ViewParams &V = vs.v[ti.v];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bx = (wave % BX) * 8, by = (wave / BX) * 8;
  const int px0 = ti.tx * TW, py0 = ti.ty * TH;
  const float *recs = w.records + (int64_t)ti.v * cfg.n * kRecFloats;
  const int64_t npix = (int64_t)V.width * V.height;
  if (tid == 0) s_maxend = 0;
  __syncthreads();
  {
    // this thread's pixel: block `wave`, lane = row-major pixel of the block
    const int lx = bx + (lane & 7), ly = by + (lane >> 3);
    const int px = px0 + lx, py = py0 + ly;
    float4 pg = make_float4(0.f, 0.f, 0.f, 0.f), pc = make_float4(0.f, 1.f, 0.f, 0.f);
    if (px < V.width && py < V.height) {
      const int64_t pix = (int64_t)py * V.width + px;
      const float *sp = state + tile_state_off(V, ti, kSortedStateValues, NT) + wave * 64 + lane;
      const float T = sp[0], S0 = sp[NT], S1 = sp[2 * NT], S2 = sp[3 * NT];
      const int end = __float_as_int(sp[4 * NT]);
      const float G0 = V.grad_rgb[pix], G1 = V.grad_rgb[npix + pix], G2 = V.grad_rgb[2 * npix + pix];
      const float gC = fmaf(G2, fmaf(T, cfg.bg[2], S2), fmaf(G1, fmaf(T, cfg.bg[1], S1),
                                                          G0 * fmaf(T, cfg.bg[0], S0)));
      pg = make_float4(G0, G1, G2, gC);
      pc = make_float4(__int_as_float(end), 1.f, 0.f, 0.f);
      if (end > 0) atomicMax(&s_maxend, end);
    }
    s_pg[ly * TW + lx] = pg;
    s_pc[ly * TW + lx] = pc;
  }
  __syncthreads();
  const uint2 rg = w.ranges[ti.t];
  // no pixel blends past max_end: later list entries get zero partials
  // (every instance's slot is written, as the preprocess backward sums them)
  const uint32_t stop = min(rg.y, rg.x + (uint32_t)s_maxend);
  const float amax = cfg.alpha_max;
  const int cx2 = 2 * px0 + TW - 1, cy2 = 2 * py0 + TH - 1;
  const float hx = 0.5f * (float)(TW - 1), hy = 0.5f * (float)(TH - 1);
  const int cols_in = V.width - (px0 + bx), rows_in = V.height - (py0 + by);
  for (uint32_t c0 = rg.x; c0 < rg.y; c0 += 64u) {
    const uint32_t j = c0 + lane;
    const bool active = j < rg.y;
    const bool work = j < stop;
    const int pos = (int)(j - rg.x);
    float qd[6], qm[6], rc = -1.f, op = 0.f, rgb[3] = {0.f, 0.f, 0.f};
    int bb[4] = {1 << 20, 1 << 20, -1, -1};
#pragma unroll
    for (int k = 0; k < 6; ++k) { qd[k] = 0.f; qm[k] = 0.f; }
    const uint32_t gid = active ? vals[j] : 0u;
    int ox = 0, oy = 0;   // moment origin: the record's reference pixel
    if (work) {
      float rec[kRecFloats];
      load_record(recs, gid, rec);
      ox = __float_as_int(rec[R_IX]);
      oy = __float_as_int(rec[R_IY]);
      float sf[F_FLOATS];
      stage_fwd(rec, cx2, cy2, sf);
#pragma unroll
      for (int k = 0; k < 6; ++k) { qd[k] = sf[F_QD + k]; qm[k] = sf[F_QM + k]; }
      rc = sf[F_RC];
      op = sf[F_O];
      rgb[0] = sf[F_R]; rgb[1] = sf[F_G]; rgb[2] = sf[F_B];
      const uint32_t b0 = __float_as_uint(rec[R_BB0]), b1 = __float_as_uint(rec[R_BB1]);
      bb[0] = (int)(b0 & 0xffffu) - px0;
      bb[1] = (int)(b0 >> 16) - py0;
      bb[2] = (int)(b1 & 0xffffu) - px0;
      bb[3] = (int)(b1 >> 16) - py0;
    }
    const float bbf[4] = {__int_as_float(bb[0]), __int_as_float(bb[1]), __int_as_float(bb[2]),
                          __int_as_float(bb[3])};
    const bool hitb = work && rect_meets_block(bbf, bx, by);
    float acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.f;
    if (__ballot(hitb) != 0ull) {
      const float fbx = (float)bx;
      for (int row = 0; row < 8; ++row) {
        const float ly = (float)(by + row);
        const float Y = ly - hy, YY = Y * Y;
        const float rd0 = fmaf(YY, qd[5], fmaf(Y, qd[2], qd[0]));
        const float rd1 = fmaf(Y, qd[4], qd[1]);
        const float s2r = fmaf(qm[4], Y, qm[5]);
        const float rm0 = fmaf(s2r, s2r, qm[0]);
        const float rm1 = fmaf(qm[2], Y, qm[3]);
        const bool row_in = hitb & (row < rows_in);
        float rs[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int col = 0; col < 8; ++col) {
          const int p = (by + row) * TW + bx + col;
          const float4 pc = s_pc[p];
          const float X = (fbx + (float)col) - hx;
          const float dd = fmaf(X, rd1, fmaf(X * X, qd[3], rd0));
          const float s1 = fmaf(qm[1], X, rm1);
          const float mm = fmaf(s1, s1, rm0);
          const bool f = row_in & (col < cols_in) & (dd >= FLT_MIN) & (mm <= rc * dd) &
                         (pos < __float_as_int(pc.x));
          if (__ballot(f) == 0ull) continue;   // uniform: no blended fragment here
          const float4 pg = s_pg[p];
          // alpha exactly as the forward forms it (0 off the fragments)
          const float inv = rcp_fast(dd);
          const float r2 = mm * inv;
          const float e = exp2_fast(r2 * kNegHalfLog2e);
          const float araw = op * e;
          const bool unclamped = araw <= amax;
          const float alpha = f ? (unclamped ? araw : amax) : 0.f;
          const float om = 1.f - alpha;
          const float incl = wave_scan_mul(om);
          float excl = __shfl_up(incl, 1, 64);
          if (lane == 0) excl = 1.f;
          const float Ti = pc.y * excl;
          const float gc = fmaf(pg.z, rgb[2], fmaf(pg.y, rgb[1], pg.x * rgb[0]));
          const float term = alpha * Ti * gc;
          const float isum = wave_scan_add(term);
          const float gP = pc.z + isum;   // G . (colour sum up to and including i)
          // the pixel's carries past this chunk
          const float tot_m = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(incl), 63));
          const float tot_s = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(isum), 63));
          if (lane == 0) s_pc[p] = make_float4(pc.x, pc.y * tot_m, pc.z + tot_s, 0.f);
          if (f) {
            ++nfr;
            const float dLda = Ti * gc - (pg.w - gP) * rcp_fast(om);
            const float wc = alpha * Ti;
            acc[13] = fmaf(wc, pg.x, acc[13]);
            acc[14] = fmaf(wc, pg.y, acc[14]);
            acc[15] = fmaf(wc, pg.z, acc[15]);
            const float g = unclamped ? dLda : 0.f;
            acc[12] = fmaf(g, e, acc[12]);
            const float w1 = -alpha * g * inv;   // weight of m
            const float w2 = -w1 * r2;           // weight of d
            rs[0] += w2;
            rs[3] += w1;
            const float fc = (float)col, fc2 = (float)(col * col);
            rs[1] = fmaf(fc, w2, rs[1]);
            rs[2] = fmaf(fc2, w2, rs[2]);
            rs[4] = fmaf(fc, w1, rs[4]);
            rs[5] = fmaf(fc2, w1, rs[5]);
          }
        }
        if constexpr (BX > 1) {
          rs[2] = fmaf(fbx, fmaf(fbx, rs[0], 2.f * rs[1]), rs[2]);
          rs[1] = fmaf(fbx, rs[0], rs[1]);
          rs[5] = fmaf(fbx, fmaf(fbx, rs[3], 2.f * rs[4]), rs[5]);
          rs[4] = fmaf(fbx, rs[3], rs[4]);
        }
        const float ly2 = ly * ly;
        acc[0] += rs[0];
        acc[1] += rs[1];
        acc[2] = fmaf(ly, rs[0], acc[2]);
        acc[3] += rs[2];
        acc[4] = fmaf(ly, rs[1], acc[4]);
        acc[5] = fmaf(ly2, rs[0], acc[5]);
        acc[6] += rs[3];
        acc[7] += rs[4];
        acc[8] = fmaf(ly, rs[3], acc[8]);
        acc[9] += rs[5];
        acc[10] = fmaf(ly, rs[4], acc[10]);
        acc[11] = fmaf(ly2, rs[3], acc[11]);
      }
    }
    if constexpr (NB > 1) {
      // the blocks' sums for each instance, added in block order
#pragma unroll
      for (int k = 0; k < 16; ++k) s_red[(wave * 16 + k) * 64 + lane] = acc[k];
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          float t = s_red[k * 64 + lane];
#pragma unroll
          for (int b2 = 1; b2 < NB; ++b2) t += s_red[(b2 * 16 + k) * 64 + lane];
          acc[k] = t;
        }
      }
      __syncthreads();
    }
    if (wave == 0 && active) {
      const int64_t vg = (int64_t)ti.v * cfg.n + gid;
      const uint32_t slot = tslot_slot(w.tslots[vg], ti.tx, ti.ty);
      if ((uint64_t)slot < (uint64_t)w.capacity) {
        // (lanes past the last blended position were not staged: their
        // moments are zero, so the origin does not matter)
        write_partial(acc, (float)(px0 - ox), (float)(py0 - oy),
                      w.partials + (int64_t)slot * kPartialFloats);
      }
    }
  }
}

template <int TW, int TH, bool PERSIST>
__global__ void __launch_bounds__(TW * TH)
    k_raster_bwd_sorted(Ws w, ViewSet vs, KCfg cfg, const float *__restrict__ state,
                        const uint32_t *__restrict__ vals) {
  if (front_failed(w)) return;
  uint32_t nfr = 0;
#define HTGS_BWDS_BODY(T) bwd_tile_sorted<TW, TH>(T, w, vs, cfg, state, vals, nfr)
  HTGS_FOR_TILES(PERSIST, kQueueBwd, HTGS_BWDS_BODY);
#undef HTGS_BWDS_BODY
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) nfr += (uint32_t)__shfl_xor((int)nfr, off, 64);
  if ((threadIdx.x & 63) == 0 && nfr) count_add(w.frags_bwd, (unsigned long long)nfr);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Workgroups of a persistent launch: as many as can be resident at once.
static int resident_blocks(const void *kernel, int threads, int tiles) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int n = per_cu * cus;
  return n < tiles ? n : (tiles > 0 ? tiles : 1);
}
template <int KMAX, int TW, int TH, int BM, bool EXACT>
static hipError_t fwd_launch_bm(const Ws &w, const ViewSet &vs, const KCfg &cfg, float *state,
                                const uint32_t *vals, hipStream_t s) {
  if (cfg.persistent) {
    auto *kern = k_raster_fwd<KMAX, TW, TH, BM, EXACT, true>;
    const int blocks = resident_blocks((const void *)kern, TW * TH, vs.total_tiles);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(TW * TH), 0, s, w, vs, cfg, state, vals);
  } else {
    auto *kern = k_raster_fwd<KMAX, TW, TH, BM, EXACT, false>;
    const int blocks = 8 * ((vs.total_tiles + 7) / 8);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(TW * TH), 0, s, w, vs, cfg, state, vals);
  }
  return hipGetLastError();
}

template <int KMAX, int TW, int TH, bool EXACT>
static hipError_t fwd_launch(const Ws &w, const ViewSet &vs, const KCfg &cfg, float *state,
                             const uint32_t *vals, hipStream_t s) {
  if constexpr (TW == 8) {
    if (cfg.batch_mult == 2) return fwd_launch_bm<KMAX, TW, TH, 2, EXACT>(w, vs, cfg, state, vals, s);
  }
  return fwd_launch_bm<KMAX, TW, TH, 1, EXACT>(w, vs, cfg, state, vals, s);
}

template <int KMAX, int TW, int TH, bool EXACT>
static hipError_t bwd_launch(const Ws &w, const ViewSet &vs, const KCfg &cfg, const float *state,
                             const uint32_t *vals, hipStream_t s) {
  constexpr int BT = 64 * bwd_waves<TW, TH>();
  if (cfg.persistent) {
    auto *kern = k_raster_bwd<KMAX, TW, TH, EXACT, true>;
    const int blocks = resident_blocks((const void *)kern, BT, vs.total_tiles);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(BT), 0, s, w, vs, cfg, state, vals);
  } else {
    auto *kern = k_raster_bwd<KMAX, TW, TH, EXACT, false>;
    const int blocks = 8 * ((vs.total_tiles + 7) / 8);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(BT), 0, s, w, vs, cfg, state, vals);
  }
  return hipGetLastError();
}

int kmax_for(int K) {
  if (K <= 1) return 1;
  if (K <= 2) return 2;
  if (K <= 4) return 4;
  if (K <= 8) return 8;
  if (K <= 16) return 16;
  return 32;
}

#define HTGS_KX(FN, KM, TW_, TH_, ...)                                          \
  (cfg.K == (KM) ? FN<KM, TW_, TH_, true>(__VA_ARGS__) : FN<KM, TW_, TH_, false>(__VA_ARGS__))
#define HTGS_DISPATCH(FN, ...)                                                   \
  do {                                                                           \
    const int km = kmax_for(cfg.K);                                              \
    if (cfg.tile_w == 8 && cfg.tile_h == 8) {                                    \
      switch (km) {                                                              \
        case 1: return HTGS_KX(FN, 1, 8, 8, __VA_ARGS__);                        \
        case 2: return HTGS_KX(FN, 2, 8, 8, __VA_ARGS__);                        \
        case 4: return HTGS_KX(FN, 4, 8, 8, __VA_ARGS__);                        \
        case 8: return HTGS_KX(FN, 8, 8, 8, __VA_ARGS__);                        \
        case 16: return HTGS_KX(FN, 16, 8, 8, __VA_ARGS__);                      \
        default: return HTGS_KX(FN, 32, 8, 8, __VA_ARGS__);                      \
      }                                                                          \
    } else if (cfg.tile_w == 16 && cfg.tile_h == 8) {                            \
      switch (km) {                                                              \
        case 1: return HTGS_KX(FN, 1, 16, 8, __VA_ARGS__);                       \
        case 2: return HTGS_KX(FN, 2, 16, 8, __VA_ARGS__);                       \
        case 4: return HTGS_KX(FN, 4, 16, 8, __VA_ARGS__);                       \
        case 8: return HTGS_KX(FN, 8, 16, 8, __VA_ARGS__);                       \
        case 16: return HTGS_KX(FN, 16, 16, 8, __VA_ARGS__);                     \
        default: return HTGS_KX(FN, 32, 16, 8, __VA_ARGS__);                     \
      }                                                                          \
    } else if (cfg.tile_w == 32 && cfg.tile_h == 8) {                            \
      switch (km) {                                                              \
        case 1: return HTGS_KX(FN, 1, 32, 8, __VA_ARGS__);                       \
        case 2: return HTGS_KX(FN, 2, 32, 8, __VA_ARGS__);                       \
        case 4: return HTGS_KX(FN, 4, 32, 8, __VA_ARGS__);                       \
        case 8: return HTGS_KX(FN, 8, 32, 8, __VA_ARGS__);                       \
        default: return HTGS_KX(FN, 16, 32, 8, __VA_ARGS__);                     \
      }                                                                          \
    } else {                                                                     \
      switch (km) {                                                              \
        case 1: return HTGS_KX(FN, 1, 16, 16, __VA_ARGS__);                      \
        case 2: return HTGS_KX(FN, 2, 16, 16, __VA_ARGS__);                      \
        case 4: return HTGS_KX(FN, 4, 16, 16, __VA_ARGS__);                      \
        case 8: return HTGS_KX(FN, 8, 16, 16, __VA_ARGS__);                      \
        default: return HTGS_KX(FN, 16, 16, 16, __VA_ARGS__);                    \
      }                                                                          \
    }                                                                            \
  } while (0)

template <int TW, int TH>
static hipError_t fwd_sorted_launch(const Ws &w, const ViewSet &vs, const KCfg &cfg, float *state,
                                    const uint32_t *vals, hipStream_t s) {
  if (cfg.persistent) {
    auto *kern = k_raster_fwd_sorted<TW, TH, true>;
    const int blocks = resident_blocks((const void *)kern, TW * TH, vs.total_tiles);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(TW * TH), 0, s, w, vs, cfg, state, vals);
  } else {
    auto *kern = k_raster_fwd_sorted<TW, TH, false>;
    const int blocks = 8 * ((vs.total_tiles + 7) / 8);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(TW * TH), 0, s, w, vs, cfg, state, vals);
  }
  return hipGetLastError();
}

hipError_t launch_raster_fwd(const Ws &w, const ViewSet &vs, const KCfg &cfg, float *state,
                             const uint32_t *vals, hipStream_t s) {
  if (cfg.sorted) {
    if (cfg.tile_w == 8 && cfg.tile_h == 8) return fwd_sorted_launch<8, 8>(w, vs, cfg, state, vals, s);
    if (cfg.tile_w == 16 && cfg.tile_h == 8) return fwd_sorted_launch<16, 8>(w, vs, cfg, state, vals, s);
    if (cfg.tile_w == 32 && cfg.tile_h == 8) return fwd_sorted_launch<32, 8>(w, vs, cfg, state, vals, s);
    return fwd_sorted_launch<16, 16>(w, vs, cfg, state, vals, s);
  }
  HTGS_DISPATCH(fwd_launch, w, vs, cfg, state, vals, s);
}

template <int TW, int TH>
static hipError_t bwd_sorted_launch(const Ws &w, const ViewSet &vs, const KCfg &cfg,
                                    const float *state, const uint32_t *vals, hipStream_t s) {
  if (cfg.persistent) {
    auto *kern = k_raster_bwd_sorted<TW, TH, true>;
    const int blocks = resident_blocks((const void *)kern, TW * TH, vs.total_tiles);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(TW * TH), 0, s, w, vs, cfg, state, vals);
  } else {
    auto *kern = k_raster_bwd_sorted<TW, TH, false>;
    const int blocks = 8 * ((vs.total_tiles + 7) / 8);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(TW * TH), 0, s, w, vs, cfg, state, vals);
  }
  return hipGetLastError();
}

hipError_t launch_raster_bwd(const Ws &w, const ViewSet &vs, const KCfg &cfg, const float *state,
                             const uint32_t *vals, hipStream_t s) {
  if (cfg.sorted) {
    if (cfg.tile_w == 8 && cfg.tile_h == 8) return bwd_sorted_launch<8, 8>(w, vs, cfg, state, vals, s);
    if (cfg.tile_w == 16 && cfg.tile_h == 8) return bwd_sorted_launch<16, 8>(w, vs, cfg, state, vals, s);
    if (cfg.tile_w == 32 && cfg.tile_h == 8) return bwd_sorted_launch<32, 8>(w, vs, cfg, state, vals, s);
    return bwd_sorted_launch<16, 16>(w, vs, cfg, state, vals, s);
  }
  HTGS_DISPATCH(bwd_launch, w, vs, cfg, state, vals, s);
}

}  // namespace htgs
