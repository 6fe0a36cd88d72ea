// libnep: HIP kernels and C ABI for one NEP loss-and-gradient evaluation on
// MI355X (gfx950).  The declarations and contracts are in include/nep.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/nep.h"
#include "nep_kernels.h"

namespace nep {

// =============================================================== neighbors
// One thread per atom i scans the atoms j of its own structure.  For each j
// the per-axis test |(x_j - x_i) + s L| < rc keeps the candidate shifts, and
// every candidate (j, s) is tested exactly with the float64 predicate of
// Eq. 2, evaluated without fused multiply-add.  j runs ascending and the
// shifts in code order, so the lists come out in canonical order.
// IEEE double product and sum with one rounding each.  The library is built
// with floating-point contraction, and d^2 = (dx dx + dy dy) + dz dz of the
// predicate must not become fused multiply-adds (a pair within an ulp of rc
// can change sides), so the squares and their sums are single instructions
// the compiler cannot merge.
__device__ __forceinline__ double mul_d(double a, double b) {
  double r;
  asm("v_mul_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double add_d(double a, double b) {
  double r;
  asm("v_add_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double dist2_d(double dx, double dy, double dz) {
  return add_d(add_d(mul_d(dx, dx), mul_d(dy, dy)), mul_d(dz, dz));
}

__device__ __forceinline__ unsigned axis_candidates(double d0, double L, double rc) {
  unsigned m = 0;
  if (fabs(__dadd_rn(d0, -L)) < rc) m |= 1u;
  if (fabs(d0) < rc) m |= 2u;
  if (fabs(__dadd_rn(d0, L)) < rc) m |= 4u;
  return m;
}

// One atom per group of 8 lanes; lane s scans the s-th contiguous eighth of
// the atom's structure, so concatenating the lanes' entries in lane order
// keeps the canonical (j, code) order.  A count pass and an exclusive scan
// over the group give each lane its write offset; a second pass writes.
//
// Fast decision.  When every cell edge is at least 2(rc + delta) and at most
// kNbrFastL, at most one image of j lies within rc + delta, and the single
// precision minimum image finds it.  Its squared distance is then within
// 3e-3 A^2 of the float64 value, far inside the margins of the shell
// |r - rc| < delta = 0.01 A (at least 0.0199 A^2 for rc >= 1 A), so pairs
// outside the shell are decided in single precision and only pairs in the
// shell, and every pair of smaller or larger cells, take the float64 test.
//
// Positions of the atoms j that a block's 32 atoms scan are staged in LDS in
// tiles of kNbrTile atoms; every lane of the block walks the same tiles.
constexpr int kNbrThreads = 256;   // threads per block
constexpr int kNbrAPB = kNbrThreads / 8;   // atoms per block
constexpr int kNbrTile = 1024;
constexpr int kNbrBuf = 24;   // entries buffered per lane (angular mask: 32 bits), plus a scratch slot
constexpr float kNbrDelta = 0.01f;
constexpr float kNbrFastL = 512.0f;

struct ScanCtx {
  int i;
  double xi, yi, zi, Lx, Ly, Lz, xy, xz, yz, rcR, rcR2, rcA2;
  float xf, yf, zf, Lxf, Lyf, Lzf, xyf, xzf, yzf, ilx, ily, ilz;
  float inR2, outR2, inA2, outA2;
  bool fast;
};

// a tile of positions in LDS holding atoms [base, base + kNbrTile)
struct PosTile {
  const float* x;
  const float* y;
  const float* z;
  int base;
};

// A value the compiler cannot see through.  The float64 paths below run for
// few candidates of the single-image scan; taking their inputs through this
// keeps their conversions inside the branch instead of being computed ahead
// of the test for every candidate.
__device__ __forceinline__ int opaque_int(int v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ float opaque_float(float v) {
  asm volatile("" : "+v"(v));
  return v;
}

// float64 predicate of Eq. 2 for the pair (i, j) over the candidate shifts;
// calls emit(j, code, is_angular) in ascending code order
template <class Emit>
__device__ __forceinline__ void exact_pair(const ScanCtx& c, const PosTile& t, int j, Emit& emit) {
  const int q = opaque_int(j - t.base);
  const double x0 = __dadd_rn((double)t.x[q], -c.xi);
  const unsigned mx = axis_candidates(x0, c.Lx, c.rcR);
  if (!mx) return;
  const double y0 = __dadd_rn((double)t.y[q], -c.yi);
  const unsigned my = axis_candidates(y0, c.Ly, c.rcR);
  if (!my) return;
  const double z0 = __dadd_rn((double)t.z[q], -c.zi);
  const unsigned mz = axis_candidates(z0, c.Lz, c.rcR);
  if (!mz) return;
  for (unsigned bx = mx; bx; bx &= bx - 1u) {
    const int sx = __builtin_ctz(bx);
    const double dx = sx == 1 ? x0 : __dadd_rn(x0, sx == 0 ? -c.Lx : c.Lx);
    const double dx2 = mul_d(dx, dx);
    for (unsigned by = my; by; by &= by - 1u) {
      const int sy = __builtin_ctz(by);
      const double dy = sy == 1 ? y0 : __dadd_rn(y0, sy == 0 ? -c.Ly : c.Ly);
      const double dxy = add_d(dx2, mul_d(dy, dy));
      for (unsigned bz = mz; bz; bz &= bz - 1u) {
        const int sz = __builtin_ctz(bz);
        const int code = 9 * sx + 3 * sy + sz;
        const double dz = sz == 1 ? z0 : __dadd_rn(z0, sz == 0 ? -c.Lz : c.Lz);
        const double d2 = add_d(dxy, mul_d(dz, dz));
        if (d2 < c.rcR2 && !(j == c.i && code == 13)) emit(j, code, d2 < c.rcA2);
      }
    }
  }
}

// The same predicate in a triclinic cell with edge vectors a = (Lx, 0, 0),
// b = (xy, Ly, 0), c = (xz, yz, Lz): d = (x_j - x_i) + sa a + sb b + sc c with
// each component summed left to right, dx = ((x0 + sa Lx) + sb xy) + sc xz,
// dy = (y0 + sb Ly) + sc yz, dz = z0 + sc Lz (the products are exact).  dz
// prunes sc, dy prunes (sb, sc), then dx is formed per surviving shift.
template <class Emit>
__device__ __forceinline__ void exact_pair_tri(const ScanCtx& c, const PosTile& t, int j, Emit& emit) {
  const int q = opaque_int(j - t.base);
  const double z0 = __dadd_rn((double)t.z[q], -c.zi);
  const unsigned mz = axis_candidates(z0, c.Lz, c.rcR);
  if (!mz) return;
  const double y0 = __dadd_rn((double)t.y[q], -c.yi);
  double dyv[9], dzv[3];
#pragma unroll
  for (int sc = 0; sc < 3; ++sc) dzv[sc] = sc == 1 ? z0 : __dadd_rn(z0, sc == 0 ? -c.Lz : c.Lz);
  unsigned myz = 0;
#pragma unroll
  for (int sb = 0; sb < 3; ++sb) {
    const double yb = sb == 1 ? y0 : __dadd_rn(y0, sb == 0 ? -c.Ly : c.Ly);
#pragma unroll
    for (int sc = 0; sc < 3; ++sc) {
      const double dy = sc == 1 ? yb : __dadd_rn(yb, sc == 0 ? -c.yz : c.yz);
      dyv[3 * sb + sc] = dy;
      myz |= (((mz >> sc) & 1u) && fabs(dy) < c.rcR) ? (1u << (3 * sb + sc)) : 0u;
    }
  }
  if (!myz) return;
  const double x0 = __dadd_rn((double)t.x[q], -c.xi);
#pragma unroll
  for (int sa = 0; sa < 3; ++sa) {
    const double xa = sa == 1 ? x0 : __dadd_rn(x0, sa == 0 ? -c.Lx : c.Lx);
#pragma unroll
    for (int sb = 0; sb < 3; ++sb) {
      const double xb = sb == 1 ? xa : __dadd_rn(xa, sb == 0 ? -c.xy : c.xy);
#pragma unroll
      for (int sc = 0; sc < 3; ++sc) {
        if (!((myz >> (3 * sb + sc)) & 1u)) continue;
        const double dx = sc == 1 ? xb : __dadd_rn(xb, sc == 0 ? -c.xz : c.xz);
        const double dy = dyv[3 * sb + sc], dz = dzv[sc];
        const double d2 = dist2_d(dx, dy, dz);
        const int code = 9 * sa + 3 * sb + sc;
        if (d2 < c.rcR2 && !(j == c.i && code == 13)) emit(j, code, d2 < c.rcA2);
      }
    }
  }
}

template <bool kTri, class Emit>
__device__ __forceinline__ void exact_any(const ScanCtx& c, const PosTile& t, int j, Emit& emit) {
  if constexpr (kTri)
    exact_pair_tri(c, t, j, emit);
  else
    exact_pair(c, t, j, emit);
}

// Single-precision minimum image: e = x_j - x_i minus the lattice vector
// H k, k the rounded fractional coordinates of e (H upper triangular, so
// f_c = e_z / Lz, f_b = (e_y - yz f_c) / Ly, f_a = (e_x - xy f_b - xz f_c) / Lx).
// In an orthorhombic cell this is the per-axis rounding.
template <bool kTri>
__device__ __forceinline__ void min_image(const ScanCtx& c, float& ex, float& ey, float& ez, float& kx, float& ky,
                                          float& kz) {
  if constexpr (kTri) {
    const float fc = ez * c.ilz;
    const float fb = (ey - c.yzf * fc) * c.ily;
    const float fa = (ex - c.xyf * fb - c.xzf * fc) * c.ilx;
    kx = rintf(fa);
    ky = rintf(fb);
    kz = rintf(fc);
    ex = ex - c.Lxf * kx - c.xyf * ky - c.xzf * kz;
    ey = ey - c.Lyf * ky - c.yzf * kz;
    ez -= c.Lzf * kz;
  } else {
    kx = rintf(ex * c.ilx);
    ky = rintf(ey * c.ily);
    kz = rintf(ez * c.ilz);
    ex -= c.Lxf * kx;
    ey -= c.Lyf * ky;
    ez -= c.Lzf * kz;
  }
}

// float64 squared length of the image s = -k of j, in the predicate's order
// (the products k L are exact, k being 0 or +-1, so contracting them is harmless)
template <bool kTri>
__device__ __forceinline__ double image_d2(const ScanCtx& c, float px, float py, float pz, float kx, float ky,
                                           float kz) {
  double dx = __dadd_rn(__dadd_rn((double)px, -c.xi), -(double)kx * c.Lx);
  double dy = __dadd_rn(__dadd_rn((double)py, -c.yi), -(double)ky * c.Ly);
  const double dz = __dadd_rn(__dadd_rn((double)pz, -c.zi), -(double)kz * c.Lz);
  if constexpr (kTri) {
    dx = __dadd_rn(__dadd_rn(dx, -(double)ky * c.xy), -(double)kz * c.xz);
    dy = __dadd_rn(dy, -(double)kz * c.yz);
  }
  return dist2_d(dx, dy, dz);
}

template <bool kTri, class Emit>
__device__ __forceinline__ void scan_range(const ScanCtx& c, const PosTile& t, int jb, int je, Emit& emit) {
  for (int j = jb; j < je; ++j) {
    if (c.fast) {
      const int q = j - t.base;
      const float px = t.x[q], py = t.y[q], pz = t.z[q];
      float ex = px - c.xf, ey = py - c.yf, ez = pz - c.zf, kx, ky, kz;
      min_image<kTri>(c, ex, ey, ez, kx, ky, kz);
      const float r2 = ex * ex + ey * ey + ez * ez;
      if (r2 >= c.outR2) continue;
      if (r2 < c.inR2 && fabsf(kx) <= 1.f && fabsf(ky) <= 1.f && fabsf(kz) <= 1.f) {
        // shift s = -k on each axis; code 9(sx+1) + 3(sy+1) + (sz+1)
        const int code = 9 * (1 - (int)kx) + 3 * (1 - (int)ky) + (1 - (int)kz);
        if (j == c.i && code == 13) continue;
        bool ang = r2 < c.inA2;
        if (!ang && r2 < c.outA2) ang = image_d2<kTri>(c, px, py, pz, kx, ky, kz) < c.rcA2;
        emit(j, code, ang);
        continue;
      }
    }
    exact_any<kTri>(c, t, j, emit);
  }
}

// The buffered decision of one candidate j at (px, py, pz).  Outside the
// shell it is made without branches: the entry is written to the lane's next
// buffer slot and the count only advances when the pair is inside, so a
// later entry overwrites a rejected one (slot kNbrBuf takes the writes once
// the buffer is full).  Pairs in the shell branch to the float64 predicate.
template <bool kTri, class Keep>
__device__ __forceinline__ void keep_one(const ScanCtx& c, const PosTile& t, int j, float px, float py, float pz,
                                         uint32_t* buf, int& nR, int& nA, uint32_t& angmask, Keep& keep) {
  float ex = px - c.xf, ey = py - c.yf, ez = pz - c.zf, kx, ky, kz;
  min_image<kTri>(c, ex, ey, ez, kx, ky, kz);
  const float r2 = ex * ex + ey * ey + ez * ez;
  // k is 0 or +-1 for positions inside the cell (the position flag's
  // condition), so the shift s = -k always has a code
  const int code = 13 - (int)fmaf(9.f, kx, fmaf(3.f, ky, kz));
  const bool decided = r2 < c.inR2;
  const bool in = decided & ((j != c.i) | (code != 13));   // bitwise: no branch per candidate
  bool ang = r2 < c.inA2;
  buf[kNbrThreads * min(nR, kNbrBuf)] = ((uint32_t)j << 5) | (uint32_t)(code & 31);
  if (in && !ang && r2 < c.outA2)
    ang = image_d2<kTri>(c, opaque_float(px), opaque_float(py), opaque_float(pz), kx, ky, kz) < c.rcA2;
  angmask |= (in && ang && nR < kNbrBuf) ? (1u << nR) : 0u;
  nR += in ? 1 : 0;
  nA += (in && ang) ? 1 : 0;
  if (!decided && r2 < c.outR2) exact_any<kTri>(c, t, j, keep);
}

// The buffered scan of the single pass over [jb, je); cells too small or too
// large for the single-image test take the float64 predicate for every pair.
template <bool kTri, class Keep>
__device__ __forceinline__ void scan_keep(const ScanCtx& c, const PosTile& t, int jb, int je, uint32_t* buf,
                                          int& nR, int& nA, uint32_t& angmask, Keep& keep) {
  // one loop per case: a shared loop let the float64 coordinate differences
  // of the exact path be computed ahead of the test for every candidate
  if (!c.fast) {
    for (int j = jb; j < je; ++j) exact_any<kTri>(c, t, j, keep);
    return;
  }
  for (int j = jb; j < je; ++j) {
    const int q = j - t.base;
    keep_one<kTri>(c, t, j, t.x[q], t.y[q], t.z[q], buf, nR, nA, angmask, keep);
  }
}

// Triclinic cells.  Every neighbor lies among the 27 images when the
// positions' fractional coordinates are in [0, 1) and each perpendicular
// width of the cell is at least rc: the fractional coordinates of a vector
// shorter than rc are then below 1 in magnitude.  Positions are accepted with
// fractional coordinates in [-kFracTol, 1 + kFracTol) and widths from
// rc / (1 - 2 kFracTol) up, which keeps the same bound.  The single-image fast
// decision needs each width at least 2 (rc + delta): an image within
// rc + delta then has fractional coordinates of magnitude below 1/2 by a
// margin of delta / (2 (rc + delta)), so the rounded fractional coordinates
// select it.
constexpr double kFracTol = 1e-5;

struct CellCheck {
  bool box_ok, pos_ok, fast_ok;
};

// perpendicular widths V / |b x c|, V / |c x a|, V / |a x b| of the cell
__device__ __forceinline__ void cell_widths(const ScanCtx& c, double& ha, double& hb, double& hc) {
  const double bc_x = c.Ly * c.Lz, bc_y = -c.xy * c.Lz, bc_z = c.xy * c.yz - c.Ly * c.xz;
  const double V = c.Lx * c.Ly * c.Lz;
  ha = fabs(V) / sqrt(bc_x * bc_x + bc_y * bc_y + bc_z * bc_z);
  hb = fabs(c.Ly * c.Lz) / sqrt(c.Lz * c.Lz + c.yz * c.yz);
  hc = fabs(c.Lz);
}

template <bool kTri>
__device__ __forceinline__ CellCheck check_cell(const ScanCtx& c, float rcR, float rcA) {
  CellCheck k;
  const float wide = 2.0f * (rcR + kNbrDelta);
  const bool small = c.Lxf <= kNbrFastL && c.Lyf <= kNbrFastL && c.Lzf <= kNbrFastL && rcA >= 1.0f;
  const bool tilted = kTri && (c.xyf != 0.f || c.xzf != 0.f || c.yzf != 0.f);
  if (!tilted) {
    k.pos_ok = c.xf >= 0.f && c.xf < c.Lxf && c.yf >= 0.f && c.yf < c.Lyf && c.zf >= 0.f && c.zf < c.Lzf;
    k.box_ok = c.Lxf >= rcR && c.Lyf >= rcR && c.Lzf >= rcR;
    k.fast_ok = c.Lxf >= wide && c.Lyf >= wide && c.Lzf >= wide && small;
    return k;
  }
  double ha, hb, hc;
  cell_widths(c, ha, hb, hc);
  const double hmin = fmin(ha, fmin(hb, hc));
  k.box_ok = c.Lxf > 0.f && c.Lyf > 0.f && c.Lzf > 0.f && hmin * (1.0 - 2.0 * kFracTol) >= (double)rcR;
  const double fc = c.zi / c.Lz;
  const double fb = (c.yi - c.yz * fc) / c.Ly;
  const double fa = (c.xi - c.xy * fb - c.xz * fc) / c.Lx;
  k.pos_ok = fa >= -kFracTol && fa < 1.0 + kFracTol && fb >= -kFracTol && fb < 1.0 + kFracTol &&
             fc >= -kFracTol && fc < 1.0 + kFracTol;
  k.fast_ok = hmin >= (double)wide && small && fabsf(c.xyf) <= kNbrFastL && fabsf(c.xzf) <= kNbrFastL &&
              fabsf(c.yzf) <= kNbrFastL;
  return k;
}

// The scan context of atom i of structure st at (x, y, z): cell, cutoffs and
// the shell bounds of the single-precision decision.
template <bool kTri>
__device__ __forceinline__ CellCheck init_ctx(const NbrArgs& a, int st, int i, float x, float y, float z,
                                              ScanCtx& c) {
  c.i = i;
  c.Lxf = a.box[3 * st];
  c.Lyf = a.box[3 * st + 1];
  c.Lzf = a.box[3 * st + 2];
  c.xyf = kTri ? a.tilt[3 * st] : 0.f;
  c.xzf = kTri ? a.tilt[3 * st + 1] : 0.f;
  c.yzf = kTri ? a.tilt[3 * st + 2] : 0.f;
  c.xf = x;
  c.yf = y;
  c.zf = z;
  c.xi = c.xf;
  c.yi = c.yf;
  c.zi = c.zf;
  c.Lx = c.Lxf;
  c.Ly = c.Lyf;
  c.Lz = c.Lzf;
  c.xy = c.xyf;
  c.xz = c.xzf;
  c.yz = c.yzf;
  const CellCheck ck = check_cell<kTri>(c, a.rcR, a.rcA);
  c.rcR = (double)a.rcR;
  c.rcR2 = c.rcR * c.rcR;  // exact: a float squared in double
  c.rcA2 = (double)a.rcA * (double)a.rcA;
  c.ilx = 1.0f / c.Lxf;
  c.ily = 1.0f / c.Lyf;
  c.ilz = 1.0f / c.Lzf;
  c.fast = ck.fast_ok;
  c.inR2 = (a.rcR - kNbrDelta) * (a.rcR - kNbrDelta);
  c.outR2 = (a.rcR + kNbrDelta) * (a.rcR + kNbrDelta);
  c.inA2 = (a.rcA - kNbrDelta) * (a.rcA - kNbrDelta);
  c.outA2 = (a.rcA + kNbrDelta) * (a.rcA + kNbrDelta);
  return ck;
}

// kCells: the cell search ran before and wrote the lists of the atoms with
// acell[i] >= 0
template <bool kTri, bool kCells>
__global__ __launch_bounds__(kNbrThreads) void k_neighbors(NbrArgs a) {
  __shared__ float tx[kNbrTile], ty[kNbrTile], tz[kNbrTile];
  __shared__ uint32_t nbuf[kNbrThreads * (kNbrBuf + 1)];
  __shared__ int jr[2];
  const int s = threadIdx.x & 7;
  const int b0 = xcd_block() * kNbrAPB;
  const int i = b0 + (threadIdx.x >> 3);
  const bool live = i < a.N;
  const int ic = live ? i : a.N - 1;
  int lo = 0, hi = a.S;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.aoff[mid] <= ic) lo = mid; else hi = mid;
  }
  const int st = lo;
  const int a0 = max(a.aoff[st], 0), a1 = min(a.aoff[st + 1], a.N);
  // the block's atoms are consecutive, so their structures cover [jr[0], jr[1])
  if (threadIdx.x == 0) jr[0] = a0;
  if (i == min(b0 + kNbrAPB - 1, a.N - 1) && s == 0) jr[1] = a1;
  ScanCtx c;
  const CellCheck ck = init_ctx<kTri>(a, st, ic, a.pos[ic], a.pos[a.N + ic], a.pos[2 * a.N + ic], c);
  int fl = 0;
  if (!ck.pos_ok) fl |= FL_POS;
  bool ok = live;
  if (!ck.box_ok) {
    fl |= FL_BOX;
    ok = false;
  }
  if (live && s == 0) {
    a.astruct[i] = st;
    const int ti = a.type[i];
    if (ti < 0 || ti >= a.T) fl |= FL_TYPE;
  }
  // atoms whose lists the cell search wrote (it leaves acell[i] >= 0)
  const bool mine = live && !(kCells && a.acell[ic] >= 0);
  const int len = ok && mine ? a1 - a0 : 0;
  const int jb = a0 + (len * s) / 8, je = a0 + (len * (s + 1)) / 8;
  // after the cell search, a block with no atom left to scan walks no tiles
  bool any = true;
  if constexpr (kCells)
    any = __syncthreads_or(len > 0);
  else
    __syncthreads();
  const int jlo = jr[0], jhi = any ? jr[1] : jr[0];
  // walks the tiles of [jlo, jhi); this lane scans [b, e) of each
  auto sweep = [&](int b, int e, auto&& scan) {
    for (int t0 = jlo; t0 < jhi; t0 += kNbrTile) {
      const int tn = min(kNbrTile, jhi - t0);
      for (int q = threadIdx.x; q < tn; q += kNbrThreads) {
        tx[q] = a.pos[t0 + q];
        ty[q] = a.pos[a.N + t0 + q];
        tz[q] = a.pos[2 * a.N + t0 + q];
      }
      __syncthreads();
      const PosTile t{tx, ty, tz, t0};
      scan(t, max(b, t0), min(e, t0 + tn));
      __syncthreads();
    }
  };
  // one scan: each lane keeps its entries in an LDS buffer (angular
  // membership as a bit mask), and after the 8-lane prefix copies them to
  // their slots; a lane with more than kNbrBuf entries makes the whole block
  // rescan and write directly
  uint32_t* mybuf = nbuf + threadIdx.x;   // slot u at mybuf[kNbrThreads u]
  int nR = 0, nA = 0;
  uint32_t angmask = 0;
  auto keep = [&](int j, int code, bool ang) {
    if (nR < kNbrBuf) {
      mybuf[kNbrThreads * nR] = ((uint32_t)j << 5) | (uint32_t)code;
      angmask |= ang ? (1u << nR) : 0u;
    }
    ++nR;
    nA += ang ? 1 : 0;
  };
  sweep(jb, je,
        [&](const PosTile& t, int b2, int e2) { scan_keep<kTri>(c, t, b2, e2, mybuf, nR, nA, angmask, keep); });
  // inclusive prefix over the 8 lanes of the atom
  int pR = nR, pA = nA;
#pragma unroll
  for (int d = 1; d < 8; d <<= 1) {
    const int uR = __shfl_up(pR, d, 8), uA = __shfl_up(pA, d, 8);
    if (s >= d) {
      pR += uR;
      pA += uA;
    }
  }
  const int totR = __shfl(pR, 7, 8), totA = __shfl(pA, 7, 8);
  int wR = pR - nR, wA = pA - nA;
  const size_t col = (size_t)c.i;
  const bool spill = nR > kNbrBuf;
  if (mine && !spill) {
    for (int u = 0; u < nR; ++u) {
      const uint32_t e = mybuf[kNbrThreads * u];
      if (wR + u < a.capR) a.idxR[col * a.capR + wR + u] = e;
      if ((angmask >> u) & 1u) {
        if (wA < a.capA) a.idxA[col * a.capA + wA] = e;
        ++wA;
      }
    }
  }
  if (__syncthreads_or(mine && spill)) {
    auto write = [&](int j, int code, bool ang) {
      const uint32_t e = ((uint32_t)j << 5) | (uint32_t)code;
      if (wR < a.capR) a.idxR[col * a.capR + wR] = e;
      ++wR;
      if (ang) {
        if (wA < a.capA) a.idxA[col * a.capA + wA] = e;
        ++wA;
      }
    };
    // angular entries are a subset, so a lane past the radial capacity may
    // still have angular slots to fill
    const bool wr = mine && spill && (wR < a.capR || wA < a.capA);
    sweep(wr ? jb : 0, wr ? je : 0,
          [&](const PosTile& t, int b2, int e2) { scan_range<kTri>(c, t, b2, e2, write); });
  }
  if (mine && s == 0) {
    a.cntR[i] = totR;
    a.cntA[i] = totA;
    if (totR > a.capR || totA > a.capA) fl |= FL_OVERFLOW;
  }
  if (live && s == 0 && fl) atomicOr(a.flags, fl);
}

// Cell-list search of large structures.  A structure of at least
// kCellMinAtoms atoms whose cell takes the single-image decision is cut into
// na x nb x nc bins along its edge vectors, each bin at least rc + kCellPad
// thick across (perpendicular width over the bin count), at least 3 bins per
// axis and no more bins than atoms.  An atom's bin comes from its
// single-precision fractional coordinates; their error, and the accepted
// positions up to 1e-5 outside the cell, move an atom by under 0.006 A for
// cells up to kNbrFastL (twice that is below kCellPad), so two atoms in bins
// that are not adjacent along some axis lie more than rc apart in every
// image.  Each atom then meets as
// candidates exactly the atoms of its 27 surrounding bins and takes the same
// per-candidate decision as the all-pairs scan, so its entries are the same.
// Within rc + delta every j has one image at most (each width is at least
// 2 (rc + delta)), so an entry's rank among the atom's entries by (j, code)
// is its canonical slot.
//
// Bins of structure n have the ids atom_offset[n] + bin (< atom_offset[n+1]);
// the bins are counted, scanned into start offsets, and the binned atoms
// placed bin by bin as (x, y, z, j).  An atom whose lane buffer overflows is
// left to the all-pairs kernel (acell[i] = -1), which runs afterwards.
constexpr int kCellMinAtoms = 1024;     // default smallest structure searched through cell lists
constexpr int kCellMinAtomsLo = 64;     // smallest value a tuning may set
constexpr double kCellPad = 0.05;
constexpr int kScanChunk = 2048;   // bin ids per block of the offset scan

// bins per axis of structure st, (0, 0, 0, 0) for the all-pairs search
template <bool kTri>
__device__ int4 cell_grid(const NbrArgs& a, int st) {
  const int4 none = make_int4(0, 0, 0, 0);
  const int n = a.aoff[st + 1] - a.aoff[st];
  if (n < a.cell_min) return none;
  ScanCtx c;
  if (!init_ctx<kTri>(a, st, a.aoff[st], 0.f, 0.f, 0.f, c).fast_ok) return none;
  double ha, hb, hc;
  cell_widths(c, ha, hb, hc);
  // the single-image cells are at most kNbrFastL wide and rc >= 1 A: at most
  // 512 bins per axis
  const double w = (double)a.rcR + kCellPad;
  int na = (int)(ha / w), nb = (int)(hb / w), nc = (int)(hc / w);
  while ((long long)na * nb * nc > n) {
    if (na >= nb && na >= nc)
      --na;
    else if (nb >= nc)
      --nb;
    else
      --nc;
  }
  if (na < 3 || nb < 3 || nc < 3) return none;
  return make_int4(na, nb, nc, na * nb * nc);
}

// zeroes the bin counts and sets every structure's bins
template <bool kTri>
__global__ __launch_bounds__(256) void k_cell_setup(NbrArgs a) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t <= a.N) a.cell[t] = 0;
  if (t < a.S) a.grid[t] = cell_grid<kTri>(a, t);
}

// bin of each atom of a binned structure and its slot in the bin
template <bool kTri>
__global__ __launch_bounds__(256) void k_cell_bin(NbrArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.N) return;
  int lo = 0, hi = a.S;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.aoff[mid] <= i) lo = mid; else hi = mid;
  }
  const int st = lo;
  a.astruct[i] = st;
  const int4 g = a.grid[st];
  int bin = -1, slot = 0;
  if (g.w > 0) {
    const float x = a.pos[i], y = a.pos[a.N + i], z = a.pos[2 * a.N + i];
    float fa, fb, fc;
    if constexpr (kTri) {
      const float xy = a.tilt[3 * st], xz = a.tilt[3 * st + 1], yz = a.tilt[3 * st + 2];
      fc = z / a.box[3 * st + 2];
      fb = (y - yz * fc) / a.box[3 * st + 1];
      fa = (x - xy * fb - xz * fc) / a.box[3 * st];
    } else {
      fa = x / a.box[3 * st];
      fb = y / a.box[3 * st + 1];
      fc = z / a.box[3 * st + 2];
    }
    // clamped in float (a NaN goes to bin 0; the position flag reports it)
    const int ia = (int)fminf(fmaxf(floorf(fa * (float)g.x), 0.f), (float)(g.x - 1));
    const int ib = (int)fminf(fmaxf(floorf(fb * (float)g.y), 0.f), (float)(g.y - 1));
    const int ic = (int)fminf(fmaxf(floorf(fc * (float)g.z), 0.f), (float)(g.z - 1));
    bin = a.aoff[st] + (ia * g.y + ib) * g.z + ic;
    slot = atomicAdd(&a.cell[bin], 1);
  }
  a.acell[i] = bin;
  a.aslot[i] = slot;
}

// exclusive prefix over 256 threads; returns the block total
__device__ __forceinline__ int block_exclusive_scan(int v, int& excl, int* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(inc, d, 64);
    if (lane >= d) inc += u;
  }
  if (lane == 63) red[w] = inc;
  __syncthreads();
  int before = 0, total = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    before += q < w ? red[q] : 0;
    total += red[q];
  }
  __syncthreads();
  excl = before + inc - v;
  return total;
}

// per chunk of kScanChunk bin ids: the sum of the counts
__global__ __launch_bounds__(256) void k_cell_part(int n, const int* __restrict__ cnt, int* __restrict__ part) {
  __shared__ int red[4];
  const int b = blockIdx.x * kScanChunk + threadIdx.x * 8;
  int v = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) v += b + q < n ? cnt[b + q] : 0;
  int excl;
  const int tot = block_exclusive_scan(v, excl, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// counts -> start offsets in place over [0, n), and the total at [n]
__global__ __launch_bounds__(256) void k_cell_start(int n, int* __restrict__ cell, const int* __restrict__ part) {
  __shared__ int red[4];
  int off = 0;
  for (int q = threadIdx.x; q < (int)blockIdx.x; q += 256) off += part[q];
  int excl;
  off = block_exclusive_scan(off, excl, red);
  const int b = blockIdx.x * kScanChunk + threadIdx.x * 8;
  int v[8], sum = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    v[q] = b + q < n ? cell[b + q] : 0;
    sum += v[q];
  }
  const int tot = block_exclusive_scan(sum, excl, red);
  int run = off + excl;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (b + q < n) cell[b + q] = run;
    run += v[q];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) cell[n] = off + tot;
}

// binned atoms bin by bin as (x, y, z, j)
__global__ __launch_bounds__(256) void k_cell_place(NbrArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.N) return;
  const int bin = a.acell[i];
  if (bin < 0) return;
  a.cpos[a.cell[bin] + a.aslot[i]] =
      make_float4(a.pos[i], a.pos[a.N + i], a.pos[2 * a.N + i], __int_as_float(i));
}

// Lists of the binned atoms, 8 lanes per atom taking the candidates of the 27
// bins in turn.  Blocks take the atoms in bin order, so a block's atoms share
// most of their candidates.
template <bool kTri>
__global__ __launch_bounds__(kNbrThreads) void k_cell_neighbors(NbrArgs a) {
  __shared__ uint32_t nbuf[kNbrThreads * (kNbrBuf + 1)];
  // the first ceil(M / 32) blocks work, renumbered over the XCDs among themselves
  const int M = a.cell[a.N], nbw = (M + kNbrAPB - 1) / kNbrAPB;
  if ((int)blockIdx.x >= nbw) return;
  const int b0 = xcd_block_of(blockIdx.x, nbw) * kNbrAPB;
  const int s = threadIdx.x & 7;
  const int k = b0 + (int)(threadIdx.x >> 3);
  const bool live = k < M;
  const float4 me = a.cpos[min(k, M - 1)];
  const int i = __float_as_int(me.w);
  const int st = a.astruct[i];
  const int4 g = a.grid[st];
  ScanCtx c;
  init_ctx<kTri>(a, st, i, me.x, me.y, me.z, c);   // single-image decision: c.fast holds
  const int base = a.aoff[st];
  const int loc = a.acell[i] - base;
  const int kc = loc % g.z, kb = (loc / g.z) % g.y, ka = loc / (g.y * g.z);
  const PosTile t{a.pos, a.pos + a.N, a.pos + 2 * a.N, 0};
  uint32_t* mybuf = nbuf + threadIdx.x;   // slot u at mybuf[kNbrThreads u]
  int nR = 0, nA = 0;
  uint32_t angmask = 0;
  auto keep = [&](int j, int code, bool ang) {
    if (nR < kNbrBuf) {
      mybuf[kNbrThreads * nR] = ((uint32_t)j << 5) | (uint32_t)code;
      angmask |= ang ? (1u << nR) : 0u;
    }
    ++nR;
    nA += ang ? 1 : 0;
  };
  // bins kc-1, kc, kc+1 of a row are consecutive ids, split in two runs when
  // the row wraps
  // (kc = 0: [0, 1] and [nc-1]; kc = nc-1: [0] and [nc-2, nc-1]; else [kc-1, kc+1])
  const bool edge = kc == 0 || kc == g.z - 1;
  const int r0lo = edge ? 0 : kc - 1, r0hi = kc == 0 ? 1 : (edge ? 0 : kc + 1);
  const int r1lo = kc == 0 ? g.z - 1 : (edge ? g.z - 2 : 1), r1hi = edge ? g.z - 1 : 0;
  int run = 0;   // candidates before the current run; lane s takes every 8th
  if (live) {
    for (int da = -1; da <= 1; ++da) {
      const int xa = ka + da < 0 ? g.x - 1 : (ka + da == g.x ? 0 : ka + da);
      for (int db = -1; db <= 1; ++db) {
        const int yb = kb + db < 0 ? g.y - 1 : (kb + db == g.y ? 0 : kb + db);
        const int row = base + (xa * g.y + yb) * g.z;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int lo = h ? r1lo : r0lo, hi = h ? r1hi : r0hi;
          if (lo > hi) continue;
          const int cb = a.cell[row + lo], ce = a.cell[row + hi + 1];
          // four of this lane's candidates per step, their loads issued
          // together (a run of three bins is about three candidates per lane)
          for (int q0 = cb + ((s - run) & 7); q0 < ce; q0 += 32) {
            float4 p[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) p[u] = a.cpos[min(q0 + 8 * u, ce - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (q0 + 8 * u < ce)
                keep_one<kTri>(c, t, __float_as_int(p[u].w), p[u].x, p[u].y, p[u].z, mybuf, nR, nA, angmask, keep);
          }
          run += ce - cb;
        }
      }
    }
  }
  __syncthreads();
  int most = nR, ntv[8], atv[8];
  uint32_t mtv[8];
#pragma unroll
  for (int d = 1; d < 8; d <<= 1) most = max(most, __shfl_xor(most, d, 8));
  int totR = 0, totA = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    ntv[q] = __shfl(nR, q, 8);
    atv[q] = __shfl(nA, q, 8);
    mtv[q] = __shfl(angmask, q, 8);
    totR += ntv[q];
    totA += atv[q];
  }
  const bool spill = most > kNbrBuf;
  if (live && !spill) {
    const uint32_t* gbuf = nbuf + (threadIdx.x & ~7);
    const size_t col = (size_t)i;
    // the atom's entries, taken in lane order, are ranked k = s, s + 8, ...,
    // so the 8 lanes share the work evenly whatever each lane found
    for (int k = s; k < totR; k += 8) {
      int q0 = 0, u0 = k;
#pragma unroll
      for (int q = 0; q < 7; ++q)
        if (q == q0 && u0 >= ntv[q]) {
          u0 -= ntv[q];
          q0 = q + 1;
        }
      const uint32_t e = gbuf[q0 + kNbrThreads * u0];
      uint32_t m0 = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) m0 = q == q0 ? mtv[q] : m0;
      int rR = 0, rA = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        for (int u2 = 0; u2 < ntv[q]; ++u2) {
          const int lt = gbuf[q + kNbrThreads * u2] < e ? 1 : 0;
          rR += lt;
          rA += lt & (int)((mtv[q] >> u2) & 1u);
        }
      }
      if (rR < a.capR) a.idxR[col * a.capR + rR] = e;
      if (((m0 >> u0) & 1u) && rA < a.capA) a.idxA[col * a.capA + rA] = e;
    }
    if (s == 0) {
      a.cntR[i] = totR;
      a.cntA[i] = totA;
      if (totR > a.capR || totA > a.capA) atomicOr(a.flags, FL_OVERFLOW);
    }
  }
  if (live && spill && s == 0) a.acell[i] = -1;
}

// Position of the key in a sorted row holding m valid entries (of cap), -1
// if absent.  The last entry of every run of 8 (four independent loads at a
// time) picks the run, then the run's 8 entries (two 16-byte loads) give the
// position.  Entries past m are treated as larger than any key.
__device__ __forceinline__ int row_find(const uint32_t* __restrict__ row, int m, int cap, uint32_t key) {
  const int nrun = (m + 7) >> 3;
  int below = 0;
  for (int r0 = 0; r0 < nrun; r0 += 4) {
    uint32_t last[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      // unconditional loads from inside the row, then the mask
      const int q = 8 * (r0 + u) + 7;
      const uint32_t x = row[min(q, cap - 1)];
      last[u] = (r0 + u < nrun && q < m) ? x : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) below += (r0 + u < nrun && last[u] < key) ? 1 : 0;
  }
  int pos = -1;
  if (below < nrun) {
    const int b = 8 * below;   // the key, if present, lies in entries b .. b + 7
    uint32_t v[8];
    if (b + 8 <= cap && (((uintptr_t)(row + b)) & 15) == 0) {
      const uint4 x = *reinterpret_cast<const uint4*>(row + b);
      const uint4 y = *reinterpret_cast<const uint4*>(row + b + 4);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
      v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = b + u < cap ? row[b + u] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b + u < m && v[u] == key) pos = b + u;
  }
  return pos;
}

// Reverse index: for entry k = (j, s) of atom i, the position of (i, -s) in
// j's list (-1 if the capacity cut it off).  The two entries of a pair are
// found by one search: the one with the larger key, (j, s) > (i, self) (j > i,
// or j = i and s past the zero shift), searches j's list and writes both
// slots.  Those entries are the tail of i's sorted list, so LPA lanes per
// atom take only them; an entry below (i, self) searches for itself only
// when its partner may be missing, i.e. j's list overflowed.
template <int LPA>
__device__ __forceinline__ void reverse_block(int blk, int N, const uint32_t* __restrict__ idx,
                                              const int* __restrict__ cnt, int cap, int* __restrict__ rev) {
  const int s = threadIdx.x % LPA;
  const int i = blk * (256 / LPA) + threadIdx.x / LPA;
  if (i >= N) return;
  const int n = min(cnt[i], cap);
  const uint32_t self = ((uint32_t)i << 5) | 13u;
  const uint32_t* li = idx + (size_t)i * cap;
  int low = 0;
  for (int k = s; k < n; k += LPA) {
    const uint32_t e = li[k];
    if (e < self) {
      ++low;
      const int j = (int)(e >> 5);
      if (cnt[j] > cap)
        rev[(size_t)i * cap + k] = row_find(idx + (size_t)j * cap, cap, cap, ((uint32_t)i << 5) | (26u - (e & 31u)));
    }
  }
#pragma unroll
  for (int d = 1; d < LPA; d <<= 1) low += __shfl_xor(low, d, LPA);
  for (int k = low + s; k < n; k += LPA) {
    const uint32_t e = li[k];
    const int j = (int)(e >> 5);
    const int pos = row_find(idx + (size_t)j * cap, min(cnt[j], cap), cap, ((uint32_t)i << 5) | (26u - (e & 31u)));
    rev[(size_t)i * cap + k] = pos;
    if (pos >= 0) rev[(size_t)j * cap + pos] = k;
  }
}

constexpr int kRevLPAR = 16, kRevLPAA = 4;   // lanes per atom: radial, angular lists

// Both lists in one launch (they are independent, and neither fills the GPU
// alone): the first nbR blocks, in XCD-aware order, take the radial list.
struct RevArgs {
  int N, nbR;
  const uint32_t* idxR;
  const int* cntR;
  int capR;
  int* revR;
  const uint32_t* idxA;
  const int* cntA;
  int capA;
  int* revA;
};

__global__ __launch_bounds__(256) void k_reverse(RevArgs a) {
  const int b = xcd_block();
  if (b < a.nbR)
    reverse_block<kRevLPAR>(b, a.N, a.idxR, a.cntR, a.capR, a.revR);
  else
    reverse_block<kRevLPAA>(b - a.nbR, a.N, a.idxA, a.cntA, a.capA, a.revA);
}

// ============================================================ species order
// Atoms are laid out by (species, angular neighbor count descending), with
// ties in atom order: every wavefront then holds one species and atoms of
// similar pair counts, so the pair loops of its 8 atoms end together.  The
// key of atom i is t * kOrdBuckets + (kOrdBuckets - 1 - min(nA_i, kOrdBuckets - 1)),
// and a counting sort over keys keeps the layout deterministic.
constexpr int kOrdBlk = 1024;      // atoms per order block
constexpr int kOrdBuckets = 64;
constexpr int kOrdMaxK = 8 * kOrdBuckets;   // keys of up to 8 species
constexpr int kSegAlign = 32;  // species segments start on multiples of the atoms per block

__device__ __forceinline__ int order_key(int t, int T, int nA) {
  if (t < 0 || t >= T) return -1;
  return t * kOrdBuckets + (kOrdBuckets - 1 - min(max(nA, 0), kOrdBuckets - 1));
}

struct OrderArgs {
  int N, Npad, T, nblk;
  const int* type;
  const int* cntA;
  int* blk;     // [nblk][K] key counts, then offsets
  int* seg;     // [2T] species segment start and count
  int* order;   // [Npad]
};

// LDS of the order bodies (ints)
constexpr int kOrdCountLds = kOrdMaxK;
constexpr int kOrdScanLds = 2 * kOrdMaxK + 16;
constexpr int kOrdScatterLds = (kOrdBlk / kWave) * kOrdMaxK;

// Key counts of order block ob (kOrdBlk atoms).
template <int NT>
__device__ __forceinline__ void order_count_body(const OrderArgs& a, int ob, int* cnt) {
  const int K = a.T * kOrdBuckets;
  for (int q = threadIdx.x; q < K; q += NT) cnt[q] = 0;
  __syncthreads();
  for (int u = 0; u < kOrdBlk; u += NT) {
    const int i = ob * kOrdBlk + u + threadIdx.x;
    if (i < a.N) {
      const int key = order_key(a.type[i], a.T, a.cntA[i]);
      if (key >= 0) atomicAdd(&cnt[key], 1);
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < K; q += NT) a.blk[(size_t)ob * K + q] = cnt[q];
  __syncthreads();
}

// One block: key totals, their exclusive scan in key order with each species
// segment starting on a multiple of kSegAlign atoms, then the per-block
// offsets.  seg[2t], seg[2t+1] = start and count of species t.  Each key's
// rows are split into P parts; a thread takes (key, part) slots.
template <int NT>
__device__ __forceinline__ void order_scan_body(const OrderArgs& a, int* sh) {
  static_assert(2 * NT >= kOrdMaxK, "two keys per thread");
  const int K = a.T * kOrdBuckets;
  const int P = max(1, NT / K);
  int* part = sh;                 // [K * P] row sums of each slot
  int* sc = sh + kOrdMaxK;        // [K] inclusive scan of the key totals
  int* sstart = sc + kOrdMaxK;    // [8]
  const int nslot = K * P;
  // slot q = p K + k of this thread: q = threadIdx.x + r NT
  for (int q = threadIdx.x; q < nslot; q += NT) {
    const int k = q % K, p = q / K;
    const int b0 = (int)((long long)a.nblk * p / P), b1 = (int)((long long)a.nblk * (p + 1) / P);
    int mine = 0;
    for (int b = b0; b < b1; b += 8) {
      int v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = b + u < b1 ? a.blk[(size_t)(b + u) * K + k] : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) mine += v[u];
    }
    part[q] = mine;
  }
  __syncthreads();
  // key totals, two keys per thread (K <= 512), then an inclusive scan of the
  // pair sums (Hillis-Steele over the 256 threads)
  int tot2[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k = 2 * threadIdx.x + h;
    int t = 0;
    if (k < K)
      for (int p = 0; p < P; ++p) t += part[p * K + k];
    tot2[h] = t;
  }
  sc[threadIdx.x] = tot2[0] + tot2[1];
  __syncthreads();
  for (int d = 1; d < NT; d <<= 1) {
    const int v = (int)threadIdx.x >= d ? sc[threadIdx.x - d] : 0;
    __syncthreads();
    sc[threadIdx.x] += v;
    __syncthreads();
  }
  const int incl_pair = sc[threadIdx.x];
  __syncthreads();
  // expand to per-key inclusive sums
  {
    const int k0 = 2 * threadIdx.x;
    if (k0 < K) sc[k0] = incl_pair - tot2[1];
    if (k0 + 1 < K) sc[k0 + 1] = incl_pair;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int start = 0;
    for (int t = 0; t < a.T; ++t) {
      const int lo = t == 0 ? 0 : sc[t * kOrdBuckets - 1];
      const int cnt = sc[(t + 1) * kOrdBuckets - 1] - lo;
      sstart[t] = start - lo;   // aligned start minus the unaligned prefix
      a.seg[2 * t] = start;
      a.seg[2 * t + 1] = cnt;
      start += (cnt + kSegAlign - 1) / kSegAlign * kSegAlign;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nslot; q += NT) {
    const int k = q % K, p = q / K;
    const int b0 = (int)((long long)a.nblk * p / P), b1 = (int)((long long)a.nblk * (p + 1) / P);
    int before = 0, tot = 0;   // rows of earlier parts, and the key's total
    for (int pp = 0; pp < P; ++pp) {
      const int v = part[pp * K + k];
      tot += v;
      before += pp < p ? v : 0;
    }
    int off = sstart[k / kOrdBuckets] + sc[k] - tot + before;
    for (int b = b0; b < b1; b += 8) {
      int v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = b + u < b1 ? a.blk[(size_t)(b + u) * K + k] : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (b + u < b1) a.blk[(size_t)(b + u) * K + k] = off;
        off += v[u];
      }
    }
  }
  __syncthreads();
}

// Rank of each atom of order block ob among the atoms of its key: lanes
// before it in its wavefront (one ballot per distinct key in the wavefront),
// then the wavefronts before it in the block.  The block's kOrdBlk atoms are
// taken NT at a time; wcnt holds [kOrdBlk / 64][K] counts.
template <int NT>
__device__ __forceinline__ void order_scatter_body(const OrderArgs& a, int ob, int* wcnt) {
  constexpr int NR = kOrdBlk / NT;   // rounds
  constexpr int NWR = NT / kWave;    // wavefronts per round
  const int K = a.T * kOrdBuckets;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int q = threadIdx.x; q < (kOrdBlk / kWave) * K; q += NT) wcnt[q] = 0;
  __syncthreads();
  int key[NR], rank[NR];
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = ob * kOrdBlk + r * NT + threadIdx.x;
    key[r] = i < a.N ? order_key(a.type[i], a.T, a.cntA[i]) : -1;
    rank[r] = 0;
    const int vw = r * NWR + wid;
    unsigned long long rem = __ballot(key[r] >= 0);
    while (rem) {
      const int leader = __ffsll(rem) - 1;
      const int kk = __shfl(key[r], leader, kWave);
      const unsigned long long m = __ballot(key[r] == kk);
      if (key[r] == kk) rank[r] = __popcll(m & below);
      if (lane == leader) wcnt[vw * K + kk] = __popcll(m);
      rem &= ~m;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (key[r] >= 0) {
      const int i = ob * kOrdBlk + r * NT + threadIdx.x;
      const int vw = r * NWR + wid;
      int before = 0;
      for (int w = 0; w < vw; ++w) before += wcnt[w * K + key[r]];
      a.order[a.blk[(size_t)ob * K + key[r]] + before + rank[r]] = i;
    }
  }
  __syncthreads();
}

// the separate kernels: a block of kOrdBlk threads per order block, 512
// threads for the scan (the counts run in k_reverse_count)
__global__ __launch_bounds__(512) void k_order_scan(OrderArgs a) {
  __shared__ int sh[kOrdScanLds];
  order_scan_body<512>(a, sh);
}

__global__ __launch_bounds__(kOrdBlk) void k_order_scatter(OrderArgs a) {
  __shared__ int wcnt[kOrdScatterLds];
  order_scatter_body<kOrdBlk>(a, blockIdx.x, wcnt);
}

// The reverse index and the species-order counts in one launch (both read
// only the neighbor lists): the first nrev blocks, numbered XCD-aware among
// themselves, take the reverse index; the rest count one order block each
// and clear the order slots.
__global__ __launch_bounds__(256) void k_reverse_count(RevArgs r, OrderArgs o, int nrev) {
  __shared__ int cnt[kOrdCountLds];
  if ((int)blockIdx.x < nrev) {
    const int b = xcd_block_of(blockIdx.x, nrev);
    if (b < r.nbR)
      reverse_block<kRevLPAR>(b, r.N, r.idxR, r.cntR, r.capR, r.revR);
    else
      reverse_block<kRevLPAA>(b - r.nbR, r.N, r.idxA, r.cntA, r.capA, r.revA);
    return;
  }
  const int ob = blockIdx.x - nrev;
  for (int q = ob * 256 + threadIdx.x; q < o.Npad; q += o.nblk * 256) o.order[q] = -1;
  order_count_body<256>(o, ob, cnt);
}

// ================================================================= helpers
// c^A of every species pair (I, J) staged in LDS with rows padded to KAP = 4k
// floats: a pair reads its 4-aligned row with a few wide LDS reads instead of
// selecting each coefficient by the neighbor's species
template <int T, int NA, int KA>
struct CTab {
  static constexpr int KAP = (KA + 3) & ~3;
  static constexpr int size = T * T * NA * KAP;
};

template <int T, int NA, int KA>
__device__ __forceinline__ void stage_ctab(float* ct, const float* __restrict__ cA) {
  constexpr int KAP = CTab<T, NA, KA>::KAP, SZ = CTab<T, NA, KA>::size, U = 8;
  // U words per thread per round, the loads issued before the stores
  for (int base = 0; base < SZ; base += U * (int)blockDim.x) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = base + u * (int)blockDim.x + (int)threadIdx.x;
      const int k = q % KAP, r = q / KAP;
      v[u] = (q < SZ && k < KA) ? cA[r * KA + k] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = base + u * (int)blockDim.x + (int)threadIdx.x;
      if (q < SZ) ct[q] = v[u];
    }
  }
}

struct PairGeom {
  int j;
  float dx, dy, dz, r, inv_r;
};

// cell of a structure: edge vectors a = (Lx, 0, 0), b = (xy, Ly, 0),
// c = (xz, yz, Lz); the tilts are read only for triclinic batches
struct Cell {
  float Lx, Ly, Lz, xy, xz, yz;
};

template <bool kTri>
__device__ __forceinline__ Cell load_cell(const float* __restrict__ box, const float* __restrict__ tilt, int st) {
  Cell c;
  c.Lx = box[3 * st];
  c.Ly = box[3 * st + 1];
  c.Lz = box[3 * st + 2];
  c.xy = kTri ? tilt[3 * st] : 0.f;
  c.xz = kTri ? tilt[3 * st + 1] : 0.f;
  c.yz = kTri ? tilt[3 * st + 2] : 0.f;
  return c;
}

// d = x_j - x_i + sa a + sb b + sc c for the entry's image shift
template <bool kTri>
__device__ __forceinline__ PairGeom pair_geom(uint32_t e, const float* __restrict__ pos, int N, float xi, float yi,
                                              float zi, const Cell& cl) {
  PairGeom g;
  g.j = (int)(e >> 5);
  float sx, sy, sz;
  decode_shift(e & 31u, sx, sy, sz);
  g.dx = (pos[g.j] - xi) + sx * cl.Lx;
  g.dy = (pos[N + g.j] - yi) + sy * cl.Ly;
  g.dz = (pos[2 * N + g.j] - zi) + sz * cl.Lz;
  if constexpr (kTri) {
    g.dx += sy * cl.xy + sz * cl.xz;
    g.dy += sz * cl.yz;
  }
  const float r2 = g.dx * g.dx + g.dy * g.dy + g.dz * g.dz;
  g.inv_r = rsq_hw(r2);
  g.r = r2 * g.inv_r;
  return g;
}

// LDS written by one lane and read by another lane of the same wavefront: a
// wavefront's LDS instructions complete in issue order, so it is enough that
// the compiler keeps every memory access on its side of this point.
__device__ __forceinline__ void lds_lane_exchange() { asm volatile("" ::: "memory"); }

// ========================================================= atom groups
// Per-atom kernels run 8 lanes per atom, 8 atoms per wavefront and 32 atoms
// per block.  Lane s = l & 7 of an atom's group splits the radial pairs
// (pairs k = s, s+8, ...); for the angular sums the group is 2 harmonic
// groups x 4 pair slots: g = s >> 2 picks the harmonics (l = 1 and 4, or
// l = 2 and 3; 12 each for l <= 4) and p = s & 3 the pairs k = p, p+4, ....
// The hidden layer is split over hidden units mu = s, s+8, ....
// Atoms are in species order with species segments aligned to 8, so every
// wavefront evaluates a single species' network.
constexpr int kLPA = 8;                    // lanes per atom
constexpr int kAPB = 256 / kLPA;           // atoms per block
constexpr int kAPW = kWave / kLPA;         // atoms per wavefront
static_assert(kSegAlign % kAPB == 0, "species segments must align to blocks (one species per block)");
}  // namespace nep
#include "nep_highl.h"
namespace nep {

template <int LM>
struct HSplit {
  static constexpr int nA0 = LM >= 1 ? 3 : 0;   // group 0: l = 1 ...
  static constexpr int nB0 = LM >= 4 ? 9 : 0;   // ... and l = 4
  static constexpr int nA1 = LM >= 2 ? 5 : 0;   // group 1: l = 2 ...
  static constexpr int nB1 = LM >= 3 ? 7 : 0;   // ... and l = 3
  static constexpr int YG = (nA0 + nB0 > nA1 + nB1) ? nA0 + nB0 : nA1 + nB1;
  // harmonic index of compact entry i of group g, -1 for padding
  static constexpr int q(int g, int i) {
    return g == 0 ? (i < nA0 ? i : (i - nA0 < nB0 ? 15 + (i - nA0) : -1))
                  : (i < nA1 ? 3 + i : (i - nA1 < nB1 ? 8 + (i - nA1) : -1));
  }
};

// B_q of compact entry i for this lane's harmonic group
template <class HS, int Y>
__device__ __forceinline__ float hsel(int g, int i, const float (&B)[Y]) {
  const int q0 = HS::q(0, i), q1 = HS::q(1, i);
  const float b0 = q0 >= 0 ? B[q0] : 0.f;
  const float b1 = q1 >= 0 ? B[q1] : 0.f;
  return g ? b1 : b0;
}
template <class HS>
__device__ __forceinline__ float csel(int g, int i) {
  const int q0 = HS::q(0, i), q1 = HS::q(1, i);
  return g ? (q1 >= 0 ? clm(q1) : 0.f) : (q0 >= 0 ? clm(q0) : 0.f);
}

// The per-atom rows of the angular sums (S, Sdot, Sbar, A), in LDS and in
// HBM, are kept in harmonic-group order: entry e of group g of channel n at
// n YR + g YG + e, YR = 2 YG.  A lane of group g then reaches its entries as
// its base plus constant offsets, with no per-entry address selects (which
// the adjoint otherwise kept live, and spilled, across its network phase).
template <int LM>
struct HRow {
  static constexpr int YG = HSplit<LM>::YG, YR = 2 * YG;
  // whether entry e of group g is a harmonic (not padding)
  static constexpr bool real(int g, int e) { return HSplit<LM>::q(g, e) >= 0; }
};

// E' of q_nl for the two l blocks of harmonic group g (l = 1, 4 or l = 2, 3)
template <int NR, int NA, int L3, int D>
__device__ __forceinline__ void ep_blocks(const float (&Ep)[D], int n, int g, float& eA, float& eB) {
  float e1 = 0.f, e2 = 0.f, e3 = 0.f, e4 = 0.f;
  if constexpr (L3 >= 1) e1 = Ep[NR + n];
  if constexpr (L3 >= 2) e2 = Ep[NR + NA + n];
  if constexpr (L3 >= 3) e3 = Ep[NR + 2 * NA + n];
  if constexpr (L3 >= 4) e4 = Ep[NR + 3 * NA + n];
  eA = g ? e2 : e1;
  eB = g ? e3 : e4;
}

struct GroupCtx {
  int s, g, p, al, pa, i, I;
  bool valid;
};

// lane roles and the atom of this lane; every lane of the block stays alive
__device__ __forceinline__ GroupCtx group_ctx(const int* __restrict__ order, const int* __restrict__ type, int Npad,
                                              int vb) {
  GroupCtx c;
  c.s = threadIdx.x & (kLPA - 1);
  c.g = c.s >> 2;
  c.p = c.s & 3;
  c.al = threadIdx.x / kLPA;
  c.pa = vb * kAPB + c.al;
  const int iraw = c.pa < Npad ? order[c.pa] : -1;
  c.valid = iraw >= 0;
  const unsigned long long vm = __ballot(c.valid);
  const int lead = vm ? __ffsll(vm) - 1 : 0;
  const int ilead = vm ? __shfl(iraw, lead, kWave) : 0;
  c.i = c.valid ? iraw : ilead;
  c.I = __builtin_amdgcn_readfirstlane(vm ? type[ilead] : 0);
  return c;
}

// Species of block vb's atoms.  Segments start on block boundaries, so a
// block holds one species, and its first position is an atom unless the
// whole block is padding.
__device__ __forceinline__ int block_species(const int* __restrict__ order, const int* __restrict__ type, int vb) {
  const int ip = order[vb * kAPB];
  return ip >= 0 ? type[ip] : 0;
}

// LDS words of the staged weights: whole 64-word rows, so that the direct
// loads below never write past them
__host__ __device__ constexpr int weights_words(int H, int DP) { return (H * DP + 2 * H + 63) / 64 * 64; }

// Species I's W0 (rows padded to DP words), b0 and w1 into LDS with direct
// global-to-LDS loads (gfx950 global_load_lds_dword: each wavefront writes
// 64 consecutive words and holds no registers for them), issued at the
// block's start and waited for by wait_weights() before the network, so
// their latency overlaps the pair passes instead of preceding them.  W0's
// padding words (d >= D, never read) receive W0[0][0].
__device__ __forceinline__ void stage_weights_async(float* wl, const float* __restrict__ nn, int nn_stride, int I,
                                                    int H, int D, int DP) {
  const int WS = H * DP + 2 * H, WSP = weights_words(H, DP);
  const float* w = nn + (size_t)I * nn_stride;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
  for (int c0 = wv * kWave; c0 < WSP; c0 += nw * kWave) {
    const int q = c0 + lane;
    const int mu = q / DP, d = q % DP;
    const int src = q < H * DP ? (d < D ? mu * D + d : 0) : (q < WS ? H * D + (q - H * DP) : 0);
    __builtin_amdgcn_global_load_lds(w + src, (__attribute__((address_space(3))) void*)(wl + c0), 4, 0, 0);
  }
}
__device__ __forceinline__ void wait_weights() { __builtin_amdgcn_s_waitcnt(0); }

// ================================================================= forward
// Per atom: radial sums F[J][k] = sum_{j of type J} f_k(r_ij) give
// q_n = sum_{J,k} c^R_{IJnk} F[J][k] (Eqs. 5-6); angular sums S_nlm (Eq. 8)
// give q_nl (Eq. 7) and the 4-/5-body invariants; the per-species network
// gives E_i and E' = dE_i/dG (D1.1-D1.5).  With forces on, every listed
// pair's partial force f_ij = dE_i/dr_ij is stored (C3.6) with this atom's
// share -sum_j f_ij (x) r_ij of the virial.
// Block vb (32 atoms of the species order); lds: lds_forward bytes.
template <class C, bool kTri>
__device__ __forceinline__ void forward_body(const FwdArgs& a, int vb, float* lds) {
  constexpr int T = C::T, NR = C::NR, NA = C::NA, KR = C::KR, KA = C::KA, Y = C::Y, D = C::D, LM = C::LMAX;
  constexpr int L3 = C::L3, L4 = C::L4, L5 = C::L5;
  using HS = HSplit<LM>;
  constexpr int YG = HS::YG;
  constexpr int DP = (D + 3) & ~3;
  const int H = a.H;
  constexpr int YR = HRow<LM>::YR;
  constexpr int RW = DP + NA * YR;        // LDS row per atom: G, S (group order)
  using CT = CTab<T, NA, KA>;
  float* ctab = lds;                     // [T][T][NA][KAP]
  float* wl = lds + CT::size;            // weights of the block's species
  float* rows = wl + weights_words(H, DP);   // [kAPB][RW]
  stage_ctab<T, NA, KA>(ctab, a.cA);
  __syncthreads();
  // issued after the barrier (a barrier waits for every outstanding load) and
  // waited for before the next one, ahead of the network
  if (a.do_mlp) stage_weights_async(wl, a.nn, a.nn_stride, block_species(a.order, a.type, vb), H, D, DP);
  const GroupCtx w = group_ctx(a.order, a.type, a.Npad, vb);
  const int N = a.N, i = w.i, I = w.I, pa = w.pa, s = w.s, g = w.g;
  float* row = rows + w.al * RW;
  float* rowS = row + DP;
  const int st = a.astruct[i];
  const Cell cell = load_cell<kTri>(a.box, a.tilt, st);
  const float xi = a.pos[i], yi = a.pos[N + i], zi = a.pos[2 * N + i];
  const int cR_i = a.nb.cntR[i], cA_i = a.nb.cntA[i];
  const int nR = w.valid ? min(cR_i, a.nb.capR) : 0;
  const int nA = w.valid ? min(cA_i, a.nb.capA) : 0;
  const cptr<float> cRI = as_const(a.cR) + (size_t)I * T * NR * KR;

  // ---- radial sums, pairs split over the 8 lanes
  float FR[T][KR];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int k = 0; k < KR; ++k) FR[t][k] = 0.f;
  for (int k = s; k < nR; k += kLPA) {
    const PairGeom q = pair_geom<kTri>(a.nb.idxR[(size_t)i * a.nb.capR + k], a.pos, N, xi, yi, zi, cell);
    float f[KR];
    radial_basis<KR>(q.r, a.inv_rcR, f);
    const int J = a.type[q.j];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const float m = (T == 1 || J == t) ? 1.f : 0.f;
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) FR[t][kk] = fmaf(m, f[kk], FR[t][kk]);
    }
  }
  // the basis sums over the 8 lanes, then q_n = sum c^R F by lane n & 7
  {
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int k = 0; k < KR; ++k) FR[t][k] = grp8_sum(FR[t][k]);
#pragma unroll
    for (int n0 = 0; n0 < NR; n0 += kLPA) {
      const int n = n0 + s;
      if (n < NR) {
        const cptr<float> cn = cRI + n * KR;
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int k = 0; k < KR; ++k) acc = fmaf(cn[t * NR * KR + k], FR[t][k], acc);
        row[n] = acc;
      }
    }
  }

  // ---- angular sums S_nlm: harmonic group g, pairs p, p+4, ...
  float Sg[NA][YG];
#pragma unroll
  for (int n = 0; n < NA; ++n)
#pragma unroll
    for (int e = 0; e < YG; ++e) Sg[n][e] = 0.f;
  for (int k = w.p; k < nA; k += 4) {
    const PairGeom q = pair_geom<kTri>(a.nb.idxA[(size_t)i * a.nb.capA + k], a.pos, N, xi, yi, zi, cell);
    float f[KA];
    radial_basis<KA>(q.r, a.inv_rcA, f);
    const int J = a.type[q.j];
    const float* cJ = ctab + (I * T + J) * NA * CT::KAP;
    float gn[NA];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      float acc = 0.f;
#pragma unroll
      for (int kk = 0; kk < KA; ++kk) acc = fmaf(cJ[n * CT::KAP + kk], f[kk], acc);
      gn[n] = acc;
    }
    float B[Y];
    harm_val<LM>(q.dx * q.inv_r, q.dy * q.inv_r, q.dz * q.inv_r, B);
#pragma unroll
    for (int e = 0; e < YG; ++e) {
      const float b = hsel<HS, Y>(g, e, B);
#pragma unroll
      for (int n = 0; n < NA; ++n) Sg[n][e] = fmaf(gn[n], b, Sg[n][e]);
    }
  }
#pragma unroll
  for (int n = 0; n < NA; ++n)
#pragma unroll
    for (int e = 0; e < YG; ++e) Sg[n][e] = quad_sum(Sg[n][e]);

  // ---- angular descriptors of this lane's harmonic group
  {
    const int nAg = g ? HS::nA1 : HS::nA0;     // size of the first l block
    const int lA = g ? 2 : 1, lB = g ? 3 : 4;
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      float qa = 0.f, qb = 0.f;
#pragma unroll
      for (int e = 0; e < YG; ++e) {
        const float v = csel<HS>(g, e) * Sg[n][e] * Sg[n][e];
        if (e < nAg) qa += v; else qb += v;
      }
      if (w.p == 0) {
        if (lA <= L3) row[NR + (lA - 1) * NA + n] = qa;
        if (lB <= L3) row[NR + (lB - 1) * NA + n] = qb;
      }
    }
    if constexpr (L4 != 0) {
#pragma unroll
      for (int n = 0; n < NA; ++n) {
        const Sym3 M = sym_of(Sg[n][0], Sg[n][1], Sg[n][2], Sg[n][3], Sg[n][4]);
        const float q4 = sym_dot(sym_mul(M, M), M);
        if (g == 1 && w.p == 0) row[NR + L3 * NA + n] = q4;
      }
    }
    if constexpr (L5 != 0) {
#pragma unroll
      for (int n = 0; n < NA; ++n) {
        const float P = Sg[n][0] * Sg[n][0] + Sg[n][1] * Sg[n][1] + Sg[n][2] * Sg[n][2];
        if (g == 0 && w.p == 0) row[NR + L3 * NA + (L4 ? NA : 0) + n] = P * P;
      }
    }
  }
  if (w.p == 0) {
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
      for (int e = 0; e < YG; ++e) {
        rowS[n * YR + g * YG + e] = Sg[n][e];   // zero at padding entries
        if (w.valid && a.Sst) a.Sst[(size_t)(n * YR + g * YG + e) * a.Npad + pa] = Sg[n][e];
      }
  }
  if constexpr (C::YH > 0) {
    // q_nl of l = 5..L3, from k_high_desc
    for (int v = NR + 4 * NA + s; v < NR + L3 * NA; v += kLPA) {
      const float x = a.G[(size_t)v * a.Npad + pa];
      row[v] = w.valid ? x : 0.f;
    }
  }
  wait_weights();   // this wavefront's weight loads have landed; the barrier covers the others'
  __syncthreads();
  float G[D];
#pragma unroll
  for (int v = 0; v < D; ++v) G[v] = row[v];
  if (w.valid) {
#pragma unroll
    for (int v = 0; v < D; ++v)
      if (s == (v & 7)) {
        if (a.G) a.G[(size_t)v * a.Npad + pa] = G[v];
        if (a.Guser) a.Guser[(size_t)v * N + i] = G[v];
      }
  }
  if (!a.do_mlp) return;

  // ---- network: hidden units mu = s, s+8, ... (weights from LDS)
  const float* Wl = wl;
  float Ep[D];
#pragma unroll
  for (int v = 0; v < D; ++v) Ep[v] = 0.f;
  float E = 0.f;
  for (int mu = s; mu < H; mu += kLPA) {
    const float* wr = Wl + mu * DP;
    float z = Wl[H * DP + mu];
#pragma unroll
    for (int v = 0; v < D; ++v) z = fmaf(wr[v], G[v], z);
    const float x = tanh_hw(z);
    const float w1 = Wl[H * DP + H + mu];
    E = fmaf(w1, x, E);
    const float sg = w1 * (1.0f - x * x);
#pragma unroll
    for (int v = 0; v < D; ++v) Ep[v] = fmaf(sg, wr[v], Ep[v]);
    if (w.valid && a.X) a.X[(size_t)mu * a.Npad + pa] = x;
  }
  // E' summed over the 8 lanes, scattered (entry v in lane v & 7), shared
  // through the atom's LDS row (G there has been read)
  {
    float eo[(D + 7) / 8];
    rs_group8(Ep, eo);
#pragma unroll
    for (int r = 0; r < (D + 7) / 8; ++r) {
      const int v = 8 * r + s;
      if (v < D) {
        row[v] = eo[r];
        if (w.valid && a.Ep) a.Ep[(size_t)v * a.Npad + pa] = eo[r];
      }
    }
    lds_lane_exchange();
#pragma unroll
    for (int v = 0; v < D; ++v) Ep[v] = row[v];
  }
  E = grp8_sum(E) + a.nn[(size_t)I * a.nn_stride + H * D + 2 * H];
  if (w.valid) {
    if (s == 0) {
      if (a.eatom) a.eatom[i] = E;
      if (a.eatom2) a.eatom2[i] = E;
    }
  }
  if (!a.do_force) return;

  // ---- radial partial forces: f_ij = (sum_k h_Jk f'_k(r)) r_hat, h_Jk = sum_n E'_n c^R_{IJnk}
  float hR[T][KR];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      float acc = 0.f;
#pragma unroll
      for (int n = 0; n < NR; ++n) acc = fmaf(Ep[n], cRI[(t * NR + n) * KR + k], acc);
      hR[t][k] = acc;
    }
  float vxx = 0.f, vyy = 0.f, vzz = 0.f, vxy = 0.f, vyz = 0.f, vzx = 0.f;
  for (int k = s; k < nR; k += kLPA) {
    const PairGeom q = pair_geom<kTri>(a.nb.idxR[(size_t)i * a.nb.capR + k], a.pos, N, xi, yi, zi, cell);
    float f[KR], fp[KR];
    radial_basis_d<KR>(q.r, a.inv_rcR, f, fp);
    const int J = a.type[q.j];
    float sc = 0.f;
#pragma unroll
    for (int kk = 0; kk < KR; ++kk) {
      float h = hR[0][kk];
#pragma unroll
      for (int t = 1; t < T; ++t) h = (J == t) ? hR[t][kk] : h;
      sc = fmaf(h, fp[kk], sc);
    }
    sc *= q.inv_r;
    const float fx = sc * q.dx, fy = sc * q.dy, fz = sc * q.dz;
    float* fo = a.fR + 3 * ((size_t)i * a.nb.capR + k);
    fo[0] = fx;
    fo[1] = fy;
    fo[2] = fz;
    vxx -= fx * q.dx; vyy -= fy * q.dy; vzz -= fz * q.dz;
    vxy -= fx * q.dy; vyz -= fy * q.dz; vzx -= fz * q.dx;
  }

  // ---- A_nlm = sum_v E'_v dG_v/dS_nlm for this lane's harmonics
  float Ag[NA][YG];
  {
    const int nAg = g ? HS::nA1 : HS::nA0;
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      float Sn[YG];
#pragma unroll
      for (int e = 0; e < YG; ++e) Sn[e] = rowS[n * YR + g * YG + e];
      float eA, eBv;
      ep_blocks<NR, NA, L3, D>(Ep, n, g, eA, eBv);
      float a4[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, a5[3] = {0.f, 0.f, 0.f};
      if constexpr (L4 != 0) {
        const Sym3 M = sym_of(Sn[0], Sn[1], Sn[2], Sn[3], Sn[4]);
        float o[5];
        sym_proj(sym_mul(M, M), o);
        const float e4 = g == 1 ? 3.0f * Ep[NR + L3 * NA + n] : 0.f;
#pragma unroll
        for (int m = 0; m < 5; ++m) a4[m] = e4 * o[m];
      }
      if constexpr (L5 != 0) {
        const float P = Sn[0] * Sn[0] + Sn[1] * Sn[1] + Sn[2] * Sn[2];
        const float e5 = g == 0 ? 4.0f * Ep[NR + L3 * NA + (L4 ? NA : 0) + n] * P : 0.f;
#pragma unroll
        for (int m = 0; m < 3; ++m) a5[m] = e5 * Sn[m];
      }
#pragma unroll
      for (int e = 0; e < YG; ++e) {
        float v = 2.0f * csel<HS>(g, e) * (e < nAg ? eA : eBv) * Sn[e];
        if (e < 5) v += a4[e];
        if (e < 3) v += a5[e];
        Ag[n][e] = v;
      }
    }
  }

  // ---- angular partial forces: f_ij = sum_nlm A_nlm (g'_n r_hat B_lm + g_n grad B_lm);
  //      each harmonic group adds its half, the two halves are summed across lanes
  for (int k = w.p; k < nA; k += 4) {
    const PairGeom q = pair_geom<kTri>(a.nb.idxA[(size_t)i * a.nb.capA + k], a.pos, N, xi, yi, zi, cell);
    const float ux = q.dx * q.inv_r, uy = q.dy * q.inv_r, uz = q.dz * q.inv_r;
    float f[KA], fp[KA];
    radial_basis_d<KA>(q.r, a.inv_rcA, f, fp);
    const int J = a.type[q.j];
    const float* cJ = ctab + (I * T + J) * NA * CT::KAP;
    float gn[NA], gp[NA];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int kk = 0; kk < KA; ++kk) {
        const float c = cJ[n * CT::KAP + kk];
        s0 = fmaf(c, f[kk], s0);
        s1 = fmaf(c, fp[kk], s1);
      }
      gn[n] = s0;
      gp[n] = s1;
    }
    float B[Y];
    harm_val<LM>(ux, uy, uz, B);
    float vv = 0.f;
    float uf[Y];
#pragma unroll
    for (int qq = 0; qq < Y; ++qq) uf[qq] = 0.f;
#pragma unroll
    for (int e = 0; e < YG; ++e) {
      float su = 0.f, sv = 0.f;
#pragma unroll
      for (int n = 0; n < NA; ++n) {
        su = fmaf(Ag[n][e], gn[n], su);
        sv = fmaf(Ag[n][e], gp[n], sv);
      }
      vv = fmaf(sv, hsel<HS, Y>(g, e, B), vv);
      const int q0 = HS::q(0, e), q1 = HS::q(1, e);
      if (q0 >= 0) uf[q0] = g ? uf[q0] : su;
      if (q1 >= 0) uf[q1] = g ? su : uf[q1];
    }
    float gx, gy, gz;
    harm_grad_sum<LM>(ux, uy, uz, uf, gx, gy, gz);
    const float rad = ux * gx + uy * gy + uz * gz;
    float fx = vv * ux + (gx - rad * ux) * q.inv_r;
    float fy = vv * uy + (gy - rad * uy) * q.inv_r;
    float fz = vv * uz + (gz - rad * uz) * q.inv_r;
    // the partner lane (other harmonic group, same pair) runs the same
    // iterations, so the DPP read below only touches active lanes
    fx += xor4_val(fx);
    fy += xor4_val(fy);
    fz += xor4_val(fz);
    if (g == 0) {
      float* fo = a.fA + 3 * ((size_t)i * a.nb.capA + k);
      fo[0] = fx;
      fo[1] = fy;
      fo[2] = fz;
      vxx -= fx * q.dx; vyy -= fy * q.dy; vzz -= fz * q.dz;
      vxy -= fx * q.dy; vyz -= fy * q.dz; vzx -= fz * q.dx;
    }
  }
  vxx = grp8_sum(vxx); vyy = grp8_sum(vyy); vzz = grp8_sum(vzz);
  vxy = grp8_sum(vxy); vyz = grp8_sum(vyz); vzx = grp8_sum(vzx);
  if (w.valid && s == 0) {
    a.wv[i] = vxx;
    a.wv[(size_t)N + i] = vyy;
    a.wv[(size_t)2 * N + i] = vzz;
    a.wv[(size_t)3 * N + i] = vxy;
    a.wv[(size_t)4 * N + i] = vyz;
    a.wv[(size_t)5 * N + i] = vzx;
  }
}

template <class C, bool kTri, int W>
__global__ __launch_bounds__(256, W) void k_forward(FwdArgs a) {
  extern __shared__ __align__(16) float lds[];
  forward_body<C, kTri>(a, blockIdx.x, lds);
}

// F_i = sum_j f_ij - f_ji (Eq. 3), gathering f_ji through the reverse index;
// 16 lanes per atom take list slots s, s + 16, ... (more loads in flight for
// the dependent reverse reads) and are summed by DPP.
constexpr int kGatherLPA = 16;   // default lanes per atom (8 or 16)
template <int LPA>
__device__ __forceinline__ void gather_list(int i, int s, const uint32_t* __restrict__ idx, const int* __restrict__ cnt,
                                            const int* __restrict__ rev, int cap, const float* __restrict__ f,
                                            float& fx, float& fy, float& fz) {
  const int n = min(cnt[i], cap);
  for (int k = s; k < n; k += LPA) {
    const size_t o = (size_t)i * cap + k;
    const int j = (int)(idx[o] >> 5);
    const int rk = rev[o];
    const float* a = f + 3 * o;
    fx += a[0];
    fy += a[1];
    fz += a[2];
    if (rk >= 0) {
      const float* b = f + 3 * ((size_t)j * cap + rk);
      fx -= b[0];
      fy -= b[1];
      fz -= b[2];
    }
  }
}

// logical block vb: atoms vb * (256 / LPA) ..
template <int LPA>
__device__ __forceinline__ void gather_body(int vb, int N, const PairLists& nb, const float* __restrict__ fR,
                                            const float* __restrict__ fA, float* __restrict__ F,
                                            float* __restrict__ Fuser) {
  static_assert(LPA == 8 || LPA == 16, "8 or 16 lanes per atom");
  const int s = threadIdx.x % LPA;
  const int i = vb * (256 / LPA) + threadIdx.x / LPA;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  if (i < N) {
    gather_list<LPA>(i, s, nb.idxR, nb.cntR, nb.revR, nb.capR, fR, fx, fy, fz);
    gather_list<LPA>(i, s, nb.idxA, nb.cntA, nb.revA, nb.capA, fA, fx, fy, fz);
  }
  // the lanes of an atom: 8-lane groups, then (16 lanes) the other half of the row
  fx = grp8_sum(fx);
  fy = grp8_sum(fy);
  fz = grp8_sum(fz);
  if (LPA == 16) {
    fx += dpp<kDppRowRor8>(fx);
    fy += dpp<kDppRowRor8>(fy);
    fz += dpp<kDppRowRor8>(fz);
  }
  if (i < N && s == 0) {
    F[i] = fx;
    F[N + i] = fy;
    F[2 * N + i] = fz;
    if (Fuser) {
      Fuser[i] = fx;
      Fuser[N + i] = fy;
      Fuser[2 * N + i] = fz;
    }
  }
}

template <int LPA>
__global__ __launch_bounds__(256) void k_force_gather(int N, PairLists nb, const float* __restrict__ fR,
                                                      const float* __restrict__ fA, float* __restrict__ F,
                                                      float* __restrict__ Fuser) {
  gather_body<LPA>(xcd_block(), N, nb, fR, fA, F, Fuser);
}

// ==================================================================== loss
// One block per structure: E(n), W(n) and, with labels, the loss terms of
// Eqs. 10-12 and the cotangents dL/dE(n), dL/dF_i, dL/dW(n).  Sums run in
// float64 in a fixed order.
constexpr int kRedBlk = 256;

// Loss of Eqs. 9-12 from the per-structure partials, float64 in a fixed
// order (one block).
constexpr int kLossLds = 3 * kRedBlk * sizeof(double);
__device__ void loss_final_block(int S, int N, float le, float lf, float lv, const double* lpart, float* loss,
                                 int* flags, void* lds) {
  double (*red)[kRedBlk] = reinterpret_cast<double (*)[kRedBlk]>(lds);
  double acc[3] = {0, 0, 0};
  for (int s = threadIdx.x; s < S; s += kRedBlk)
    for (int q = 0; q < 3; ++q) acc[q] += lpart[3 * s + q];
  for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int st = kRedBlk / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double Le = S > 0 ? red[0][0] / S : 0.0;
    const double Lf = N > 0 ? red[1][0] / (3.0 * N) : 0.0;
    const double Lv = S > 0 ? red[2][0] / (6.0 * S) : 0.0;
    const double L = le * Le + lf * Lf + lv * Lv;
    loss[0] = (float)L;
    loss[1] = (float)Le;
    loss[2] = (float)Lf;
    loss[3] = (float)Lv;
    if (flags && !isfinite(L)) atomicOr(flags, FL_NONFINITE);
  }
}

struct StructArgs {
  int S, N;
  const int* aoff;
  const float* eatom;
  const float* wv;
  const float* F;
  const float* Et;
  const float* Ft;
  const float* Wt;
  float le, lf, lv;
  float* Es;
  float* Ws;
  float* Es_user;
  float* Ws_user;
  float* eps;
  float* wbar;
  float* fbar;
  double* lpart;  // [S][3]
  // structures of at least 2 kStructChunk atoms are summed from chunk partials
  int split;
  double* spart;  // [N / kStructChunk + 1][2][8]
};

constexpr int kStructChunk = 1024;

__device__ __forceinline__ int find_struct(const int* __restrict__ aoff, int S, int i) {
  int lo = 0, hi = S;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (aoff[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// Sums over atoms [lo, hi) of one structure: energy, the six virial
// components and the squared force error (acc[0..7]); writes F-bar.
__device__ __forceinline__ void struct_accumulate(const StructArgs& a, int lo, int hi, double* acc) {
  const int N = a.N;
  const bool lab = a.Et != nullptr;
  const float cf = 2.0f * a.lf / (3.0f * (float)max(N, 1));
  for (int i = lo + threadIdx.x; i < hi; i += kRedBlk) {
    acc[0] += a.eatom[i];
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[1 + c] += a.wv[(size_t)c * N + i];
    if (lab) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float d = a.F[(size_t)c * N + i] - a.Ft[(size_t)c * N + i];
        acc[7] += (double)d * d;
        a.fbar[(size_t)c * N + i] = cf * d;
      }
    }
  }
}

// block tree sum of acc[0..7]; the result is in red[q][0]
__device__ __forceinline__ void struct_reduce(double (*red)[kRedBlk], const double* acc) {
#pragma unroll
  for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int st = kRedBlk / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st)
#pragma unroll
      for (int q = 0; q < 8; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + st];
    __syncthreads();
  }
}

// Chunk partials of the large structures: a chunk of kStructChunk atoms
// meets at most two structures of 2 kStructChunk atoms or more, those of its
// first and last atoms (slots 0 and 1).
// chunk vb; lds: 8 kRedBlk doubles
__device__ __forceinline__ void struct_part_body(const StructArgs& a, int vb, void* lds) {
  double (*red)[kRedBlk] = reinterpret_cast<double (*)[kRedBlk]>(lds);
  const int c0 = vb * kStructChunk, c1 = min(c0 + kStructChunk, a.N);
  const int sa = find_struct(a.aoff, a.S, c0), sb = find_struct(a.aoff, a.S, c1 - 1);
  for (int h = 0; h < 2; ++h) {
    const int st = h ? sb : sa;
    if (h && sb == sa) break;
    const int a0 = a.aoff[st], a1 = a.aoff[st + 1];
    if (a1 - a0 < 2 * kStructChunk) continue;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    struct_accumulate(a, max(a0, c0), min(a1, c1), acc);
    struct_reduce(red, acc);
    if (threadIdx.x < 8) a.spart[(2 * (size_t)vb + h) * 8 + threadIdx.x] = red[threadIdx.x][0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kRedBlk) void k_struct_part(StructArgs a) {
  __shared__ double red[8][kRedBlk];
  struct_part_body(a, blockIdx.x, red);
}

constexpr int kStructLds = 8 * kRedBlk * sizeof(double);
// structure s; lds: kStructLds bytes
__device__ __forceinline__ void struct_body(const StructArgs& a, int s, void* lds) {
  double (*red)[kRedBlk] = reinterpret_cast<double (*)[kRedBlk]>(lds);
  const int a0 = a.aoff[s], a1 = a.aoff[s + 1];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const bool lab = a.Et != nullptr;
  if (a.split && a1 - a0 >= 2 * kStructChunk) {
    // chunk b holds this structure in slot 0 if it starts at or before the chunk
    for (int b = a0 / kStructChunk + threadIdx.x; b <= (a1 - 1) / kStructChunk; b += kRedBlk) {
      const int h = a0 > b * kStructChunk ? 1 : 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += a.spart[(2 * (size_t)b + h) * 8 + q];
    }
  } else {
    struct_accumulate(a, a0, a1, acc);
  }
  struct_reduce(red, acc);
  if (threadIdx.x == 0) {
    const double E = red[0][0];
    a.Es[s] = (float)E;
    if (a.Es_user) a.Es_user[s] = (float)E;
    for (int c = 0; c < 6; ++c) {
      a.Ws[6 * s + c] = (float)red[1 + c][0];
      if (a.Ws_user) a.Ws_user[6 * s + c] = (float)red[1 + c][0];
    }
    if (lab) {
      const int n = a1 - a0;
      double le = 0, lv = 0;
      if (n > 0) {
        const double e = (E - (double)a.Et[s]) / n;
        le = e * e;
        a.eps[s] = (float)(2.0 * a.le * e / ((double)a.S * n));
        for (int c = 0; c < 6; ++c) {
          const double wc = (red[1 + c][0] - (double)a.Wt[6 * s + c]) / n;
          lv += wc * wc;
          a.wbar[6 * s + c] = (float)(2.0 * a.lv * wc / (6.0 * a.S * n));
        }
      } else {
        a.eps[s] = 0.f;
        for (int c = 0; c < 6; ++c) a.wbar[6 * s + c] = 0.f;
      }
      a.lpart[3 * s] = le;
      a.lpart[3 * s + 1] = red[7][0];
      a.lpart[3 * s + 2] = lv;
    }
  }
  __syncthreads();   // red is read above before the next use of the LDS
}

__global__ __launch_bounds__(kRedBlk) void k_struct(StructArgs a) {
  __shared__ double red[8][kRedBlk];
  struct_body(a, blockIdx.x, red);
}

__global__ __launch_bounds__(kRedBlk) void k_loss_final(int S, int N, float le, float lf, float lv,
                                                        const double* __restrict__ lpart, float* __restrict__ loss,
                                                        int* __restrict__ flags) {
  __shared__ double red[3][kRedBlk];
  loss_final_block(S, N, le, lf, lv, lpart, loss, flags, red);
}

// ================================================================= adjoint
// Per atom, with the cotangents eps = dL/dE(n), Fbar = dL/dF and
// Gamma = dL/dW(n) frozen, the parameter gradient is the gradient of
//   Phi_i = eps E_i - E'_i . Gdot_i,  Gdot_i = sum_j dG_i/dr_ij t_ij,
//   t_ij = Fbar_j - Fbar_i + Gamma r_ij
// (the E, F and V terms of Eqs. 13-16 contracted with the residuals; the
// force and virial parts are the mixed second derivatives of C1.4-C3.20 and
// D1.11-D1.17 applied to t).
//   network: a = W0 Gdot, beta = w1 sigma (eps + 2 x a): dPhi/dW0 =
//            beta G^T - (w1 sigma) Gdot^T, dPhi/db0 = beta, dPhi/dw1 =
//            eps x - sigma a, dPhi/db1 = eps, Gbar = W0^T beta
//   radial:  dPhi/dc^R_{IJnk} = Gbar_n F[J][k] - E'_n Fp[J][k],
//            Fp[J][k] = sum_{j of type J} f'_k(r_ij) (r_hat . t)
//   angular: dPhi/dc^A_{IJnk} = sum_{j of type J} f_k X_n - f'_k (r_hat.t) Y_n,
//            X_n = sum_lm Sbar_nlm B_lm - A_nlm grad B_lm . t,
//            Y_n = sum_lm A_nlm B_lm,
//            Sbar = Gbar . dG/dS - E' . (d2G/dS2) Sdot  (the pairwise
//            coupling that Algorithm 1 enumerates).
// Outputs: per-atom vectors for the outer-product sums (W0, c^R) and, per
// wavefront, the sums of the c^A, b0, w1, b1 partials over its 8 atoms.
// Block vb (32 atoms of the species order); lds: lds_adjoint bytes.
template <class C, bool kTri>
__device__ __forceinline__ void adjoint_body(const AdjArgs& a, int vb, float* lds) {
  constexpr int T = C::T, NR = C::NR, NA = C::NA, KR = C::KR, KA = C::KA, Y = C::Y, D = C::D, LM = C::LMAX;
  constexpr int L3 = C::L3, L4 = C::L4, L5 = C::L5;
  using HS = HSplit<LM>;
  constexpr int YG = HS::YG;
  constexpr int DP = (D + 3) & ~3;
  constexpr int NAH = (NA + 1) / 2;          // channels per lane in the coefficient pass
  constexpr int YR = HRow<LM>::YR;
  constexpr int RW = DP + 2 * NA * YR;       // LDS row per atom: Gdot, Sbar, A (group order)
  constexpr int PSA = T * NA * KA;
  const int H = a.H;
  using CT = CTab<T, NA, KA>;
  float* ctab = lds;                     // [T][T][NA][KAP]
  float* wl = lds + CT::size;            // weights of the block's species
  float* rows = wl + weights_words(H, DP);   // [kAPB][RW]
  stage_ctab<T, NA, KA>(ctab, a.cA);
  __syncthreads();
  // as in the forward: issued after the barrier, waited for before the next
  stage_weights_async(wl, a.nn, a.nn_stride, block_species(a.order, a.type, vb), H, D, DP);
  const GroupCtx w = group_ctx(a.order, a.type, a.Npad, vb);
  const int N = a.N, i = w.i, I = w.I, pa = w.pa, s = w.s, g = w.g;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = (vb * 256 + (int)threadIdx.x) / kWave;
  const bool first_atom = (lane >> 3) == 0;   // atom slot 0 of the wavefront writes the sums
  float* part = a.part + (size_t)wave * a.PW;
  float* row = rows + w.al * RW;
  float* rowSb = row + DP;
  float* rowA = rowSb + NA * YR;
  const int st = a.astruct[i];
  const Cell cell = load_cell<kTri>(a.box, a.tilt, st);
  const float xi = a.pos[i], yi = a.pos[N + i], zi = a.pos[2 * N + i];
  const int cR_i = a.nb.cntR[i], cA_i = a.nb.cntA[i];
  const int nR = w.valid ? min(cR_i, a.nb.capR) : 0;
  const int nA = w.valid ? min(cA_i, a.nb.capA) : 0;
  const cptr<float> cRI = as_const(a.cR) + (size_t)I * T * NR * KR;
  const float eps_v = a.eps[st];
  const float eps = w.valid ? eps_v : 0.f;
  const float* wb = a.wbar + 6 * st;
  const float gxx = wb[0], gyy = wb[1], gzz = wb[2], gxy = wb[3], gyz = wb[4], gzx = wb[5];
  const float fbx = a.fbar[i], fby = a.fbar[N + i], fbz = a.fbar[2 * N + i];

  // ---- radial tangent pass, pairs split over the 8 lanes
  float FR[T][KR], FP[T][KR];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int k = 0; k < KR; ++k) FR[t][k] = FP[t][k] = 0.f;
  for (int k = s; k < nR; k += kLPA) {
    const PairGeom q = pair_geom<kTri>(a.nb.idxR[(size_t)i * a.nb.capR + k], a.pos, N, xi, yi, zi, cell);
    const float tx = (a.fbar[q.j] - fbx) + gxx * q.dx + gxy * q.dy;
    const float ty = (a.fbar[N + q.j] - fby) + gyy * q.dy + gyz * q.dz;
    const float tz = (a.fbar[2 * N + q.j] - fbz) + gzz * q.dz + gzx * q.dx;
    const float dt = (q.dx * tx + q.dy * ty + q.dz * tz) * q.inv_r;
    float f[KR], fp[KR];
    radial_basis_d<KR>(q.r, a.inv_rcR, f, fp);
    const int J = a.type[q.j];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const float m = (T == 1 || J == t) ? 1.f : 0.f;
      const float md = m * dt;
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        FR[t][kk] = fmaf(m, f[kk], FR[t][kk]);
        FP[t][kk] = fmaf(md, fp[kk], FP[t][kk]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      FR[t][k] = grp8_sum(FR[t][k]);
      FP[t][k] = grp8_sum(FP[t][k]);
      const int e = t * KR + k;
      if (w.valid && s == (e & 7)) {
        a.FRst[(size_t)e * a.Npad + pa] = FR[t][k];
        a.FPst[(size_t)e * a.Npad + pa] = FP[t][k];
      }
    }
  // every lane holds the sums: lane s takes channels n = s, s + 8, ... at once
#pragma unroll
  for (int n0 = 0; n0 < NR; n0 += kLPA) {
    const int n = n0 + s;
    if (n < NR) {
      const cptr<float> cn = cRI + n * KR;
      float acc = 0.f;
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int k = 0; k < KR; ++k) acc = fmaf(cn[t * NR * KR + k], FP[t][k], acc);
      row[n] = acc;
    }
  }

  // ---- angular tangent pass: Sdot_nlm = sum_j g'_n (r_hat.t) B_lm + g_n grad B_lm . t
  float Sd[NA][YG];
#pragma unroll
  for (int n = 0; n < NA; ++n)
#pragma unroll
    for (int e = 0; e < YG; ++e) Sd[n][e] = 0.f;
  for (int k = w.p; k < nA; k += 4) {
    const PairGeom q = pair_geom<kTri>(a.nb.idxA[(size_t)i * a.nb.capA + k], a.pos, N, xi, yi, zi, cell);
    const float ux = q.dx * q.inv_r, uy = q.dy * q.inv_r, uz = q.dz * q.inv_r;
    const float tx = (a.fbar[q.j] - fbx) + gxx * q.dx + gxy * q.dy;
    const float ty = (a.fbar[N + q.j] - fby) + gyy * q.dy + gyz * q.dz;
    const float tz = (a.fbar[2 * N + q.j] - fbz) + gzz * q.dz + gzx * q.dx;
    const float dt = ux * tx + uy * ty + uz * tz;
    float f[KA], fp[KA];
    radial_basis_d<KA>(q.r, a.inv_rcA, f, fp);
    const int J = a.type[q.j];
    const float* cJ = ctab + (I * T + J) * NA * CT::KAP;
    float gn[NA], gpd[NA];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int kk = 0; kk < KA; ++kk) {
        const float c = cJ[n * CT::KAP + kk];
        s0 = fmaf(c, f[kk], s0);
        s1 = fmaf(c, fp[kk], s1);
      }
      gn[n] = s0;
      gpd[n] = s1 * dt;
    }
    float B[Y], gbt[Y];
    harm_val<LM>(ux, uy, uz, B);
    // grad B . t = grad b(u) . (t - (u.t) u) / r
    harm_dir<LM>(ux, uy, uz, (tx - dt * ux) * q.inv_r, (ty - dt * uy) * q.inv_r, (tz - dt * uz) * q.inv_r, gbt);
#pragma unroll
    for (int e = 0; e < YG; ++e) {
      const float b = hsel<HS, Y>(g, e, B), c = hsel<HS, Y>(g, e, gbt);
#pragma unroll
      for (int n = 0; n < NA; ++n) Sd[n][e] = fmaf(gpd[n], b, fmaf(gn[n], c, Sd[n][e]));
    }
  }
#pragma unroll
  for (int n = 0; n < NA; ++n)
#pragma unroll
    for (int e = 0; e < YG; ++e) Sd[n][e] = quad_sum(Sd[n][e]);

  // ---- Gdot of the angular descriptors.  Sdot is parked in the atom's LDS
  //      row; channel n is then handled by the lanes of pair slot n mod 4
  //      (both harmonic groups), which also park S (stored by the forward
  //      pass) for the later phases
  {
    const int nAg = g ? HS::nA1 : HS::nA0;
    const int lA = g ? 2 : 1, lB = g ? 3 : 4;
#pragma unroll
    for (int n = 0; n < NA; ++n)
      if (w.p == (n & 3)) {
#pragma unroll
        for (int e = 0; e < YG; ++e) rowSb[n * YR + g * YG + e] = Sd[n][e];   // zero at padding entries
      }
    lds_lane_exchange();
    for (int n = w.p; n < NA; n += 4) {
      float Sn[YG], Sdn[YG];
#pragma unroll
      for (int e = 0; e < YG; ++e) {
        // unconditional loads, then the mask: a guarded load would become a
        // branch that waits for each value in turn
        const float v = a.Sst[(size_t)(n * YR + g * YG + e) * a.Npad + pa];
        Sn[e] = w.valid ? v : 0.f;
        Sdn[e] = rowSb[n * YR + g * YG + e];
      }
      float qa = 0.f, qb = 0.f;
#pragma unroll
      for (int e = 0; e < YG; ++e) {
        const float v = 2.0f * csel<HS>(g, e) * Sn[e] * Sdn[e];
        if (e < nAg) qa += v; else qb += v;
      }
      if (lA <= L3) row[NR + (lA - 1) * NA + n] = qa;
      if (lB <= L3) row[NR + (lB - 1) * NA + n] = qb;
      if constexpr (L4 != 0) {
        const Sym3 M = sym_of(Sn[0], Sn[1], Sn[2], Sn[3], Sn[4]);
        const Sym3 Md = sym_of(Sdn[0], Sdn[1], Sdn[2], Sdn[3], Sdn[4]);
        const float v = 3.0f * sym_dot(sym_mul(M, M), Md);
        if (g == 1) row[NR + L3 * NA + n] = v;
      }
      if constexpr (L5 != 0) {
        const float P = Sn[0] * Sn[0] + Sn[1] * Sn[1] + Sn[2] * Sn[2];
        const float SS = Sn[0] * Sdn[0] + Sn[1] * Sdn[1] + Sn[2] * Sdn[2];
        if (g == 0) row[NR + L3 * NA + (L4 ? NA : 0) + n] = 4.0f * P * SS;
      }
#pragma unroll
      for (int e = 0; e < YG; ++e) rowA[n * YR + g * YG + e] = Sn[e];
    }
  }
  if constexpr (C::YH > 0) {
    // Gdot of q_nl, l = 5..L3, from k_high_tangent
    for (int v = NR + 4 * NA + s; v < NR + L3 * NA; v += kLPA) {
      const float x = a.Gd[(size_t)v * a.Npad + pa];
      row[v] = w.valid ? x : 0.f;
    }
  }
  wait_weights();   // this wavefront's weight loads have landed; the barrier covers the others'
  __syncthreads();
  float Gd[D];
#pragma unroll
  for (int v = 0; v < D; ++v) {
    Gd[v] = row[v];
    if (w.valid && s == (v & 7)) a.Gd[(size_t)v * a.Npad + pa] = Gd[v];
  }

  // ---- network adjoint, hidden units mu = s, s+8, ...
  const float* Wl = wl;
  float Gb[D];
#pragma unroll
  for (int v = 0; v < D; ++v) Gb[v] = 0.f;
  const int RH = (H + kLPA - 1) / kLPA;
  for (int r = 0; r < RH; ++r) {
    const int mu = r * kLPA + s;
    const bool act = mu < H;
    const int mm = act ? mu : H - 1;
    const float* wr = Wl + mm * DP;
    float aa = 0.f;
#pragma unroll
    for (int v = 0; v < D; ++v) aa = fmaf(wr[v], Gd[v], aa);
    const bool live = act && w.valid;
    const float xv = a.X[(size_t)mm * a.Npad + pa];
    const float x = live ? xv : 0.f;
    const float sg = 1.0f - x * x;
    const float ws = Wl[H * DP + H + mm] * sg;
    const float be = live ? ws * (eps + 2.0f * x * aa) : 0.f;
#pragma unroll
    for (int v = 0; v < D; ++v) Gb[v] = fmaf(be, wr[v], Gb[v]);
    if (live) {
      a.beta[(size_t)mu * a.Npad + pa] = be;
      a.w1s[(size_t)mu * a.Npad + pa] = ws;
    }
    const float r0 = atoms8_sum(be);
    const float r1 = atoms8_sum(live ? eps * x - sg * aa : 0.f);
    if (act && first_atom) {
      part[PSA + mu] = r0;
      part[PSA + H + mu] = r1;
    }
  }
#pragma unroll
  for (int v = 0; v < D; ++v) Gb[v] = grp8_sum(Gb[v]);
  {
    const float r = atoms8_sum(s == 0 ? eps : 0.f);
    if (lane == 0) part[PSA + 2 * H] = r;
  }
#pragma unroll
  for (int n = 0; n < NR; ++n)
    if (w.valid && s == (n & 7)) a.Gbr[(size_t)n * a.Npad + pa] = Gb[n];
  if constexpr (C::YH > 0) {
    // Gbar of q_nl, l = 5..L3, for k_high_coef (the rows hold D entries)
#pragma unroll
    for (int v = NR + 4 * NA; v < NR + L3 * NA; ++v)
      if (w.valid && s == (v & 7)) a.Gbr[(size_t)v * a.Npad + pa] = Gb[v];
  }

  // ---- Sbar and A of this lane's harmonic group, in place in the atom's LDS
  //      row, channel n by the lanes of pair slot n mod 4; Gbar goes to the
  //      row's first D floats (Gdot there has been read)
#pragma unroll
  for (int v = 0; v < D; ++v)
    if (s == (v & 7)) row[v] = Gb[v];
  lds_lane_exchange();
  {
    const int nAg = g ? HS::nA1 : HS::nA0;
    const int lA = g ? 2 : 1, lB = g ? 3 : 4;
    const int lAc = lA <= L3 ? lA : 1, lBc = lB <= L3 ? lB : 1;
    const size_t Np = a.Npad;
    for (int n = w.p; n < NA; n += 4) {
      float Sn[YG], Sdn[YG];
#pragma unroll
      for (int e = 0; e < YG; ++e) {
        Sn[e] = rowA[n * YR + g * YG + e];
        Sdn[e] = rowSb[n * YR + g * YG + e];
      }
      // E' and Gbar of the descriptors built from these sums
      const float vA = a.Ep[(size_t)(NR + (lAc - 1) * NA + n) * Np + pa];
      const float vB = a.Ep[(size_t)(NR + (lBc - 1) * NA + n) * Np + pa];
      const float bA = row[NR + (lAc - 1) * NA + n], bB = row[NR + (lBc - 1) * NA + n];
      const float eA = (w.valid && lA <= L3) ? vA : 0.f;
      const float eB = (w.valid && lB <= L3) ? vB : 0.f;
      const float gA = lA <= L3 ? bA : 0.f, gB = lB <= L3 ? bB : 0.f;
      float o[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, od[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
      float e4 = 0.f, g4 = 0.f, e5 = 0.f, g5 = 0.f, P = 0.f, SS = 0.f;
      if constexpr (L4 != 0) {
        const Sym3 M = sym_of(Sn[0], Sn[1], Sn[2], Sn[3], Sn[4]);
        const Sym3 Md = sym_of(Sdn[0], Sdn[1], Sdn[2], Sdn[3], Sdn[4]);
        sym_proj(sym_mul(M, M), o);
        sym_proj(sym_mul(Md, M), od);
        const int v4 = NR + L3 * NA + n;
        const float v = a.Ep[(size_t)v4 * Np + pa], b = row[v4];
        e4 = (w.valid && g == 1) ? v : 0.f;
        g4 = g == 1 ? b : 0.f;
      }
      if constexpr (L5 != 0) {
        P = Sn[0] * Sn[0] + Sn[1] * Sn[1] + Sn[2] * Sn[2];
        SS = Sn[0] * Sdn[0] + Sn[1] * Sdn[1] + Sn[2] * Sdn[2];
        const int v5 = NR + L3 * NA + (L4 ? NA : 0) + n;
        const float v = a.Ep[(size_t)v5 * Np + pa], b = row[v5];
        e5 = (w.valid && g == 0) ? v : 0.f;
        g5 = g == 0 ? b : 0.f;
      }
#pragma unroll
      for (int e = 0; e < YG; ++e) {
        const bool real = g ? HRow<LM>::real(1, e) : HRow<LM>::real(0, e);
        const float c2 = 2.0f * csel<HS>(g, e);
        const float eL = e < nAg ? eA : eB, gL = e < nAg ? gA : gB;
        float Av = c2 * eL * Sn[e];
        float Sb = c2 * (gL * Sn[e] - eL * Sdn[e]);
        if (e < 5) {
          Av += 3.0f * e4 * o[e];
          Sb += 3.0f * g4 * o[e] - 6.0f * e4 * od[e];
        }
        if (e < 3) {
          Av += 4.0f * e5 * P * Sn[e];
          Sb += 4.0f * g5 * P * Sn[e] - e5 * (8.0f * SS * Sn[e] + 4.0f * P * Sdn[e]);
        }
        rowA[n * YR + g * YG + e] = real ? Av : 0.f;
        rowSb[n * YR + g * YG + e] = real ? Sb : 0.f;
      }
    }
  }
  __syncthreads();

  // ---- angular coefficient gradient: channels g*NAH + j, pairs p, p+4, ...
  float cb[T][NAH][KA];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int j = 0; j < NAH; ++j)
#pragma unroll
      for (int k = 0; k < KA; ++k) cb[t][j][k] = 0.f;
  for (int k = w.p; k < nA; k += 4) {
    // reload Sbar and A from LDS every pair: hoisted out of the loop they
    // would take 2 NAH Y registers and halve the occupancy
    asm volatile("" ::: "memory");
    const PairGeom q = pair_geom<kTri>(a.nb.idxA[(size_t)i * a.nb.capA + k], a.pos, N, xi, yi, zi, cell);
    const float ux = q.dx * q.inv_r, uy = q.dy * q.inv_r, uz = q.dz * q.inv_r;
    const float tx = (a.fbar[q.j] - fbx) + gxx * q.dx + gxy * q.dy;
    const float ty = (a.fbar[N + q.j] - fby) + gyy * q.dy + gyz * q.dz;
    const float tz = (a.fbar[2 * N + q.j] - fbz) + gzz * q.dz + gzx * q.dx;
    const float dt = ux * tx + uy * ty + uz * tz;
    float f[KA], fp[KA];
    radial_basis_d<KA>(q.r, a.inv_rcA, f, fp);
    const int J = a.type[q.j];
    float B[Y], gbt[Y];
    harm_val<LM>(ux, uy, uz, B);
    // grad B . t = grad b(u) . (t - (u.t) u) / r
    harm_dir<LM>(ux, uy, uz, (tx - dt * ux) * q.inv_r, (ty - dt * uy) * q.inv_r, (tz - dt * uz) * q.inv_r, gbt);
#pragma unroll
    for (int j = 0; j < NAH; ++j) {
      const int n = g * NAH + j;
      const bool on = n < NA;
      const float* sb = rowSb + (on ? n : 0) * YR;
      const float* av = rowA + (on ? n : 0) * YR;
      float X = 0.f, Yv = 0.f;
#pragma unroll
      for (int gg = 0; gg < 2; ++gg)
#pragma unroll
        for (int e = 0; e < YG; ++e) {
          const int qq = HS::q(gg, e);
          if (qq >= 0) {
            X = fmaf(sb[gg * YG + e], B[qq], fmaf(-av[gg * YG + e], gbt[qq], X));
            Yv = fmaf(av[gg * YG + e], B[qq], Yv);
          }
        }
      X = on ? X : 0.f;
      const float Yd = on ? Yv * dt : 0.f;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const float m = (T == 1 || J == t) ? 1.f : 0.f;
        const float mX = m * X, mY = m * Yd;
#pragma unroll
        for (int kk = 0; kk < KA; ++kk) cb[t][j][kk] = fmaf(mX, f[kk], fmaf(-mY, fp[kk], cb[t][j][kk]));
      }
    }
  }
  // sums over the pair slots and atoms, scattered over the lanes of each
  // harmonic group: value v = (t NAH + j) KA + k
  {
    constexpr int V = T * NAH * KA;
    float cv[V];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int j = 0; j < NAH; ++j)
#pragma unroll
        for (int k = 0; k < KA; ++k) cv[(t * NAH + j) * KA + k] = cb[t][j][k];
    float out[(V + 31) / 32];
    rs_slots_atoms(cv, out);
    const int c = rs_slots_atoms_code();
#pragma unroll
    for (int r = 0; r < (V + 31) / 32; ++r) {
      const int v = 32 * r + c;
      const int t = v / (NAH * KA), j = (v / KA) % NAH, k = v % KA;
      const int n = g * NAH + j;
      if (v < V && n < NA) part[(t * NA + n) * KA + k] = out[r];
    }
  }
}

template <class C, bool kTri, int W>
__global__ __launch_bounds__(256, W) void k_adjoint(AdjArgs a) {
  extern __shared__ __align__(16) float lds[];
  adjoint_body<C, kTri>(a, blockIdx.x, lds);
}

// Sums over the atoms of each species of an outer product,
//   out[I][b][m][v] = sum_p A1[m][p] B1[v][p] - A2[m][p] B2[v][p],
// over block b's share of species I's atoms (species order).  Used for
// dL/dW0 = sum beta G^T - (w1 sigma) Gdot^T and for
// dL/dc^R = sum Gbar_n F[J][k] - E'_n Fp[J][k].
// This is a product contracted over atoms, so it runs on the fp32 matrix
// cores: v_mfma_f32_16x16x4f32 takes a 16 x 4 slice of A (lane l: row l % 16,
// atom slot l / 16) and a 4 x 16 slice of B, and accumulates a 16 x 16 tile
// of which lane l holds rows 4 (l / 16) + r, column l % 16.  Each lane loads
// float4 runs of 4 consecutive atoms and feeds component j to the j-th of 4
// MFMAs, so atom slot l / 16 of MFMA j is atom 4 (l / 16) + j of the 16-atom
// group.  A block covers a 4 x 3 grid of 16 x 16 output tiles (blockIdx.z
// picks the grid cell for larger products); its 4 wavefronts take
// consecutive 16-atom groups and are summed through LDS at the end.
// blocks per species: the W0 sums stream about three times the data of the
// c^R sums, so they get more blocks (all blocks are resident at once)
constexpr int kOSBlocksW = 192, kOSBlocksC = 64;            // defaults
constexpr int kOSBlocksMaxW = 512, kOSBlocksMaxC = 256;
constexpr int kOSTM = 4, kOSTV = 3;

struct OuterArgs {
  int Npad, M, V, NB;
  const int* seg;
  const float* A1;
  const float* B1;
  const float* A2;
  const float* B2;
  float* out;
};

typedef float f32x4 __attribute__((ext_vector_type(4)));

// atoms p .. p + 3 of a row (p a multiple of 4 inside the padded row), zero
// past p1 or when off; the load itself is unconditional so that a group's
// loads issue back to back
__device__ __forceinline__ f32x4 ld_atoms4(const float* row, int p, int p1, bool on) {
  const float4 v = *reinterpret_cast<const float4*>(row + p);
  f32x4 r;
  r[0] = (on && p < p1) ? v.x : 0.f;
  r[1] = (on && p + 1 < p1) ? v.y : 0.f;
  r[2] = (on && p + 2 < p1) ? v.z : 0.f;
  r[3] = (on && p + 3 < p1) ? v.w : 0.f;
  return r;
}

constexpr int kOuterLds = 3 * kOSTM * kOSTV * kWave * sizeof(f32x4);
__device__ __forceinline__ void outer_sum_block(const OuterArgs& o, int b, int I, int z,
                                                f32x4 (&red)[3][kOSTM * kOSTV][kWave]) {
  if (b >= o.NB) return;
  const int nzv = (o.V + 16 * kOSTV - 1) / (16 * kOSTV);
  const int mz = z / nzv, vz = z % nzv;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int start = o.seg[2 * I], count = o.seg[2 * I + 1];
  const int per = ((count + o.NB - 1) / o.NB + 15) & ~15;   // multiple of 16 atoms
  const int p0 = start + b * per;
  const int p1 = min(start + count, p0 + per);
  const int row = lane & 15, slot = lane >> 4;
  const float* a1[kOSTM];
  const float* a2[kOSTM];
  const float* b1[kOSTV];
  const float* b2[kOSTV];
  bool am[kOSTM], bm[kOSTV];
#pragma unroll
  for (int t = 0; t < kOSTM; ++t) {
    const int m = (mz * kOSTM + t) * 16 + row;
    am[t] = m < o.M;
    a1[t] = o.A1 + (size_t)(am[t] ? m : 0) * o.Npad;
    a2[t] = o.A2 + (size_t)(am[t] ? m : 0) * o.Npad;
  }
#pragma unroll
  for (int t = 0; t < kOSTV; ++t) {
    const int v = (vz * kOSTV + t) * 16 + row;
    bm[t] = v < o.V;
    b1[t] = o.B1 + (size_t)(bm[t] ? v : 0) * o.Npad;
    b2[t] = o.B2 + (size_t)(bm[t] ? v : 0) * o.Npad;
  }
  // tiles with no row or no column inside the product are skipped (uniform)
  const int tm_live = min(kOSTM, (o.M - mz * kOSTM * 16 + 15) / 16);
  const int tv_live = min(kOSTV, (o.V - vz * kOSTV * 16 + 15) / 16);
  f32x4 acc[kOSTM][kOSTV];
#pragma unroll
  for (int x = 0; x < kOSTM; ++x)
#pragma unroll
    for (int y = 0; y < kOSTV; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
  // operands of one 16-atom group; the next group's loads are issued before
  // the current group's MFMAs
  f32x4 va1[kOSTM], va2[kOSTM], vb1[kOSTV], vb2[kOSTV];
  auto load = [&](int g) {
    // past the block's atoms the loads read the segment start instead (always
    // inside the padded rows) and are masked to zero
    const bool in = g < p1;
    const int p = (in ? g : start) + 4 * slot;
#pragma unroll
    for (int t = 0; t < kOSTM; ++t) {
      va1[t] = ld_atoms4(a1[t], p, p1, in && am[t]);
      va2[t] = -ld_atoms4(a2[t], p, p1, in && am[t]);
    }
#pragma unroll
    for (int t = 0; t < kOSTV; ++t) {
      vb1[t] = ld_atoms4(b1[t], p, p1, in && bm[t]);
      vb2[t] = ld_atoms4(b2[t], p, p1, in && bm[t]);
    }
  };
  load(p0 + 16 * wv);
  for (int g = p0 + 16 * wv; g < p1; g += 64) {
    f32x4 ca1[kOSTM], ca2[kOSTM], cb1[kOSTV], cb2[kOSTV];
#pragma unroll
    for (int t = 0; t < kOSTM; ++t) {
      ca1[t] = va1[t];
      ca2[t] = va2[t];
    }
#pragma unroll
    for (int t = 0; t < kOSTV; ++t) {
      cb1[t] = vb1[t];
      cb2[t] = vb2[t];
    }
    load(g + 64);
#pragma unroll
    for (int x = 0; x < kOSTM; ++x) {
      if (x >= tm_live) break;
#pragma unroll
      for (int y = 0; y < kOSTV; ++y) {
        if (y >= tv_live) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca1[x][j], cb1[y][j], acc[x][y], 0, 0, 0);
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(ca2[x][j], cb2[y][j], acc[x][y], 0, 0, 0);
        }
      }
    }
  }
  if (wv > 0) {
#pragma unroll
    for (int x = 0; x < kOSTM; ++x)
#pragma unroll
      for (int y = 0; y < kOSTV; ++y) red[wv - 1][x * kOSTV + y][lane] = acc[x][y];
  }
  __syncthreads();
  if (wv != 0) {
    __syncthreads();
    return;
  }
  float* out = o.out + ((size_t)I * o.NB + b) * o.M * o.V;
#pragma unroll
  for (int x = 0; x < kOSTM; ++x)
#pragma unroll
    for (int y = 0; y < kOSTV; ++y) {
      f32x4 s4 = acc[x][y];
#pragma unroll
      for (int w = 0; w < 3; ++w) s4 += red[w][x * kOSTV + y][lane];
      const int v = (vz * kOSTV + y) * 16 + row;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = (mz * kOSTM + x) * 16 + 4 * slot + r;
        if (m < o.M && v < o.V) out[m * o.V + v] = s4[r];
      }
    }
  __syncthreads();   // the other wavefronts wait here: red is read above
}

int outer_slices(int M, int V) {
  const int nzm = (M + 16 * kOSTM - 1) / (16 * kOSTM), nzv = (V + 16 * kOSTV - 1) / (16 * kOSTV);
  return nzm * nzv;
}

// First stage of the final reduction for the wavefront partials (c^A, b0,
// w1, b1): block (b, I) sums, in float64 and in wave order, chunk b of the
// wavefronts of species I; one thread per slot, so reads run along rows.
constexpr int kPRChunks = 128;   // default chunks per species
constexpr int kPRChunksMax = 512;

// Loss reduction carried by k_outer_reduce (one extra block) so that a
// loss-and-gradient pass spends no launch on it.
struct LossArgs {
  int on, S, N;
  float le, lf, lv;
  const double* lpart;
  float* loss;
  int* flags;
};

// chunk b of species I's wavefront partials
__device__ __forceinline__ void part_reduce_body(int PW, const int* seg, const float* part, double* pp, int b, int I,
                                                 int nch) {
  const int start = seg[2 * I], count = seg[2 * I + 1];
  const int w0 = start / kAPW, w1 = count > 0 ? (start + count + kAPW - 1) / kAPW : w0;
  const int per = (w1 - w0 + nch - 1) / nch;
  const int r0 = w0 + b * per, r1 = min(w1, r0 + per);
  for (int slot = threadIdx.x; slot < PW; slot += blockDim.x) {
    double sum = 0.0;
    int r = r0;
    for (; r + 4 <= r1; r += 4) {
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = part[(size_t)(r + u) * PW + slot];
#pragma unroll
      for (int u = 0; u < 4; ++u) sum += (double)v[u];
    }
    for (; r < r1; ++r) sum += (double)part[(size_t)r * PW + slot];
    pp[((size_t)I * nch + b) * PW + slot] = sum;
  }
}

// The outer-product sums, the first stage of the wavefront partial sums and
// the loss sum in one launch (all three read only the adjoint's outputs):
// blocks [0, n_outer) take the outer products (block x of species I, output
// slice z; slices [0, nzw) of dW0, the rest of dc^R), the next prc T blocks
// the partial sums, the last one the loss.
struct OuterReduceArgs {
  OuterArgs ow, oc;
  int nzw, nzc, os_x, T, PW, prc;
  const int* seg;
  const float* part;
  double* pp;
  LossArgs la;
};

__global__ __launch_bounds__(256) void k_outer_reduce(OuterReduceArgs a) {
  __shared__ f32x4 red[3][kOSTM * kOSTV][kWave];
  const int T = a.T, n_outer = a.os_x * T * (a.nzw + a.nzc), n_pr = a.prc * T;
  const int v = blockIdx.x;
  if (v < n_outer) {
    const int x = v % a.os_x, I = (v / a.os_x) % T, z = v / (a.os_x * T);
    if (z < a.nzw)
      outer_sum_block(a.ow, x, I, z, red);
    else
      outer_sum_block(a.oc, x, I, z - a.nzw, red);
  } else if (v < n_outer + n_pr) {
    const int u = v - n_outer;
    part_reduce_body(a.PW, a.seg, a.part, a.pp, u % a.prc, u / a.prc, a.prc);
  } else if (a.la.on) {
    loss_final_block(a.la.S, a.la.N, a.la.le, a.la.lf, a.la.lv, a.la.lpart, a.la.loss, a.la.flags, red);
  }
}


// Final gradient: 16 lanes per parameter; lane l sums rows l, l + 16, ... of
// that parameter's partials in float64, then a fixed xor tree adds the 16
// lane sums.  Parameter layout: c^R [T][T][NR][KR], c^A [T][T][NA][KA], then
// per species W0 [H][D], b0 [H], w1 [H], b1.
// ==================================================================== Adam
__device__ __forceinline__ void adam_one(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                                         float g, float lr, float b1, float b2, float eps, float c1, float c2,
                                         int64_t q) {
  const float mm = b1 * m[q] + (1.0f - b1) * g;
  const float vv = b2 * v[q] + (1.0f - b2) * g * g;
  m[q] = mm;
  v[q] = vv;
  th[q] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ __launch_bounds__(256) void k_adam(int64_t P, float* __restrict__ th, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ g, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < P) adam_one(th, m, v, g[q], lr, b1, b2, eps, c1, c2, q);
}

struct AdamDev {
  float lr_start, lr_stop;
  int64_t n_warmup, n_total;
  float b1, b2, eps;
};

__device__ float lr_at(const AdamDev& c, int64_t s) {
  if (c.n_total <= 0) return c.lr_start;
  if (s < c.n_warmup) return c.lr_stop + (float)((double)s / (double)c.n_warmup) * (c.lr_start - c.lr_stop);
  double fr = (double)(s - c.n_warmup) / (double)max((int64_t)1, c.n_total - c.n_warmup);
  fr = fr > 1.0 ? 1.0 : fr;
  return c.lr_stop + (c.lr_start - c.lr_stop) * 0.5f * (1.0f + (float)cos(3.14159265358979323846 * fr));
}

struct GradArgs {
  int T, NR, NA, KR, KA, H, D, PW, NBw, NBc, PRC;
  int64_t P;
  const double* pp;      // [T][PRC][PW]
  const float* w0part;   // [T][NBw][H*D]
  const float* crpart;   // [T][NBc][NR*T*KR]
  float* grad;
  // Adam on each parameter as soon as its gradient is summed (the captured
  // training step); step is the 1-based device step counter
  int adam;
  AdamDev ad;
  float* th;
  float* mm;
  float* vv;
  const int* step;
  int* flags;   // the replay's flag word: any raised flag skips the update
};

// Whether a captured step may update parameter q: no flag was raised by this
// replay's neighbor build or loss (their launches precede this one), the
// latched step is valid, and the gradient entry is finite (else the flag is
// raised and this entry alone keeps its value).
__device__ __forceinline__ bool adam_allowed(int* flags, int fl0, int st, float g) {
  if (!isfinite(g)) {
    atomicOr(flags, FL_NONFINITE);
    return false;
  }
  return fl0 == 0 && st >= 1;
}

// block vb: parameters 16 vb .. 16 vb + 15
__device__ __forceinline__ void grad_final_body(const GradArgs& a, int vb) {
  const int64_t q = ((int64_t)vb * 256 + threadIdx.x) >> 4;
  const int l = threadIdx.x & 15;
  const int P_R = a.T * a.T * a.NR * a.KR, P_A = a.T * a.T * a.NA * a.KA;
  const int blk = a.H * a.D + 2 * a.H + 1;
  const int PSA = a.T * a.NA * a.KA;
  const int HD = a.H * a.D, CR = a.NR * a.T * a.KR;
  double sum = 0.0;
  if (q < a.P) {
    const int qi = (int)q;
    const float* fsrc = nullptr;
    const double* dsrc = nullptr;
    int stride = 0, rows = 0;
    if (qi < P_R) {
      const int I = qi / (a.T * a.NR * a.KR), rem = qi % (a.T * a.NR * a.KR);
      const int t = rem / (a.NR * a.KR), n = (rem / a.KR) % a.NR, k = rem % a.KR;
      fsrc = a.crpart + (size_t)I * a.NBc * CR + n * (a.T * a.KR) + t * a.KR + k;
      stride = CR;
      rows = a.NBc;
    } else if (qi < P_R + P_A) {
      const int I = (qi - P_R) / PSA, slot = (qi - P_R) % PSA;
      dsrc = a.pp + (size_t)I * a.PRC * a.PW + slot;
      stride = a.PW;
      rows = a.PRC;
    } else {
      const int I = (qi - P_R - P_A) / blk, o = (qi - P_R - P_A) % blk;
      if (o < HD) {
        fsrc = a.w0part + (size_t)I * a.NBw * HD + o;
        stride = HD;
        rows = a.NBw;
      } else {
        dsrc = a.pp + (size_t)I * a.PRC * a.PW + PSA + (o - HD);
        stride = a.PW;
        rows = a.PRC;
      }
    }
    if (fsrc) {
      for (int r = l; r < rows; r += 16) sum += (double)fsrc[(size_t)r * stride];
    } else {
      for (int r = l; r < rows; r += 16) sum += dsrc[(size_t)r * stride];
    }
  }
#pragma unroll
  for (int d = 8; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 16);
  if (q < a.P && l == 0) {
    const float gq = (float)sum;
    a.grad[q] = gq;
    if (a.adam) {
      const int st = *a.step;
      if (adam_allowed(a.flags, __hip_atomic_load(a.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), st, gq)) {
        const float lr = lr_at(a.ad, (int64_t)(st - 1));
        const float c1 = 1.0f - powf(a.ad.b1, (float)st), c2 = 1.0f - powf(a.ad.b2, (float)st);
        adam_one(a.th, a.mm, a.vv, gq, lr, a.ad.b1, a.ad.b2, a.ad.eps, c1, c2, q);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_grad_final(GradArgs a) { grad_final_body(a, blockIdx.x); }

// Adam with the step counter read from device memory (graph replays).
__global__ __launch_bounds__(256) void k_adam_dev(int64_t P, float* __restrict__ th, float* __restrict__ m,
                                                  float* __restrict__ v, const float* __restrict__ g,
                                                  const int* __restrict__ step, int* flags, AdamDev c) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P) return;
  const int st = *step;
  if (!adam_allowed(flags, __hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), st, g[q])) return;
  const float lr = lr_at(c, (int64_t)(st - 1));
  const float c1 = 1.0f - powf(c.b1, (float)st), c2 = 1.0f - powf(c.b2, (float)st);
  adam_one(th, m, v, g[q], lr, c.b1, c.b2, c.eps, c1, c2, q);
}

// First node of a captured train step: clear the flags, latch the step this
// replay uses (Adam reads the latched copy) and advance the caller's counter.
// A step counter below 1 (Adam's bias correction needs step >= 1) raises
// FL_STEP, which makes this replay skip its update.
__device__ __forceinline__ void graph_head(int* flags, int* step, int* cur) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int st = step[0];
    flags[0] = st < 1 ? FL_STEP : 0;
    cur[0] = st;
    step[0] = st + 1;
  }
}
__global__ void k_graph_head(int* flags, int* step, int* cur) { graph_head(flags, step, cur); }


__global__ void k_fill_i32(int* p, int n, int v) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) p[q] = v;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) p[q] = v;
}

// ============================================================ persistent step
// The whole step after the neighbor build in one launch: the species order,
// forward, force gather, per-structure sums and loss, adjoint, gradient
// reductions and Adam, as phases of one persistent grid separated by a
// software grid barrier.  The grid holds as many blocks as are resident at
// once, each phase deals its work items (the blocks of the separate kernels)
// to them, and every phase's intermediate stays in the same workspace arrays
// as in the separate kernels.

// Grid barrier, two levels.  The blocks of XCD x (blockIdx.x mod 8) count
// their arrivals in a counter of their own (bar[kBarStride (x + 1)], one per
// 64-byte line); the block that completes its XCD's count for barrier k adds
// one to the device counter bar[0], and every block waits until that reaches
// 8 k.  Same-address atomics from hundreds of blocks serialise at the memory
// side, so one level costs tens of microseconds where two cost a few.  The
// counters are zeroed by the step's head.  A wait longer than kBarrierTicks
// of the 100 MHz constant clock, or a flag raised by a block that timed out,
// makes the block leave with FL_BARRIER raised, so a grid whose blocks are
// not all resident ends with an error, not a hang.
// The wait polls with relaxed loads: an acquire load at device scope also
// invalidates the L2 of the polling XCD, and dozens of waiting blocks would
// keep invalidating the cache under the blocks still working.  A release
// fence before the arrival and an acquire fence after the wait order the
// phases' memory.
constexpr uint64_t kBarrierTicks = 200000000ull;   // 2 s
constexpr int kBarStride = 16;                     // words between counters
constexpr int kBarWords = kBarStride * (kXCD + 1);
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned k, int* flags, int* abort_sh) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned per = gridDim.x / kXCD;   // blocks per XCD (gridDim.x is a multiple of 8)
    const int x = blockIdx.x % kXCD;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned old = __hip_atomic_fetch_add(bar + kBarStride * (x + 1), 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (old == k * per - 1u) __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = k * (unsigned)kXCD;
    const uint64_t t0 = wall_clock64();
    int ok = 1;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if ((__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & FL_BARRIER) ||
          wall_clock64() - t0 > kBarrierTicks) {
        atomicOr(flags, FL_BARRIER);
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *abort_sh = !ok;
  }
  __syncthreads();
  return *abort_sh == 0;
}

// A phase's arguments, read again for each work item behind a compiler
// barrier, into scalar registers.  Values derived from arguments that stay
// the same across a phase's loop would otherwise be computed once before the
// loop and kept live through the whole body (the per-atom bodies are sized
// for the registers of one block's work); here nothing in the body is
// invariant, so the loop body compiles as the separate kernel does.
template <class T>
__device__ __forceinline__ T item_args(const T& p) {
  static_assert(sizeof(T) % 4 == 0, "read as words");
  asm volatile("" ::: "memory");
  T v;
  const int* q = reinterpret_cast<const int*>(&p);
  int* d = reinterpret_cast<int*>(&v);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) d[k] = __builtin_amdgcn_readfirstlane(q[k]);
  return v;
}

// Work items [0, n) of a phase dealt to the persistent blocks: the blocks of
// XCD x (blockIdx.x mod 8; gridDim.x is a multiple of 8) take the x-th
// contiguous eighth, so items that share data share an L2.
template <class F>
__device__ __forceinline__ void for_items(int n, F&& f) {
  const int per = gridDim.x / kXCD;
  const int x = blockIdx.x % kXCD, r = blockIdx.x / kXCD;
  const int q = n / kXCD, rem = n % kXCD;
  const int lo = x * q + min(x, rem), cnt = q + (x < rem ? 1 : 0);
  for (int j = r; j < cnt; j += per) f(lo + j);
}

struct StepArgs {
  OrderArgs ord;
  FwdArgs fwd;
  PairLists nb;
  float* F;
  StructArgs st;
  AdjArgs adj;
  OuterArgs ow, oc;
  int nzw, nzc, os_x;
  int PW;
  const int* seg;
  double* pp;
  LossArgs la;
  GradArgs g;
  int n_gf;        // blocks of the final gradient reduction
  unsigned* bar;
  int* flags;
};

// The arguments are read from device memory (written by k_step_head), not
// from the kernel-argument segment: loads of kernel arguments are all issued
// at entry and would stay live in registers through every phase.  Two
// wavefronts per SIMD: at three (168 registers) the merged phases spill
// several hundred bytes per lane, although each body alone fits.
template <class C>
__global__ __launch_bounds__(256, 2) void k_step(const StepArgs* pa) {
  const StepArgs& a = *pa;
  extern __shared__ __align__(16) float lds[];
  __shared__ int abort_sh;
  unsigned k = 0;
#define NEP_BARRIER() \
  if (!grid_barrier(a.bar, ++k, a.flags, &abort_sh)) return
  // species order: key counts (and every slot cleared), offsets, ranks
  for (int q = blockIdx.x * 256 + threadIdx.x; q < a.ord.Npad; q += (int)gridDim.x * 256) a.ord.order[q] = -1;
  {
    const int nblk = a.ord.nblk;
    for_items(nblk, [&](int ob) { order_count_body<256>(item_args(a.ord), ob, reinterpret_cast<int*>(lds)); });
  }
  NEP_BARRIER();
  if (blockIdx.x == 0) order_scan_body<256>(item_args(a.ord), reinterpret_cast<int*>(lds));
  NEP_BARRIER();
  {
    const int nblk = a.ord.nblk;
    for_items(nblk, [&](int ob) { order_scatter_body<256>(item_args(a.ord), ob, reinterpret_cast<int*>(lds)); });
  }
  NEP_BARRIER();
  // forward: descriptors, network, partial forces
  for_items(a.fwd.Npad / kAPB, [&](int vb) {
    forward_body<C, false>(item_args(a.fwd), vb, lds);
    __syncthreads();
  });
  NEP_BARRIER();
  for_items((a.fwd.N + 256 / kGatherLPA - 1) / (256 / kGatherLPA), [&](int vb) {
    const PairLists nb = item_args(a.nb);
    const FwdArgs f = item_args(a.fwd);
    gather_body<kGatherLPA>(vb, f.N, nb, f.fR, f.fA, a.F, nullptr);
  });
  NEP_BARRIER();
  // per-structure sums, loss partials and cotangents
  if (a.st.split) {
    for_items((a.st.N + kStructChunk - 1) / kStructChunk,
              [&](int vb) { struct_part_body(item_args(a.st), vb, lds); });
    NEP_BARRIER();
  }
  for_items(a.st.S, [&](int s) { struct_body(item_args(a.st), s, lds); });
  NEP_BARRIER();
  for_items(a.adj.Npad / kAPB, [&](int vb) {
    adjoint_body<C, false>(item_args(a.adj), vb, lds);
    __syncthreads();
  });
  NEP_BARRIER();
  // outer-product sums, first stage of the partial sums, and the loss
  {
    const int T = a.ord.T;
    const int os_x = a.os_x, nzw = a.nzw;
    const int prc = a.g.PRC;
    const int n_outer = os_x * T * (nzw + a.nzc), n_pr = prc * T;
    auto& red = *reinterpret_cast<f32x4(*)[3][kOSTM * kOSTV][kWave]>(lds);
    for_items(n_outer + n_pr + (a.la.on ? 1 : 0), [&](int v) {
      if (v < n_outer) {
        const int x = v % os_x, I = (v / os_x) % T, z = v / (os_x * T);
        if (z < nzw)
          outer_sum_block(item_args(a.ow), x, I, z, red);
        else
          outer_sum_block(item_args(a.oc), x, I, z - nzw, red);
      } else if (v < n_outer + n_pr) {
        const int u = v - n_outer;
        part_reduce_body(a.PW, a.seg, a.adj.part, a.pp, u % prc, u / prc, prc);
      } else {
        const LossArgs la = item_args(a.la);
        loss_final_block(la.S, la.N, la.le, la.lf, la.lv, la.lpart, la.loss, la.flags, lds);
        __syncthreads();
      }
    });
  }
  NEP_BARRIER();
  // final gradient reduction with Adam
  for_items(a.n_gf, [&](int vb) { grad_final_body(item_args(a.g), vb); });
#undef NEP_BARRIER
}

// Head of the persistent step: the graph head, the step's arguments copied
// to device memory, and the barrier's arrival counter cleared.
__global__ void k_step_head(StepArgs a, StepArgs* dst, int* flags, int* step, int* cur) {
  static_assert(sizeof(StepArgs) % 4 == 0, "copied as words");
  const int* src = reinterpret_cast<const int*>(&a);
  int* d = reinterpret_cast<int*>(dst);
  for (int q = threadIdx.x; q < (int)(sizeof(StepArgs) / 4); q += blockDim.x) d[q] = src[q];
  for (int q = threadIdx.x; q < kBarWords; q += blockDim.x) a.bar[q] = 0u;
  graph_head(flags, step, cur);
}

// ============================================================ padded models
// A model smaller than a compiled size class runs in that class with its
// parameters zero-padded: radial and angular channels, Chebyshev terms and
// species the model does not have get zero coefficients, and the network's
// columns of descriptors it does not have (higher channels, degrees up to the
// class's, the 4- and 5-body terms) get zero weights.  Every padded quantity
// then adds an exact zero to the energies, forces and virials, and the
// gradient entries of the model's own parameters are those of the class run.
// PadDims maps a parameter of the model to its slot in the class layout.
struct PadDims {
  int T, NR, NA, KR, KA, D, H, l3, l4, l5;   // the model
  int Tc, NRc, NAc, KRc, KAc, Dc, L3c;       // the class (4- and 5-body terms on)
  int64_t P;                                 // parameters of the model
};

// class column of descriptor v of the model
__device__ __forceinline__ int pad_col(const PadDims& d, int v) {
  if (v < d.NR) return v;
  v -= d.NR;
  if (v < d.l3 * d.NA) return d.NRc + (v / d.NA) * d.NAc + v % d.NA;
  v -= d.l3 * d.NA;
  if (d.l4) {
    if (v < d.NA) return d.NRc + d.L3c * d.NAc + v;
    v -= d.NA;
  }
  return d.NRc + d.L3c * d.NAc + d.NAc + v;   // 5-body
}

__device__ __forceinline__ int64_t pad_index(const PadDims& d, int64_t q) {
  const int64_t PR = (int64_t)d.T * d.T * d.NR * d.KR, PA = (int64_t)d.T * d.T * d.NA * d.KA;
  const int64_t PRc = (int64_t)d.Tc * d.Tc * d.NRc * d.KRc, PAc = (int64_t)d.Tc * d.Tc * d.NAc * d.KAc;
  if (q < PR) {
    const int64_t k = q % d.KR, n = (q / d.KR) % d.NR, J = (q / ((int64_t)d.KR * d.NR)) % d.T;
    const int64_t I = q / ((int64_t)d.KR * d.NR * d.T);
    return ((I * d.Tc + J) * d.NRc + n) * d.KRc + k;
  }
  q -= PR;
  if (q < PA) {
    const int64_t k = q % d.KA, n = (q / d.KA) % d.NA, J = (q / ((int64_t)d.KA * d.NA)) % d.T;
    const int64_t I = q / ((int64_t)d.KA * d.NA * d.T);
    return PRc + ((I * d.Tc + J) * d.NAc + n) * d.KAc + k;
  }
  q -= PA;
  const int64_t HD = (int64_t)d.H * d.D;
  const int64_t blk = HD + 2 * d.H + 1, blkc = (int64_t)d.H * d.Dc + 2 * d.H + 1;
  const int64_t I = q / blk, o = q % blk;
  const int64_t base = PRc + PAc + I * blkc;
  if (o < HD) return base + (o / d.D) * d.Dc + pad_col(d, (int)(o % d.D));
  return base + (int64_t)d.H * d.Dc + (o - HD);   // b0, w1, b1
}

__global__ __launch_bounds__(256) void k_pad_params(PadDims d, const float* __restrict__ p, float* __restrict__ pc) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q < d.P) pc[pad_index(d, q)] = p[q];
}

__global__ __launch_bounds__(256) void k_unpad_grad(PadDims d, const float* __restrict__ gc, float* __restrict__ g) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q < d.P) g[q] = gc[pad_index(d, q)];
}

// descriptor rows [Dc][N] of the class to the model's [D][N]
__global__ __launch_bounds__(256) void k_unpad_desc(PadDims d, int N, const float* __restrict__ Gc,
                                                    float* __restrict__ G) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q < (int64_t)d.D * N) G[q] = Gc[(int64_t)pad_col(d, (int)(q / N)) * N + q % N];
}

// ================================================================ dispatch
// ====================================================================== MD
// Velocity Verlet for the inference path, in eV, A, fs and amu: the
// acceleration of atom i is F_i / m_i times kAccel, and 1 amu A^2/fs^2 is
// 1/kAccel eV.
constexpr float kAccel = 9.648533212e-3f;

struct MDArgs {
  int N, T;
  const int* type;
  const int* astruct;
  const float* box;
  const float* tilt;   // null: every cell orthorhombic
  const float* mass;   // [T] amu
  float* pos;          // [3][N]
  float* vel;          // [3][N] A/fs
  const float* F;      // [3][N] eV/A
  float* ekin;         // [N] eV (kick only)
  float hdt, dt;
};

__device__ __forceinline__ float inv_mass(const MDArgs& a, int i) {
  const int t = a.type[i];
  return (t >= 0 && t < a.T) ? kAccel / a.mass[t] : 0.f;
}

// half kick with the forces at the current positions, drift, wrap into the
// cell: [0, L) per axis for an orthorhombic cell; for a triclinic one, minus
// the lattice vector H floor(f) of the fractional coordinates f = H^-1 x
__global__ __launch_bounds__(256) void k_md_drift(MDArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const float im = inv_mass(a, i);
  const int st = a.astruct[i];
  float x[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const size_t q = (size_t)c * a.N + i;
    const float v = fmaf(a.hdt * im, a.F[q], a.vel[q]);
    a.vel[q] = v;
    x[c] = fmaf(a.dt, v, a.pos[q]);
  }
  const float Lx = a.box[3 * st], Ly = a.box[3 * st + 1], Lz = a.box[3 * st + 2];
  const float xy = a.tilt ? a.tilt[3 * st] : 0.f, xz = a.tilt ? a.tilt[3 * st + 1] : 0.f,
              yz = a.tilt ? a.tilt[3 * st + 2] : 0.f;
  if (xy != 0.f || xz != 0.f || yz != 0.f) {
    const float fc = x[2] / Lz;
    const float fb = (x[1] - yz * fc) / Ly;
    const float fa = (x[0] - xy * fb - xz * fc) / Lx;
    const float ka = floorf(fa), kb = floorf(fb), kc = floorf(fc);
    x[0] = x[0] - Lx * ka - xy * kb - xz * kc;
    x[1] = x[1] - Ly * kb - yz * kc;
    x[2] = x[2] - Lz * kc;
  } else {
    const float L[3] = {Lx, Ly, Lz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[c] -= L[c] * floorf(x[c] / L[c]);
      if (x[c] >= L[c]) x[c] -= L[c];
      if (!(x[c] >= 0.f)) x[c] = 0.f;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) a.pos[(size_t)c * a.N + i] = x[c];
}

// half kick with the forces at the new positions; kinetic energy per atom
__global__ __launch_bounds__(256) void k_md_kick(MDArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const float im = inv_mass(a, i);
  float v2 = 0.f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const size_t q = (size_t)c * a.N + i;
    const float v = fmaf(a.hdt * im, a.F[q], a.vel[q]);
    a.vel[q] = v;
    v2 = fmaf(v, v, v2);
  }
  a.ekin[i] = im > 0.f ? 0.5f * v2 / im : 0.f;
}

// out[s] = sum of x over the atoms of structure s (float64, one block each)
__global__ __launch_bounds__(256) void k_struct_sum(const int* __restrict__ aoff, const float* __restrict__ x,
                                                    float* __restrict__ out) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  double acc = 0.0;
  for (int i = aoff[s] + threadIdx.x; i < aoff[s + 1]; i += blockDim.x) acc += x[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[s] = (float)red[0];
}

enum HighKernel { kHighDesc, kHighForce, kHighTangent, kHighCoef };

struct Ops {
  int T, NR, NA, KR, KA, L3, L4, L5, D, Y, PS, YH, YR;
  void (*forward)(const FwdArgs&, dim3, hipStream_t, int);
  void (*adjoint)(const AdjArgs&, dim3, hipStream_t, int);
  size_t (*lds_fwd)(int);
  size_t (*lds_adj)(int);
  void (*high)(HighKernel, const HighArgs&, dim3, hipStream_t);   // null without degrees l > 4
  // persistent step (null with degrees l > 4): launch, and resident blocks per CU
  void (*step)(const StepArgs*, int, size_t, hipStream_t);
  int (*step_occupancy)(size_t);
  bool padded;   // a size class: models up to its sizes run zero-padded
};

template <class C>
static size_t lds_forward(int H) {
  const int DP = (C::D + 3) & ~3;
  return sizeof(float) * ((size_t)CTab<C::T, C::NA, C::KA>::size + (size_t)weights_words(H, DP) +
                          (size_t)kAPB * (DP + C::NA * HRow<C::LMAX>::YR));
}
template <class C>
static size_t lds_adjoint(int H) {
  const int DP = (C::D + 3) & ~3;
  return sizeof(float) * ((size_t)CTab<C::T, C::NA, C::KA>::size + (size_t)weights_words(H, DP) +
                          (size_t)kAPB * (DP + 2 * C::NA * HRow<C::LMAX>::YR));
}
// LDS of a workgroup on gfx950 (160 KiB per CU); dynamic LDS beyond 64 KiB is
// requested from the runtime per kernel before its launch
constexpr size_t kMaxLds = 160 * 1024;
template <class K>
static void allow_lds(K* k, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

// the per-atom kernels are compiled for 2 and 3 wavefronts per SIMD
template <class C, int W>
static void launch_forward_w(const FwdArgs& a, dim3 grid, hipStream_t st) {
  const size_t lds = lds_forward<C>(a.H);
  if (a.tilt) {
    allow_lds(&k_forward<C, true, W>, lds);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_forward<C, true, W>), grid, dim3(256), lds, st, a);
  } else {
    allow_lds(&k_forward<C, false, W>, lds);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_forward<C, false, W>), grid, dim3(256), lds, st, a);
  }
}
template <class C>
static void launch_forward(const FwdArgs& a, dim3 grid, hipStream_t st, int waves) {
  if constexpr (C::FIXED_WAVES != 0)
    launch_forward_w<C, C::FIXED_WAVES>(a, grid, st);
  else if (waves == 2)
    launch_forward_w<C, 2>(a, grid, st);
  else
    launch_forward_w<C, 3>(a, grid, st);
}
template <class C, int W>
static void launch_adjoint_w(const AdjArgs& a, dim3 grid, hipStream_t st) {
  const size_t lds = lds_adjoint<C>(a.H);
  if (a.tilt) {
    allow_lds(&k_adjoint<C, true, W>, lds);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adjoint<C, true, W>), grid, dim3(256), lds, st, a);
  } else {
    allow_lds(&k_adjoint<C, false, W>, lds);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adjoint<C, false, W>), grid, dim3(256), lds, st, a);
  }
}
template <class C>
static void launch_adjoint(const AdjArgs& a, dim3 grid, hipStream_t st, int waves) {
  if constexpr (C::FIXED_WAVES != 0)
    launch_adjoint_w<C, C::FIXED_WAVES>(a, grid, st);
  else if (waves == 2)
    launch_adjoint_w<C, 2>(a, grid, st);
  else
    launch_adjoint_w<C, 3>(a, grid, st);
}
template <class C, bool kTri>
static void launch_high_t(HighKernel k, const HighArgs& a, dim3 grid, hipStream_t st) {
  switch (k) {
    case kHighDesc: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_high_desc<C, kTri>), grid, dim3(256), 0, st, a); break;
    case kHighForce: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_high_force<C, kTri>), grid, dim3(256), 0, st, a); break;
    case kHighTangent:
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_high_tangent<C, kTri>), grid, dim3(256), 0, st, a);
      break;
    case kHighCoef:   // one wavefront per block
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_high_coef<C, kTri>), dim3(grid.x * 4), dim3(kWave), 0, st, a);
      break;
  }
}
template <class C>
static void launch_high(HighKernel k, const HighArgs& a, dim3 grid, hipStream_t st) {
  if (a.tilt)
    launch_high_t<C, true>(k, a, grid, st);
  else
    launch_high_t<C, false>(k, a, grid, st);
}
template <class C>
static void launch_step(const StepArgs* a, int grid, size_t lds, hipStream_t st) {
  allow_lds(&k_step<C>, lds);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_step<C>), dim3(grid), dim3(256), lds, st, a);
}
template <class C>
static int step_occupancy(size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_step<C>), 256, lds) !=
      hipSuccess)
    return 0;
  return nb;
}
template <class C>
static Ops make_ops() {
  void (*high)(HighKernel, const HighArgs&, dim3, hipStream_t) = nullptr;
  void (*step)(const StepArgs*, int, size_t, hipStream_t) = nullptr;
  int (*occ)(size_t) = nullptr;
  if constexpr (C::YH > 0) high = &launch_high<C>;
  if constexpr (C::YH == 0 && C::FIXED_WAVES == 0) {
    step = &launch_step<C>;
    occ = &step_occupancy<C>;
  }
  return Ops{C::T, C::NR, C::NA, C::KR, C::KA, C::L3, C::L4, C::L5, C::D, C::Y, C::PS, C::YH,
             HRow<C::LMAX>::YR, &launch_forward<C>, &launch_adjoint<C>, &lds_forward<C>, &lds_adjoint<C>, high, step, occ,
             C::FIXED_WAVES != 0};
}

// Compiled-in model sizes (n_types, n_rad, n_ang, k_rad, k_ang, l3, l4, l5):
// exact shapes, then size classes that run any model up to their sizes with
// the parameters zero-padded (kPadClasses, smallest first).
static const Ops kOps[] = {
    make_ops<Cfg<2, 5, 5, 9, 9, 4, 0, 0>>(),    // 3-body NEP, basis 8, n_max 4
    make_ops<Cfg<2, 7, 5, 11, 11, 4, 2, 1>>(),  // 3/4/5-body NEP, basis 10, n_max 6/4
    make_ops<Cfg<2, 3, 2, 4, 3, 4, 2, 1>>(),    // small two-species model
    make_ops<Cfg<1, 4, 3, 6, 5, 2, 2, 0>>(),    // small one-species model
    make_ops<Cfg<2, 5, 4, 8, 8, 8, 2, 1>>(),    // 3-body degrees up to l = 8, n_max 4/3
};
static const Ops kPadClasses[] = {
    make_ops<Cfg<1, 12, 8, 12, 12, 4, 2, 1, 2>>(),
    make_ops<Cfg<2, 12, 8, 12, 12, 4, 2, 1, 2>>(),
    make_ops<Cfg<4, 12, 8, 12, 12, 4, 2, 1, 2>>(),
    make_ops<Cfg<1, 12, 8, 12, 12, 8, 2, 1, 2>>(),
    make_ops<Cfg<2, 12, 8, 12, 12, 8, 2, 1, 2>>(),
    make_ops<Cfg<4, 12, 8, 12, 12, 8, 2, 1, 2>>(),
};

}  // namespace nep

// ===================================================================== ABI
using namespace nep;

namespace {

// Kernels for a model: an exact compiled shape, else the smallest size class
// that holds it (the model then runs zero-padded as the class model `cls`).
struct Resolved {
  const Ops* o = nullptr;
  nep_model cls{};
  bool pad = false;
};

Resolved resolve(const nep_model* m) {
  Resolved r;
  for (const Ops& o : kOps)
    if (o.T == m->n_types && o.NR == m->n_rad && o.NA == m->n_ang && o.KR == m->k_rad && o.KA == m->k_ang &&
        o.L3 == m->l3 && o.L4 == m->l4 && o.L5 == m->l5) {
      r.o = &o;
      r.cls = *m;
      return r;
    }
  for (const Ops& o : kPadClasses)
    if (o.T >= m->n_types && o.NR >= m->n_rad && o.NA >= m->n_ang && o.KR >= m->k_rad && o.KA >= m->k_ang &&
        o.L3 >= m->l3 && o.L4 >= m->l4 && o.L5 >= m->l5) {
      r.o = &o;
      r.pad = true;
      r.cls = *m;
      r.cls.n_types = o.T;
      r.cls.n_rad = o.NR;
      r.cls.n_ang = o.NA;
      r.cls.k_rad = o.KR;
      r.cls.k_ang = o.KA;
      r.cls.l3 = o.L3;
      r.cls.l4 = o.L4;
      r.cls.l5 = o.L5;
      return r;
    }
  return r;
}

const Ops* find_ops(const nep_model* m) { return resolve(m).o; }

int model_valid(const nep_model* m) {
  if (!m) return NEP_ERR_ARG;
  if (m->n_types < 1 || m->n_types > 8 || m->n_rad < 1 || m->n_ang < 0 || m->k_rad < 1 || m->k_ang < 1 ||
      m->l3 < 0 || m->l3 > 8 || (m->l4 != 0 && m->l4 != 2) || (m->l5 != 0 && m->l5 != 1) || m->hidden < 1 ||
      m->hidden > 256 || !(m->rc_rad > 0.f) || !(m->rc_ang > 0.f) || m->rc_ang > m->rc_rad || m->cap_rad < 1 ||
      m->cap_ang < 1 || m->cap_rad > 4096 || m->cap_ang > 4096)
    return NEP_ERR_ARG;
  return NEP_OK;
}

int32_t desc_count(const nep_model* m) {
  return m->n_rad + m->n_ang * m->l3 + (m->l4 ? m->n_ang : 0) + (m->l5 ? m->n_ang : 0);
}

int64_t param_count(const nep_model* m) {
  const int64_t T = m->n_types, D = desc_count(m), H = m->hidden;
  return T * T * (m->n_rad * m->k_rad + m->n_ang * m->k_ang) + T * (H * D + 2 * H + 1);
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  int N, S, T, D, Y, H, NR, TKR, Npad, nwaves, nblk, PW, NA, capR, capA;
  size_t order, seg, blk, astruct, revR, revA, G, Sst, Ep, X, eatom, fR, fA, wv, F, fbar, Es, Ws, eps, wbar, lpart,
      Gd, FRst, FPst, Gbr, beta, w1s, part, pp, w0part, crpart, Sh, Sdh, cgrid, cell, cpart, acell, aslot, cpos, spart,
      cur_step, bar, sargs, prm, grd, Gtmp, total;
};

// m: the model the kernels run (the class model when padded)
Layout make_layout(const nep_model* m, const Ops* o, int S, int N, bool pad = false) {
  Layout L{};
  L.N = N;
  L.S = S;
  L.T = m->n_types;
  L.D = o->D;
  L.Y = o->Y;
  L.H = m->hidden;
  L.NA = m->n_ang;
  L.NR = m->n_rad;
  L.TKR = m->n_types * m->k_rad;
  L.capR = m->cap_rad;
  L.capA = m->cap_ang;
  // species segments (each rounded up to 32 atoms, one block) plus 16 atoms of slack for
  // the 16-atom groups of the outer-product sums
  const int n8 = ((N + kSegAlign - 1) / kSegAlign) * kSegAlign + L.T * kSegAlign + 16;
  L.Npad = ((n8 + kAPB - 1) / kAPB) * kAPB;
  L.nwaves = L.Npad / kAPW;
  L.nblk = N > 0 ? (N + kOrdBlk - 1) / kOrdBlk : 1;
  L.PW = L.T * m->n_ang * m->k_ang + 2 * L.H + 1;
  const size_t Np = L.Npad, Nn = (size_t)(N > 0 ? N : 1), Ss = (size_t)(S > 0 ? S : 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t r = off;
    off += al(bytes);
    return r;
  };
  L.order = take(4 * Np);
  L.seg = take(4 * 2 * 8);
  L.blk = take(4 * (size_t)L.nblk * L.T * kOrdBuckets);
  L.astruct = take(4 * Nn);
  L.revR = take(4 * (size_t)L.capR * Nn);
  L.revA = take(4 * (size_t)L.capA * Nn);
  L.G = take(4 * (size_t)L.D * Np);
  L.Sst = take(4 * (size_t)L.NA * o->YR * Np);
  L.Ep = take(4 * (size_t)L.D * Np);
  L.X = take(4 * (size_t)L.H * Np);
  L.eatom = take(4 * Nn);
  L.fR = take(4 * 3 * (size_t)L.capR * Nn);
  L.fA = take(4 * 3 * (size_t)L.capA * Nn);
  L.wv = take(4 * 6 * Nn);
  L.F = take(4 * 3 * Nn);
  L.fbar = take(4 * 3 * Nn);
  L.Es = take(4 * Ss);
  L.Ws = take(4 * 6 * Ss);
  L.eps = take(4 * Ss);
  L.wbar = take(4 * 6 * Ss);
  L.lpart = take(8 * 3 * Ss);
  L.Gd = take(4 * (size_t)L.D * Np);
  L.FRst = take(4 * (size_t)L.TKR * Np);
  L.FPst = take(4 * (size_t)L.TKR * Np);
  L.Gbr = take(4 * (size_t)(o->YH > 0 ? L.D : L.NR) * Np);
  L.beta = take(4 * (size_t)L.H * Np);
  L.w1s = take(4 * (size_t)L.H * Np);
  L.part = take(4 * (size_t)L.nwaves * L.PW);
  L.pp = take(8 * (size_t)L.T * kPRChunksMax * L.PW);
  L.w0part = take(4 * (size_t)L.T * kOSBlocksMaxW * L.H * L.D);
  L.crpart = take(4 * (size_t)L.T * kOSBlocksMaxC * L.NR * L.TKR);
  L.Sh = take(4 * (size_t)Np * L.NA * o->YH);
  L.Sdh = take(4 * (size_t)Np * L.NA * o->YH);
  L.cgrid = take(16 * Ss);
  L.cell = take(4 * (Nn + 1));
  L.cpart = take(4 * (Nn / kScanChunk + 1));
  L.acell = take(4 * Nn);
  L.aslot = take(4 * Nn);
  L.cpos = take(16 * Nn);
  L.spart = take(8 * 16 * (Nn / kStructChunk + 1));
  L.cur_step = take(4);
  L.bar = take(4 * kBarWords);
  L.sargs = take(sizeof(StepArgs));
  // a padded model: the class-layout parameters and gradient, and the class
  // descriptor rows of nep_descriptors
  const size_t Pc = pad ? (size_t)param_count(m) : 0;
  L.prm = take(4 * Pc);
  L.grd = take(4 * Pc);
  L.Gtmp = take(pad ? 4 * (size_t)L.D * Nn : 0);
  L.total = off;
  return L;
}

template <class P>
P* at(void* ws, size_t off) {
  return reinterpret_cast<P*>(static_cast<char*>(ws) + off);
}

int check_batch(const nep_batch* b) {
  if (!b || b->n_struct < 0 || b->n_atom < 0 || b->n_atom >= (1 << 27)) return NEP_ERR_ARG;
  if (b->n_struct == 0 && b->n_atom != 0) return NEP_ERR_ARG;
  if (b->n_struct > 0 && (!b->atom_offset || !b->box)) return NEP_ERR_ARG;
  if (b->n_atom > 0 && (!b->pos || !b->type)) return NEP_ERR_ARG;
  if (b->max_atoms < 0) return NEP_ERR_ARG;
  return NEP_OK;
}

int check_ws(const void* ws) {
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) return NEP_ERR_WORKSPACE;
  return NEP_OK;
}

int check_nbrs(const nep_neighbors* n, int N) {
  if (!n) return NEP_ERR_ARG;
  if (N > 0 && (!n->idx_rad || !n->cnt_rad || !n->idx_ang || !n->cnt_ang)) return NEP_ERR_ARG;
  return NEP_OK;
}

// Optional per-launch timing (nep_profile_loss_grad).
struct Prof {
  hipStream_t st;
  std::vector<hipEvent_t> ev;
  std::vector<const char*> names;
  void begin() {
    hipEvent_t e;
    (void)hipEventCreate(&e);
    (void)hipEventRecord(e, st);
    ev.push_back(e);
  }
  void end(const char* n) {
    begin();
    names.push_back(n);
  }
};

#define NEP_LAUNCH(prof, name, ...)  \
  do {                               \
    if (prof) (prof)->begin();       \
    __VA_ARGS__;                     \
    if (prof) (prof)->end(name);     \
  } while (0)

int hip_ok() { return hipGetLastError() == hipSuccess ? NEP_OK : NEP_ERR_HIP; }

// Launch choices of one evaluation (nep_tuning with the defaults filled in).
struct Tune {
  int persistent, outer_w, outer_c, reduce_chunks, cell_min, gather_lanes, forward_waves, adjoint_waves,
      reverse_branch;
};

Tune default_tune(const Ops* o) {
  return Tune{0, kOSBlocksW, kOSBlocksC, kPRChunks, kCellMinAtoms, kGatherLPA, 3, o->YH > 0 ? 2 : 3, 1};
}

struct Ctx {
  const nep_model* m;    // the model the kernels run: the caller's, or its size class
  const nep_model* mu;   // the caller's model
  nep_model mcls;        // the size-class model of a padded run
  bool pad = false;
  PadDims pd{};
  const Ops* o;
  const nep_batch* b;
  Tune tune;
  Layout L;
  void* ws;
  hipStream_t st;
  // the captured training step: Adam after the gradient, fused into its
  // final reduction
  const struct AdamFuse* adam = nullptr;
  // the captured step's side branch: the reverse index runs there, beside the
  // species order and the forward pass, and rejoins before the force gather
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  mutable bool rev_pending = false;
};

struct AdamFuse {
  int64_t P;
  float* th;
  float* mm;
  float* vv;
  const int* step;
  AdamDev ad;
  int* flags;
};

int grid1(int n, int blk = 256) { return (n + blk - 1) / blk; }

PairLists pair_lists(const Ctx& c, const nep_neighbors* nb) {
  PairLists p;
  p.idxR = nb->idx_rad;
  p.cntR = nb->cnt_rad;
  p.idxA = nb->idx_ang;
  p.cntA = nb->cnt_ang;
  p.revR = at<int>(c.ws, c.L.revR);
  p.revA = at<int>(c.ws, c.L.revA);
  p.capR = c.m->cap_rad;
  p.capA = c.m->cap_ang;
  return p;
}

OrderArgs order_args(const Ctx& c, const nep_neighbors* nb) {
  return OrderArgs{c.L.N, c.L.Npad, c.L.T, c.L.nblk, c.b->type, nb->cnt_ang, at<int>(c.ws, c.L.blk),
                   at<int>(c.ws, c.L.seg), at<int>(c.ws, c.L.order)};
}

void run_neighbors(const Ctx& c, nep_neighbors* nb, int32_t* flags, Prof* pr, bool with_order = true) {
  const int N = c.L.N;
  if (N == 0) return;
  NbrArgs a;
  a.N = N;
  a.S = c.b->n_struct;
  a.T = c.mu->n_types;   // types are checked against the caller's model
  a.capR = c.m->cap_rad;
  a.capA = c.m->cap_ang;
  a.rcR = c.m->rc_rad;
  a.rcA = c.m->rc_ang;
  a.aoff = c.b->atom_offset;
  a.box = c.b->box;
  a.tilt = c.b->tilt;
  a.pos = c.b->pos;
  a.type = c.b->type;
  a.idxR = nb->idx_rad;
  a.cntR = nb->cnt_rad;
  a.idxA = nb->idx_ang;
  a.cntA = nb->cnt_ang;
  a.astruct = at<int>(c.ws, c.L.astruct);
  a.flags = flags;
  // the cell-list kernels run unless the caller's bound rules out every structure
  const int S = c.b->n_struct;
  a.cell_min = c.tune.cell_min;
  a.cells = N >= a.cell_min && (c.b->max_atoms == 0 || c.b->max_atoms >= a.cell_min);
  a.grid = at<int4>(c.ws, c.L.cgrid);
  a.cell = at<int>(c.ws, c.L.cell);
  a.cpart = at<int>(c.ws, c.L.cpart);
  a.acell = at<int>(c.ws, c.L.acell);
  a.aslot = at<int>(c.ws, c.L.aslot);
  a.cpos = at<float4>(c.ws, c.L.cpos);
  if (a.cells) {
    const int nch = grid1(N, kScanChunk);
    if (a.tilt) {
      NEP_LAUNCH(pr, "cell_setup",
                 hipLaunchKernelGGL(k_cell_setup<true>, dim3(grid1(max(N + 1, S), 256)), dim3(256), 0, c.st, a));
      NEP_LAUNCH(pr, "cell_bin", hipLaunchKernelGGL(k_cell_bin<true>, dim3(grid1(N, 256)), dim3(256), 0, c.st, a));
    } else {
      NEP_LAUNCH(pr, "cell_setup",
                 hipLaunchKernelGGL(k_cell_setup<false>, dim3(grid1(max(N + 1, S), 256)), dim3(256), 0, c.st, a));
      NEP_LAUNCH(pr, "cell_bin", hipLaunchKernelGGL(k_cell_bin<false>, dim3(grid1(N, 256)), dim3(256), 0, c.st, a));
    }
    NEP_LAUNCH(pr, "cell_part",
               hipLaunchKernelGGL(k_cell_part, dim3(nch), dim3(256), 0, c.st, N, a.cell, a.cpart));
    NEP_LAUNCH(pr, "cell_start",
               hipLaunchKernelGGL(k_cell_start, dim3(nch), dim3(256), 0, c.st, N, a.cell, a.cpart));
    NEP_LAUNCH(pr, "cell_place", hipLaunchKernelGGL(k_cell_place, dim3(grid1(N, 256)), dim3(256), 0, c.st, a));
    if (a.tilt)
      NEP_LAUNCH(pr, "cell_neighbors", hipLaunchKernelGGL(k_cell_neighbors<true>, dim3(grid1(N, kNbrAPB)),
                                                          dim3(kNbrThreads), 0, c.st, a));
    else
      NEP_LAUNCH(pr, "cell_neighbors", hipLaunchKernelGGL(k_cell_neighbors<false>, dim3(grid1(N, kNbrAPB)),
                                                          dim3(kNbrThreads), 0, c.st, a));
  }
  {
    auto* k = a.tilt ? (a.cells ? k_neighbors<true, true> : k_neighbors<true, false>)
                     : (a.cells ? k_neighbors<false, true> : k_neighbors<false, false>);
    NEP_LAUNCH(pr, "neighbors", hipLaunchKernelGGL(k, dim3(grid1(N, kNbrAPB)), dim3(kNbrThreads), 0, c.st, a));
  }
  const RevArgs r{N, grid1(N, 256 / kRevLPAR), nb->idx_rad, nb->cnt_rad, c.m->cap_rad, at<int>(c.ws, c.L.revR),
                  nb->idx_ang, nb->cnt_ang, c.m->cap_ang, at<int>(c.ws, c.L.revA)};
  const int nrev = r.nbR + grid1(N, 256 / kRevLPAA);
  if (!with_order) {   // the persistent step computes the species order itself
    NEP_LAUNCH(pr, "reverse", hipLaunchKernelGGL(k_reverse, dim3(nrev), dim3(256), 0, c.st, r));
    return;
  }
  const OrderArgs oa = order_args(c, nb);
  if (c.side) {
    (void)hipEventRecord(c.fork, c.st);
    (void)hipStreamWaitEvent(c.side, c.fork, 0);
    NEP_LAUNCH(pr, "reverse", hipLaunchKernelGGL(k_reverse, dim3(nrev), dim3(256), 0, c.side, r));
    (void)hipEventRecord(c.join, c.side);
    c.rev_pending = true;
    NEP_LAUNCH(pr, "order_count",
               hipLaunchKernelGGL(k_reverse_count, dim3(c.L.nblk), dim3(256), 0, c.st, r, oa, 0));
  } else {
    NEP_LAUNCH(pr, "reverse_order_count",
               hipLaunchKernelGGL(k_reverse_count, dim3(nrev + c.L.nblk), dim3(256), 0, c.st, r, oa, nrev));
  }
  NEP_LAUNCH(pr, "order_scan", hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(512), 0, c.st, oa));
  NEP_LAUNCH(pr, "order_scatter",
             hipLaunchKernelGGL(k_order_scatter, dim3(c.L.nblk), dim3(kOrdBlk), 0, c.st, oa));
}

FwdArgs fwd_args(const Ctx& c, const nep_neighbors* nb, const float* params) {
  FwdArgs a;
  const nep_model* m = c.m;
  a.N = c.L.N;
  a.Npad = c.L.Npad;
  a.H = m->hidden;
  a.inv_rcR = 1.0f / m->rc_rad;
  a.inv_rcA = 1.0f / m->rc_ang;
  a.order = at<int>(c.ws, c.L.order);
  a.astruct = at<int>(c.ws, c.L.astruct);
  a.box = c.b->box;
  a.tilt = c.b->tilt;
  a.pos = c.b->pos;
  a.type = c.b->type;
  a.nb = pair_lists(c, nb);
  const int T = m->n_types;
  a.cR = params;
  a.cA = params + (size_t)T * T * m->n_rad * m->k_rad;
  a.nn = a.cA + (size_t)T * T * m->n_ang * m->k_ang;
  a.nn_stride = m->hidden * c.o->D + 2 * m->hidden + 1;
  a.G = at<float>(c.ws, c.L.G);
  a.Guser = nullptr;
  a.Sst = at<float>(c.ws, c.L.Sst);
  a.Ep = at<float>(c.ws, c.L.Ep);
  a.X = at<float>(c.ws, c.L.X);
  a.eatom = at<float>(c.ws, c.L.eatom);
  a.eatom2 = nullptr;
  a.fR = at<float>(c.ws, c.L.fR);
  a.fA = at<float>(c.ws, c.L.fA);
  a.wv = at<float>(c.ws, c.L.wv);
  a.do_mlp = 1;
  a.do_force = 1;
  return a;
}

// forward + force gather + per-structure sums (+ loss when labels given)
// arguments of the kernels of degrees l > 4 (fbar/wbar only for the adjoint's)
HighArgs high_args(const Ctx& c, const nep_neighbors* nb, const float* params, const float* fbar = nullptr,
                   const float* wbar = nullptr) {
  HighArgs h;
  const nep_model* m = c.m;
  h.N = c.L.N;
  h.Npad = c.L.Npad;
  h.PW = c.L.PW;
  h.inv_rcA = 1.0f / m->rc_ang;
  h.order = at<int>(c.ws, c.L.order);
  h.astruct = at<int>(c.ws, c.L.astruct);
  h.box = c.b->box;
  h.tilt = c.b->tilt;
  h.pos = c.b->pos;
  h.type = c.b->type;
  h.nb = pair_lists(c, nb);
  h.cA = params + (size_t)m->n_types * m->n_types * m->n_rad * m->k_rad;
  h.Sh = at<float>(c.ws, c.L.Sh);
  h.Sdh = at<float>(c.ws, c.L.Sdh);
  h.G = at<float>(c.ws, c.L.G);
  h.Ep = at<float>(c.ws, c.L.Ep);
  h.Gd = at<float>(c.ws, c.L.Gd);
  h.Gb = at<float>(c.ws, c.L.Gbr);
  h.fA = at<float>(c.ws, c.L.fA);
  h.wv = at<float>(c.ws, c.L.wv);
  h.fbar = fbar;
  h.wbar = wbar;
  h.part = at<float>(c.ws, c.L.part);
  return h;
}

void run_high(const Ctx& c, HighKernel k, const HighArgs& h, Prof* pr) {
  static const char* const names[] = {"high_desc", "high_force", "high_tangent", "high_coef"};
  if (c.o->high) NEP_LAUNCH(pr, names[k], c.o->high(k, h, dim3(c.L.Npad / kAPB), c.st));
}

// forward pass with the degrees l > 4 around it
void launch_forward_pass(const Ctx& c, const nep_neighbors* nb, const float* params, const FwdArgs& a, Prof* pr) {
  const HighArgs h = high_args(c, nb, params);
  run_high(c, kHighDesc, h, pr);
  NEP_LAUNCH(pr, "forward", c.o->forward(a, dim3(c.L.Npad / kAPB), c.st, c.tune.forward_waves));
  if (a.do_mlp && a.do_force) run_high(c, kHighForce, h, pr);
}

StructArgs struct_args(const Ctx& c, float* e_struct, float* virial, const nep_labels* lab, const float* lam) {
  StructArgs s;
  const int N = c.L.N;
  s.S = c.b->n_struct;
  s.N = N;
  s.aoff = c.b->atom_offset;
  s.eatom = at<float>(c.ws, c.L.eatom);
  s.wv = at<float>(c.ws, c.L.wv);
  s.F = at<float>(c.ws, c.L.F);
  s.Et = lab ? lab->energy : nullptr;
  s.Ft = lab ? lab->force : nullptr;
  s.Wt = lab ? lab->virial : nullptr;
  s.le = lam ? lam[0] : 0.f;
  s.lf = lam ? lam[1] : 0.f;
  s.lv = lam ? lam[2] : 0.f;
  s.Es = at<float>(c.ws, c.L.Es);
  s.Ws = at<float>(c.ws, c.L.Ws);
  s.Es_user = e_struct;
  s.Ws_user = virial;
  s.eps = at<float>(c.ws, c.L.eps);
  s.wbar = at<float>(c.ws, c.L.wbar);
  s.fbar = at<float>(c.ws, c.L.fbar);
  s.lpart = at<double>(c.ws, c.L.lpart);
  // large structures take chunk partials first, unless the caller's bound rules them out
  s.split = N >= 2 * kStructChunk && (c.b->max_atoms == 0 || c.b->max_atoms >= 2 * kStructChunk);
  s.spart = at<double>(c.ws, c.L.spart);
  return s;
}

void run_forward(const Ctx& c, const nep_neighbors* nb, const float* params, float* e_atom, float* e_struct,
                 float* force, float* virial, const nep_labels* lab, const float* lam, float* loss, int32_t* flags,
                 Prof* pr, bool defer_loss = false) {
  const int N = c.L.N, S = c.b->n_struct;
  if (N > 0) {
    FwdArgs a = fwd_args(c, nb, params);
    a.eatom2 = e_atom;
    launch_forward_pass(c, nb, params, a, pr);
    if (c.rev_pending) {
      (void)hipStreamWaitEvent(c.st, c.join, 0);
      c.rev_pending = false;
    }
    if (c.tune.gather_lanes == 8)
      NEP_LAUNCH(pr, "force_gather", hipLaunchKernelGGL(k_force_gather<8>, dim3(grid1(N, 256 / 8)), dim3(256), 0, c.st,
                                                        N, a.nb, a.fR, a.fA, at<float>(c.ws, c.L.F), force));
    else
      NEP_LAUNCH(pr, "force_gather", hipLaunchKernelGGL(k_force_gather<16>, dim3(grid1(N, 256 / 16)), dim3(256), 0,
                                                        c.st, N, a.nb, a.fR, a.fA, at<float>(c.ws, c.L.F), force));
  }
  if (S > 0) {
    const StructArgs s = struct_args(c, e_struct, virial, lab, lam);
    if (s.split)
      NEP_LAUNCH(pr, "struct_part",
                 hipLaunchKernelGGL(k_struct_part, dim3(grid1(N, kStructChunk)), dim3(kRedBlk), 0, c.st, s));
    NEP_LAUNCH(pr, "struct_sums", hipLaunchKernelGGL(k_struct, dim3(S), dim3(kRedBlk), 0, c.st, s));
    // with defer_loss the adjoint's first reduction launch sums the loss
    if (lab && !defer_loss)
      NEP_LAUNCH(pr, "loss_final",
                 hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kRedBlk), 0, c.st, S, N, s.le, s.lf, s.lv, s.lpart,
                                    loss, flags));
  }
}

AdjArgs adj_args(const Ctx& c, const nep_neighbors* nb, const float* params, const float* eps, const float* fbar,
                 const float* wbar) {
  const nep_model* m = c.m;
  AdjArgs a;
  a.N = c.L.N;
  a.Npad = c.L.Npad;
  a.H = m->hidden;
  a.S = c.b->n_struct;
  a.inv_rcR = 1.0f / m->rc_rad;
  a.inv_rcA = 1.0f / m->rc_ang;
  a.order = at<int>(c.ws, c.L.order);
  a.astruct = at<int>(c.ws, c.L.astruct);
  a.box = c.b->box;
  a.tilt = c.b->tilt;
  a.pos = c.b->pos;
  a.type = c.b->type;
  a.nb = pair_lists(c, nb);
  const int T = m->n_types;
  a.cR = params;
  a.cA = params + (size_t)T * T * m->n_rad * m->k_rad;
  a.nn = a.cA + (size_t)T * T * m->n_ang * m->k_ang;
  a.nn_stride = m->hidden * c.o->D + 2 * m->hidden + 1;
  a.Sst = at<float>(c.ws, c.L.Sst);
  a.Ep = at<float>(c.ws, c.L.Ep);
  a.X = at<float>(c.ws, c.L.X);
  a.eps = eps;
  a.fbar = fbar;
  a.wbar = wbar;
  a.Gd = at<float>(c.ws, c.L.Gd);
  a.FRst = at<float>(c.ws, c.L.FRst);
  a.FPst = at<float>(c.ws, c.L.FPst);
  a.Gbr = at<float>(c.ws, c.L.Gbr);
  a.beta = at<float>(c.ws, c.L.beta);
  a.w1s = at<float>(c.ws, c.L.w1s);
  a.part = at<float>(c.ws, c.L.part);
  a.PW = c.L.PW;
  return a;
}

// the two outer-product sums: dW0 (W) and dc^R (C)
void outer_args(const Ctx& c, const AdjArgs& a, OuterArgs& ow, OuterArgs& oc) {
  const nep_model* m = c.m;
  const int* seg = at<int>(c.ws, c.L.seg);
  ow = OuterArgs{c.L.Npad, m->hidden, c.o->D, c.tune.outer_w, seg, a.beta, at<float>(c.ws, c.L.G), a.w1s, a.Gd,
                 at<float>(c.ws, c.L.w0part)};
  oc = OuterArgs{c.L.Npad, m->n_rad, c.L.TKR, c.tune.outer_c, seg, a.Gbr, a.FRst, at<float>(c.ws, c.L.Ep), a.FPst,
                 at<float>(c.ws, c.L.crpart)};
}

GradArgs grad_args(const Ctx& c, float* grad) {
  const nep_model* m = c.m;
  GradArgs g;
  g.T = m->n_types;
  g.NR = m->n_rad;
  g.NA = m->n_ang;
  g.KR = m->k_rad;
  g.KA = m->k_ang;
  g.H = m->hidden;
  g.D = c.o->D;
  g.PW = c.L.PW;
  g.NBw = c.tune.outer_w;
  g.NBc = c.tune.outer_c;
  g.PRC = c.tune.reduce_chunks;
  g.P = param_count(m);
  g.pp = at<double>(c.ws, c.L.pp);
  g.w0part = at<float>(c.ws, c.L.w0part);
  g.crpart = at<float>(c.ws, c.L.crpart);
  g.grad = grad;
  g.adam = c.adam != nullptr && !c.pad;   // a padded model's Adam runs on its own layout
  if (c.adam) {
    g.ad = c.adam->ad;
    g.th = c.adam->th;
    g.mm = c.adam->mm;
    g.vv = c.adam->vv;
    g.step = c.adam->step;
    g.flags = c.adam->flags;
  }
  return g;
}

unsigned grad_final_blocks(const GradArgs& g) { return (unsigned)((g.P * 16 + 255) / 256); }

// adjoint + gradient reductions; cotangents from eps/fbar/wbar pointers
void run_adjoint(const Ctx& c, const nep_neighbors* nb, const float* params, const float* eps, const float* fbar,
                 const float* wbar, float* grad, Prof* pr, LossArgs la = LossArgs{}) {
  const nep_model* m = c.m;
  const int N = c.L.N;
  if (N > 0) {
    const AdjArgs a = adj_args(c, nb, params, eps, fbar, wbar);
    const int T = m->n_types;
    const HighArgs h = high_args(c, nb, params, fbar, wbar);
    run_high(c, kHighTangent, h, pr);
    NEP_LAUNCH(pr, "adjoint", c.o->adjoint(a, dim3(c.L.Npad / kAPB), c.st, c.tune.adjoint_waves));
    run_high(c, kHighCoef, h, pr);
    {
      OuterReduceArgs ra;
      outer_args(c, a, ra.ow, ra.oc);
      ra.nzw = outer_slices(ra.ow.M, ra.ow.V);
      ra.nzc = outer_slices(ra.oc.M, ra.oc.V);
      ra.os_x = std::max(ra.ow.NB, ra.oc.NB);
      ra.T = T;
      ra.PW = c.L.PW;
      ra.prc = c.tune.reduce_chunks;
      ra.seg = at<int>(c.ws, c.L.seg);
      ra.part = a.part;
      ra.pp = at<double>(c.ws, c.L.pp);
      ra.la = la;
      const int nblk = ra.os_x * T * (ra.nzw + ra.nzc) + ra.prc * T + (la.on ? 1 : 0);
      NEP_LAUNCH(pr, "outer_sums_reduce",
                 hipLaunchKernelGGL(k_outer_reduce, dim3(nblk), dim3(256), 0, c.st, ra));
    }
    // a padded model: the class gradient in the workspace, then the model's
    // entries, then Adam on the model's parameters
    float* gk = c.pad ? at<float>(c.ws, c.L.grd) : grad;
    const GradArgs g = grad_args(c, gk);
    NEP_LAUNCH(pr, "grad_final", hipLaunchKernelGGL(k_grad_final, dim3(grad_final_blocks(g)), dim3(256), 0, c.st, g));
    if (c.pad) {
      const unsigned nb = (unsigned)((c.pd.P + 255) / 256);
      NEP_LAUNCH(pr, "unpad_grad", hipLaunchKernelGGL(k_unpad_grad, dim3(nb), dim3(256), 0, c.st, c.pd, gk, grad));
      if (c.adam)
        hipLaunchKernelGGL(k_adam_dev, dim3(nb), dim3(256), 0, c.st, c.pd.P, c.adam->th, c.adam->mm, c.adam->vv, grad,
                           c.adam->step, c.adam->flags, c.adam->ad);
    }
  } else {
    const int64_t P = param_count(c.mu);
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, c.st, grad, P, 0.f);
    if (c.adam)
      hipLaunchKernelGGL(k_adam_dev, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, c.st, P, c.adam->th,
                         c.adam->mm, c.adam->vv, grad, c.adam->step, c.adam->flags, c.adam->ad);
  }
}

PadDims pad_dims(const nep_model* m, const nep_model* cls) {
  PadDims d;
  d.T = m->n_types;
  d.NR = m->n_rad;
  d.NA = m->n_ang;
  d.KR = m->k_rad;
  d.KA = m->k_ang;
  d.D = desc_count(m);
  d.H = m->hidden;
  d.l3 = m->l3;
  d.l4 = m->l4;
  d.l5 = m->l5;
  d.Tc = cls->n_types;
  d.NRc = cls->n_rad;
  d.NAc = cls->n_ang;
  d.KRc = cls->k_rad;
  d.KAc = cls->k_ang;
  d.Dc = desc_count(cls);
  d.L3c = cls->l3;
  d.P = param_count(m);
  return d;
}

// kernels exist for the model and their LDS fits
int model_supported(const nep_model* m, Resolved* out = nullptr) {
  int rc = model_valid(m);
  if (rc) return rc;
  const Resolved r = resolve(m);
  if (!r.o) return NEP_ERR_ARG;
  if (r.o->lds_adj(m->hidden) > kMaxLds || r.o->lds_fwd(m->hidden) > kMaxLds) return NEP_ERR_ARG;
  if (out) *out = r;
  return NEP_OK;
}

size_t workspace_size(const nep_model* m, int S, int N) {
  const Resolved r = resolve(m);
  return make_layout(&r.cls, r.o, S, N, r.pad).total;
}

int setup(Ctx& c, const nep_model* m, const nep_batch* b, void* ws, void* stream) {
  Resolved r;
  int rc = model_supported(m, &r);
  if (rc) return rc;
  if ((rc = check_batch(b))) return rc;
  if ((rc = check_ws(ws))) return rc;
  c.o = r.o;
  c.mu = m;
  c.pad = r.pad;
  c.mcls = r.cls;
  c.m = r.pad ? &c.mcls : m;
  if (r.pad) c.pd = pad_dims(m, &c.mcls);
  c.b = b;
  c.tune = default_tune(c.o);
  c.ws = ws;
  c.st = static_cast<hipStream_t>(stream);
  c.L = make_layout(c.m, c.o, b->n_struct, b->n_atom, r.pad);
  return NEP_OK;
}

// The parameters the kernels read: the caller's, or for a padded model their
// class-layout copy in the workspace (filled by launches on the call's stream).
const float* kernel_params(const Ctx& c, const float* params) {
  if (!c.pad) return params;
  float* pc = at<float>(c.ws, c.L.prm);
  const int64_t Pc = param_count(c.m);
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((Pc + 255) / 256)), dim3(256), 0, c.st, pc, Pc, 0.f);
  hipLaunchKernelGGL(k_pad_params, dim3((unsigned)((c.pd.P + 255) / 256)), dim3(256), 0, c.st, c.pd, params, pc);
  return pc;
}

// loss sum carried by the first reduction launch after the adjoint
LossArgs loss_args(const Ctx& c, const nep_labels* labels, const float* lam, float* loss, int32_t* flags) {
  LossArgs la{};
  const int N = c.L.N, S = c.b->n_struct;
  if (N > 0 && S > 0 && labels) {
    la.on = 1;
    la.S = S;
    la.N = N;
    la.le = lam[0];
    la.lf = lam[1];
    la.lv = lam[2];
    la.lpart = at<double>(c.ws, c.L.lpart);
    la.loss = loss;
    la.flags = flags;
  }
  return la;
}

int loss_grad_seq(Ctx& c, nep_neighbors* nb, const float* params, const nep_labels* labels, const float* lam,
                  float* loss, float* grad, float* e_struct, float* force, float* virial, int32_t* flags, Prof* pr,
                  bool with_neighbors) {
  if (with_neighbors) run_neighbors(c, nb, flags, pr);
  if (c.b->n_struct == 0) hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(64), 0, c.st, loss, (int64_t)4, 0.f);
  // with atoms present the loss is summed by the adjoint's reduction launch
  const LossArgs la = loss_args(c, labels, lam, loss, flags);
  run_forward(c, nb, params, nullptr, e_struct, force, virial, labels, lam, loss, flags, pr, la.on != 0);
  run_adjoint(c, nb, params, at<float>(c.ws, c.L.eps), at<float>(c.ws, c.L.fbar), at<float>(c.ws, c.L.wbar), grad,
              pr, la);
  return hip_ok();
}

// ---- persistent step: everything after the neighbor build in one launch
size_t step_lds(const Ctx& c) {
  size_t l = std::max(c.o->lds_fwd(c.m->hidden), c.o->lds_adj(c.m->hidden));
  l = std::max(l, (size_t)kOrdScatterLds * sizeof(int));
  l = std::max(l, (size_t)kOrdScanLds * sizeof(int));
  l = std::max(l, (size_t)kStructLds);
  l = std::max(l, (size_t)kOuterLds);
  l = std::max(l, (size_t)kLossLds);
  return l;
}

// Blocks of the persistent grid: as many as are resident at once, a multiple
// of the XCD count; 0 when the kernel cannot run.
int step_grid(const Ctx& c, size_t lds) {
  if (!c.o->step) return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const int per = c.o->step_occupancy(lds);
  return per * cus / kXCD * kXCD;
}

// The persistent step covers orthorhombic batches with atoms and structures,
// for models without degrees l > 4.
bool persistent_ok(const Ctx& c) { return c.o->step && !c.b->tilt && c.L.N > 0 && c.b->n_struct > 0; }

StepArgs step_args(const Ctx& c, nep_neighbors* nb, const float* params, const nep_labels* labels,
                   const float* lam, float* loss, float* grad, int32_t* flags) {
  StepArgs a;
  a.ord = order_args(c, nb);
  a.fwd = fwd_args(c, nb, params);
  a.nb = a.fwd.nb;
  a.F = at<float>(c.ws, c.L.F);
  a.st = struct_args(c, nullptr, nullptr, labels, lam);
  a.adj = adj_args(c, nb, params, at<float>(c.ws, c.L.eps), at<float>(c.ws, c.L.fbar), at<float>(c.ws, c.L.wbar));
  outer_args(c, a.adj, a.ow, a.oc);
  a.nzw = outer_slices(a.ow.M, a.ow.V);
  a.nzc = outer_slices(a.oc.M, a.oc.V);
  a.os_x = std::max(a.ow.NB, a.oc.NB);
  a.PW = c.L.PW;
  a.seg = at<int>(c.ws, c.L.seg);
  a.pp = at<double>(c.ws, c.L.pp);
  a.la = loss_args(c, labels, lam, loss, flags);
  a.g = grad_args(c, grad);
  a.n_gf = (int)grad_final_blocks(a.g);
  a.bar = at<unsigned>(c.ws, c.L.bar);
  a.flags = flags;
  return a;
}

struct GraphHandle {
  hipGraph_t g;
  hipGraphExec_t e;
};

// Adam's hyper-parameters: beta in [0, 1) (the bias correction divides by
// 1 - beta^step), eps >= 0 finite.
bool adam_hparams_ok(float beta1, float beta2, float eps) {
  return beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f && std::isfinite(eps);
}

// Overrides of the launch choices; 0 keeps the default.  NEP_ERR_ARG out of range.
int apply_tuning(Tune& t, const nep_tuning* u) {
  if (!u) return NEP_OK;
  auto set = [](int& dst, int v, int lo, int hi) {
    if (v == 0) return true;
    if (v < lo || v > hi) return false;
    dst = v;
    return true;
  };
  bool ok = u->persistent == 0 || u->persistent == 1;
  t.persistent = u->persistent;
  ok = ok && set(t.outer_w, u->outer_blocks_w, 1, kOSBlocksMaxW);
  ok = ok && set(t.outer_c, u->outer_blocks_c, 1, kOSBlocksMaxC);
  ok = ok && set(t.reduce_chunks, u->reduce_chunks, 1, kPRChunksMax);
  ok = ok && set(t.cell_min, u->cell_min_atoms, kCellMinAtomsLo, 1 << 27);
  ok = ok && (u->gather_lanes == 0 || u->gather_lanes == 8 || u->gather_lanes == 16);
  if (u->gather_lanes) t.gather_lanes = u->gather_lanes;
  ok = ok && set(t.forward_waves, u->forward_waves, 2, 3);
  ok = ok && set(t.adjoint_waves, u->adjoint_waves, 2, 3);
  ok = ok && set(t.reverse_branch, u->reverse_branch, 1, 2);
  return ok ? NEP_OK : NEP_ERR_ARG;
}

int check_adam_config(const nep_adam_config* a) {
  if (!adam_hparams_ok(a->beta1, a->beta2, a->eps)) return NEP_ERR_ARG;
  if (!std::isfinite(a->lr_start) || !std::isfinite(a->lr_stop) || a->n_warmup < 0) return NEP_ERR_ARG;
  return NEP_OK;
}

// Scratch of nep_loss_grad_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol); it uses the
// device address hipGetSymbolAddress returns, taken once per device with that
// device current.
static __device__ __align__(256) unsigned char scratch[NEP_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return NEP_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NEP_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NEP_OK;
}

}  // namespace

extern "C" {

int64_t nep_param_count(const nep_model* m) {
  const int rc = model_valid(m);
  return rc ? rc : param_count(m);
}

int32_t nep_descriptor_count(const nep_model* m) {
  const int rc = model_valid(m);
  return rc ? rc : desc_count(m);
}

int nep_model_supported(const nep_model* m) { return model_supported(m); }

int nep_workspace_bytes(const nep_model* m, int32_t n_struct, int32_t n_atom, size_t* bytes) {
  int rc = nep_model_supported(m);
  if (rc) return rc;
  if (!bytes || n_struct < 0 || n_atom < 0 || n_atom >= (1 << 27)) return NEP_ERR_ARG;
  *bytes = workspace_size(m, n_struct, n_atom);
  return NEP_OK;
}

int nep_build_neighbors(const nep_model* m, const nep_batch* b, nep_neighbors* out, void* ws, int32_t* d_flags,
                        void* stream) {
  Ctx c;
  int rc = setup(c, m, b, ws, stream);
  if (rc) return rc;
  if ((rc = check_nbrs(out, b->n_atom))) return rc;
  if (!d_flags) return NEP_ERR_ARG;
  run_neighbors(c, out, d_flags, nullptr);
  return hip_ok();
}

int nep_descriptors(const nep_model* m, const nep_batch* b, const nep_neighbors* nb, const float* params, float* G,
                    void* ws, void* stream) {
  Ctx c;
  int rc = setup(c, m, b, ws, stream);
  if (rc) return rc;
  if ((rc = check_nbrs(nb, b->n_atom))) return rc;
  if (b->n_atom > 0 && (!params || !G)) return NEP_ERR_ARG;
  if (b->n_atom == 0) return NEP_OK;
  const float* kp = kernel_params(c, params);
  FwdArgs a = fwd_args(c, nb, kp);
  a.Guser = c.pad ? at<float>(c.ws, c.L.Gtmp) : G;
  a.do_mlp = 0;
  a.do_force = 0;
  launch_forward_pass(c, nb, kp, a, nullptr);
  if (c.pad)
    hipLaunchKernelGGL(k_unpad_desc, dim3((unsigned)(((int64_t)c.pd.D * b->n_atom + 255) / 256)), dim3(256), 0, c.st,
                       c.pd, b->n_atom, a.Guser, G);
  return hip_ok();
}

int nep_energy_force_virial(const nep_model* m, const nep_batch* b, const nep_neighbors* nb, const float* params,
                            float* e_atom, float* e_struct, float* force, float* virial, void* ws, void* stream) {
  Ctx c;
  int rc = setup(c, m, b, ws, stream);
  if (rc) return rc;
  if ((rc = check_nbrs(nb, b->n_atom))) return rc;
  if (!params) return NEP_ERR_ARG;
  run_forward(c, nb, kernel_params(c, params), e_atom, e_struct, force, virial, nullptr, nullptr, nullptr, nullptr,
              nullptr);
  return hip_ok();
}

int nep_md_step(const nep_model* m, const nep_batch* b, float* pos, nep_neighbors* nb, const float* params,
                const float* mass, float* vel, float* force, float dt, int32_t n_steps, float* e_pot, float* e_kin,
                void* ws, int32_t* d_flags, void* stream) {
  Ctx c;
  int rc = setup(c, m, b, ws, stream);
  if (rc) return rc;
  if ((rc = check_nbrs(nb, b->n_atom))) return rc;
  const int N = b->n_atom, S = b->n_struct;
  if (!params || !mass || !d_flags || n_steps < 0 || !std::isfinite(dt)) return NEP_ERR_ARG;
  if (N > 0 && (pos != b->pos || !vel || !force)) return NEP_ERR_ARG;
  if (N == 0 || n_steps == 0) return NEP_OK;
  MDArgs a;
  a.N = N;
  a.T = m->n_types;
  a.type = b->type;
  a.astruct = at<int>(c.ws, c.L.astruct);
  a.box = b->box;
  a.tilt = b->tilt;
  a.mass = mass;
  a.pos = pos;
  a.vel = vel;
  a.F = force;
  a.ekin = at<float>(c.ws, c.L.eatom);   // reused after the last force evaluation
  a.hdt = 0.5f * dt;
  a.dt = dt;
  params = kernel_params(c, params);
  for (int k = 0; k < n_steps; ++k) {
    hipLaunchKernelGGL(k_md_drift, dim3(grid1(N)), dim3(256), 0, c.st, a);
    run_neighbors(c, nb, d_flags, nullptr);
    run_forward(c, nb, params, nullptr, e_pot, force, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    hipLaunchKernelGGL(k_md_kick, dim3(grid1(N)), dim3(256), 0, c.st, a);
  }
  if (e_kin && S > 0)
    hipLaunchKernelGGL(k_struct_sum, dim3(S), dim3(256), 0, c.st, b->atom_offset, a.ekin, e_kin);
  return hip_ok();
}

int nep_vjp(const nep_model* m, const nep_batch* b, const nep_neighbors* nb, const float* params, const float* e_bar,
            const float* f_bar, const float* v_bar, float* grad, void* ws, void* stream) {
  Ctx c;
  int rc = setup(c, m, b, ws, stream);
  if (rc) return rc;
  if ((rc = check_nbrs(nb, b->n_atom))) return rc;
  if (!params || !grad) return NEP_ERR_ARG;
  if (b->n_atom > 0 && (!e_bar || !f_bar || !v_bar)) return NEP_ERR_ARG;
  params = kernel_params(c, params);
  if (b->n_atom > 0) {
    FwdArgs a = fwd_args(c, nb, params);
    a.do_force = 0;
    launch_forward_pass(c, nb, params, a, nullptr);
  }
  run_adjoint(c, nb, params, e_bar, f_bar, v_bar, grad, nullptr);
  return hip_ok();
}

int nep_loss_grad(const nep_model* m, const nep_batch* b, const nep_neighbors* nb, const float* params,
                  const nep_labels* labels, const float lambda[3], float* loss, float* grad, float* e_struct,
                  float* force, float* virial, void* ws, int32_t* d_flags, void* stream) {
  Ctx c;
  int rc = setup(c, m, b, ws, stream);
  if (rc) return rc;
  if ((rc = check_nbrs(nb, b->n_atom))) return rc;
  if (!params || !labels || !lambda || !loss || !grad) return NEP_ERR_ARG;
  if (b->n_struct > 0 && (!labels->energy || !labels->virial)) return NEP_ERR_ARG;
  if (b->n_atom > 0 && !labels->force) return NEP_ERR_ARG;
  return loss_grad_seq(c, const_cast<nep_neighbors*>(nb), kernel_params(c, params), labels, lambda, loss, grad,
                       e_struct, force, virial, d_flags, nullptr, false);
}

int nep_loss_grad_noalloc(const nep_model* m, const nep_batch* b, nep_neighbors* nb, const float* params,
                          const nep_labels* labels, const float lambda[3], float* loss, float* grad, float* e_struct,
                          float* force, float* virial, int32_t* d_flags, void* stream) {
  int rc = nep_model_supported(m);
  if (rc) return rc;
  if ((rc = check_batch(b))) return rc;
  if (workspace_size(m, b->n_struct, b->n_atom) > (size_t)NEP_STATIC_SCRATCH_BYTES)
    return NEP_ERR_SCRATCH;
  void* ws = nullptr;
  if ((rc = static_scratch(&ws))) return rc;
  Ctx c;
  if ((rc = setup(c, m, b, ws, stream))) return rc;
  if ((rc = check_nbrs(nb, b->n_atom))) return rc;
  if (!params || !labels || !lambda || !loss || !grad || !d_flags) return NEP_ERR_ARG;
  if (b->n_struct > 0 && (!labels->energy || !labels->virial)) return NEP_ERR_ARG;
  if (b->n_atom > 0 && !labels->force) return NEP_ERR_ARG;
  return loss_grad_seq(c, nb, kernel_params(c, params), labels, lambda, loss, grad, e_struct, force, virial, d_flags,
                       nullptr, true);
}

int nep_adam_step(int64_t P, float* params, float* mm, float* vv, const float* grad, float lr, float beta1,
                  float beta2, float eps, int32_t step, void* stream) {
  if (P < 0 || step < 1 || !adam_hparams_ok(beta1, beta2, eps) || !std::isfinite(lr)) return NEP_ERR_ARG;
  if (P == 0) return NEP_OK;
  if (!params || !mm || !vv || !grad) return NEP_ERR_ARG;
  const float c1 = 1.0f - (float)std::pow((double)beta1, (double)step);
  const float c2 = 1.0f - (float)std::pow((double)beta2, (double)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream), P,
                     params, mm, vv, grad, lr, beta1, beta2, eps, c1, c2);
  return hip_ok();
}

float nep_lr_schedule(int64_t s, float lr_start, float lr_stop, int64_t n_warmup, int64_t n_total) {
  if (n_total <= 0) return lr_start;
  if (s < n_warmup) return lr_stop + (float)((double)s / (double)n_warmup) * (lr_start - lr_stop);
  double fr = (double)(s - n_warmup) / (double)std::max<int64_t>(1, n_total - n_warmup);
  fr = fr > 1.0 ? 1.0 : fr;
  return lr_stop + (lr_start - lr_stop) * 0.5f * (1.0f + (float)std::cos(3.14159265358979323846 * fr));
}

int nep_train_step_graph_create(const nep_model* m, const nep_batch* b, nep_neighbors* nb, const nep_labels* labels,
                                const float lambda[3], float* params, float* mm, float* vv, float* grad, float* loss,
                                int32_t* d_step, const nep_adam_config* adam, void* ws, int32_t* d_flags,
                                int32_t graph_flags, void* stream, void** graph) {
  return nep_train_step_graph_create_tuned(m, b, nb, labels, lambda, params, mm, vv, grad, loss, d_step, adam, ws,
                                           d_flags, graph_flags, nullptr, stream, graph);
}

int nep_train_step_graph_create_tuned(const nep_model* m, const nep_batch* b, nep_neighbors* nb,
                                      const nep_labels* labels, const float lambda[3], float* params, float* mm,
                                      float* vv, float* grad, float* loss, int32_t* d_step,
                                      const nep_adam_config* adam, void* ws, int32_t* d_flags, int32_t graph_flags,
                                      const nep_tuning* tuning, void* stream, void** graph) {
  Ctx c;
  int rc = setup(c, m, b, ws, stream);
  if (rc) return rc;
  if ((rc = apply_tuning(c.tune, tuning))) return rc;
  if ((rc = check_nbrs(nb, b->n_atom))) return rc;
  if (!labels || !lambda || !params || !mm || !vv || !grad || !loss || !d_step || !adam || !d_flags || !graph)
    return NEP_ERR_ARG;
  if ((rc = check_adam_config(adam))) return rc;
  const bool persistent = (graph_flags & NEP_GRAPH_PERSISTENT) != 0 || c.tune.persistent;
  size_t slds = 0;
  int sgrid = 0;
  if (persistent) {
    if (!persistent_ok(c)) return NEP_ERR_ARG;
    slds = step_lds(c);
    sgrid = step_grid(c, slds);
    if (sgrid < kXCD) return NEP_ERR_HIP;
  }
  hipStream_t cap;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return NEP_ERR_HIP;
  c.st = cap;
  // the reverse index's own branch (a stream of default priority, as every stream here)
  auto drop_side = [&c]() {
    if (c.side) (void)hipStreamDestroy(c.side);
    if (c.fork) (void)hipEventDestroy(c.fork);
    if (c.join) (void)hipEventDestroy(c.join);
    c.side = nullptr;
  };
  if (!persistent && c.tune.reverse_branch == 2 && (hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking) != hipSuccess ||
                      hipEventCreateWithFlags(&c.fork, hipEventDisableTiming) != hipSuccess ||
                      hipEventCreateWithFlags(&c.join, hipEventDisableTiming) != hipSuccess)) {
    drop_side();
    (void)hipStreamDestroy(cap);
    return NEP_ERR_HIP;
  }
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    drop_side();
    (void)hipStreamDestroy(cap);
    return NEP_ERR_HIP;
  }
  int* cur = at<int>(c.ws, c.L.cur_step);
  // Adam runs inside the gradient's final reduction
  const AdamFuse af{param_count(m), params, mm, vv, cur,
                    AdamDev{adam->lr_start, adam->lr_stop, adam->n_warmup, adam->n_total, adam->beta1, adam->beta2,
                            adam->eps},
                    d_flags};
  c.adam = &af;
  if (persistent) {
    StepArgs* sa = at<StepArgs>(c.ws, c.L.sargs);
    hipLaunchKernelGGL(k_step_head, dim3(1), dim3(64), 0, cap,
                       step_args(c, nb, params, labels, lambda, loss, grad, d_flags), sa, d_flags, d_step, cur);
    if ((graph_flags & NEP_GRAPH_CACHED_NEIGHBORS) == 0) run_neighbors(c, nb, d_flags, nullptr, false);
    c.o->step(sa, sgrid, slds, cap);
  } else {
    hipLaunchKernelGGL(k_graph_head, dim3(1), dim3(64), 0, cap, d_flags, d_step, cur);
    // a padded model's class-layout parameters are refreshed by every replay
    loss_grad_seq(c, nb, kernel_params(c, params), labels, lambda, loss, grad, nullptr, nullptr, nullptr, d_flags,
                  nullptr, (graph_flags & NEP_GRAPH_CACHED_NEIGHBORS) == 0);
  }
  const hipError_t e1 = hipStreamEndCapture(cap, &g);
  (void)hipStreamDestroy(cap);
  drop_side();
  if (e1 != hipSuccess || !g) return NEP_ERR_HIP;
  hipGraphExec_t ex;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return NEP_ERR_HIP;
  }
  GraphHandle* h = new (std::nothrow) GraphHandle{g, ex};
  if (!h) {
    (void)hipGraphExecDestroy(ex);
    (void)hipGraphDestroy(g);
    return NEP_ERR_HIP;
  }
  *graph = h;
  return NEP_OK;
}

int nep_train_step_graph_launch(void* graph, void* stream) {
  if (!graph) return NEP_ERR_ARG;
  GraphHandle* h = static_cast<GraphHandle*>(graph);
  return hipGraphLaunch(h->e, static_cast<hipStream_t>(stream)) == hipSuccess ? NEP_OK : NEP_ERR_HIP;
}

int nep_train_step_graph_destroy(void* graph) {
  if (!graph) return NEP_OK;
  GraphHandle* h = static_cast<GraphHandle*>(graph);
  (void)hipGraphExecDestroy(h->e);
  (void)hipGraphDestroy(h->g);
  delete h;
  return NEP_OK;
}

int nep_profile_loss_grad(const nep_model* m, const nep_batch* b, nep_neighbors* nb, const float* params,
                          const nep_labels* labels, const float lambda[3], float* loss, float* grad, void* ws,
                          int32_t* d_flags, void* stream, float* ms, const char** names, int32_t max_kernels,
                          int32_t* n_kernels) {
  Ctx c;
  int rc = setup(c, m, b, ws, stream);
  if (rc) return rc;
  if ((rc = check_nbrs(nb, b->n_atom))) return rc;
  if (!labels || !lambda || !params || !loss || !grad || !d_flags || !n_kernels) return NEP_ERR_ARG;
  Prof pr;
  pr.st = c.st;
  rc = loss_grad_seq(c, nb, kernel_params(c, params), labels, lambda, loss, grad, nullptr, nullptr, nullptr, d_flags,
                     &pr, true);
  if (hipStreamSynchronize(c.st) != hipSuccess) rc = NEP_ERR_HIP;
  const int n = (int)pr.names.size();
  *n_kernels = n;
  for (int k = 0; k < n && k < max_kernels; ++k) {
    float t = 0.f;
    (void)hipEventElapsedTime(&t, pr.ev[2 * k], pr.ev[2 * k + 1]);
    if (ms) ms[k] = t;
    if (names) names[k] = pr.names[k];
  }
  for (hipEvent_t e : pr.ev) (void)hipEventDestroy(e);
  return rc;
}

int nep_flags_status(int32_t f) {
  if (f & FL_BARRIER) return NEP_ERR_HIP;
  if (f & FL_BOX) return NEP_ERR_BOX;
  if (f & FL_TYPE) return NEP_ERR_TYPE;
  if (f & FL_POS) return NEP_ERR_POSITION;
  if (f & FL_OVERFLOW) return NEP_ERR_NBR_OVERFLOW;
  if (f & FL_NONFINITE) return NEP_ERR_NONFINITE;
  if (f & FL_STEP) return NEP_ERR_ARG;
  return NEP_OK;
}

const char* nep_status_string(int code) {
  switch (code) {
    case NEP_OK: return "ok";
    case NEP_ERR_ARG: return "invalid argument or unsupported model";
    case NEP_ERR_BOX: return "a box edge is shorter than rc_rad";
    case NEP_ERR_NBR_OVERFLOW: return "neighbor list capacity exceeded";
    case NEP_ERR_NONFINITE: return "loss is not finite";
    case NEP_ERR_HIP: return "HIP runtime error";
    case NEP_ERR_WORKSPACE: return "workspace missing or not 256-byte aligned";
    case NEP_ERR_TYPE: return "atom type out of range";
    case NEP_ERR_POSITION: return "coordinate outside [0, L)";
    case NEP_ERR_SCRATCH: return "batch needs more than the static scratch of nep_loss_grad_noalloc";
    default: return "unknown status";
  }
}

}  // extern "C"
