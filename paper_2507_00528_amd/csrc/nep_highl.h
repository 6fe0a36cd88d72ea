// Angular degrees l = 5..L3 of the 3-body descriptor (Eq. 7, Appendix B up
// to B8.17).  The kernels in nep_lib.hip keep the l <= 4 sums in registers, 8
// lanes per atom; the 56 harmonics of l = 5..8 do not fit there, so these
// degrees run in kernels of their own around the forward and adjoint passes:
//
//   k_high_desc    (before the forward)  S_nlm and q_nl into the G rows
//   k_high_force   (after the forward)   pair forces and virial of these q_nl
//   k_high_tangent (before the adjoint)  Sdot_nlm and Gdot of these q_nl
//   k_high_coef    (after the adjoint)   their share of dL/dc^A
//
// One wavefront takes the 8 atoms of an atom group (the same species-ordered
// positions as the main kernels), one atom after the other; lane c holds
// harmonic (l, m) number c of l = 5..L3 (at most 56), for every channel n.
// Pair data (direction, g_n, g'_n, tangent) is staged once per pair in LDS by
// the lane of that pair and read back by every lane.
//
// Harmonic basis.  q_nl = sum_m C_lm S_nlm^2 with C_lm = 1 / integral of b_lm^2
// equals sum_m S~_nlm^2 for the sums S~ of any orthonormal real harmonics of
// degree l (both are (2l+1)/(4 pi) sum_jk g_n g_n P_l(u_j . u_k), the addition
// theorem).  So these kernels use the orthonormal real harmonics
//   Y_lm = N_lM Q_l^M(z) Re (x + i y)^M   (m = 2M - 1, or m = 0 with M = 0)
//   Y_lm = N_lM Q_l^M(z) Im (x + i y)^M   (m = 2M)
// with Q_l^M the associated Legendre function over (1 - z^2)^(M/2), from the
// three-term recurrence in l, and N_lM^2 = (2l+1)/(4 pi) (l-M)!/(l+M)! (times
// 2 for M > 0).  With C = 1 in this basis, dq/dS~ = 2 S~.
#pragma once
#include "nep_device.h"
#include "nep_kernels.h"

namespace nep {

struct HighLane {
  int l, M;
  bool sine;
  float N;   // 0 for lanes past the last harmonic
};

__device__ __forceinline__ HighLane high_lane(int c, int L3) {
  HighLane h{5, 0, false, 0.f};
  int off = 0;
  bool on = false;
  for (int l = 5; l <= L3; ++l) {
    const int w = 2 * l + 1;
    if (c >= off && c < off + w) {
      const int mi = c - off;
      h.l = l;
      h.M = (mi + 1) >> 1;
      h.sine = mi > 0 && (mi & 1) == 0;
      on = true;
    }
    off += w;
  }
  double r = (2.0 * h.l + 1.0) / (4.0 * 3.141592653589793);
  for (int k = h.l - h.M + 1; k <= h.l + h.M; ++k) r /= (double)k;
  if (h.M > 0) r *= 2.0;
  h.N = on ? (float)sqrt(r) : 0.f;
  return h;
}

// Y_lm(u) and the gradient of its polynomial extension at u (on the unit
// sphere its tangential part is the surface gradient).
__device__ __forceinline__ void high_harm(const HighLane& h, float x, float y, float z, float& v, float& gx, float& gy,
                                          float& gz) {
  float c = 1.f, s = 0.f, c1 = 0.f, s1 = 0.f;   // (x + iy)^M and (x + iy)^(M-1)
  for (int k = 0; k < h.M; ++k) {
    c1 = c;
    s1 = s;
    const float cn = c * x - s * y;
    s = s * x + c * y;
    c = cn;
  }
  float q1 = 1.f;   // Q_M^M = (2M - 1)!!
  for (int k = 1; k <= h.M; ++k) q1 *= (float)(2 * k - 1);
  float q0 = 0.f, d0 = 0.f, d1 = 0.f;
  for (int lp = h.M + 1; lp <= h.l; ++lp) {
    const float a = (float)(2 * lp - 1), b = (float)(lp + h.M - 1), inv = 1.0f / (float)(lp - h.M);
    const float qn = (a * z * q1 - b * q0) * inv;
    const float dn = (a * fmaf(z, d1, q1) - b * d0) * inv;
    q0 = q1;
    d0 = d1;
    q1 = qn;
    d1 = dn;
  }
  const float Mf = (float)h.M;
  const float P = h.sine ? s : c;
  const float Px = Mf * (h.sine ? s1 : c1);
  const float Py = Mf * (h.sine ? c1 : -s1);
  const float nq = h.N * q1;
  v = nq * P;
  gx = nq * Px;
  gy = nq * Py;
  gz = h.N * d1 * P;
}

// sum over the 64 lanes (every lane must be active)
__device__ __forceinline__ float wave_total(float v) { return atoms8_sum(grp8_sum(v)); }

// Per-wave LDS record of up to 64 pairs, field-major: rec[f * 64 + slot].
template <int NA, int KA>
struct HighRec {
  static constexpr int DX = 0, DY = 1, DZ = 2, IR = 3, DT = 4, WX = 5, WY = 6, WZ = 7, J = 8, K = 9;
  static constexpr int G = 10, GP = G + NA, F = GP + NA, FP = F + KA, W = FP + KA;
};

template <class C, bool kTri>
struct HighAtom {
  int pa, i, I, st, nA;
  float xi, yi, zi;
  Cell cell;
};

// Stages pairs [k0, k0 + 64) of atom A: lane k0 + lane writes its pair.
template <class C, bool kTri, bool kTangent>
__device__ __forceinline__ void high_stage(const HighArgs& a, const HighAtom<C, kTri>& at, int k0, float* rec,
                                           float fbx, float fby, float fbz, const float (&gw)[6]) {
  constexpr int T = C::T, NA = C::NA, KA = C::KA;
  using R = HighRec<NA, KA>;
  const int lane = threadIdx.x & (kWave - 1);
  const int k = k0 + lane;
  if (k < at.nA) {
    const PairGeom q = pair_geom<kTri>(a.nb.idxA[(size_t)at.i * a.nb.capA + k], a.pos, a.N, at.xi, at.yi, at.zi,
                                       at.cell);
    float f[KA], fp[KA];
    radial_basis_d<KA>(q.r, a.inv_rcA, f, fp);
    const int J = a.type[q.j];
    const float* cJ = a.cA + (size_t)(at.I * T + J) * NA * KA;
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int kk = 0; kk < KA; ++kk) {
        s0 = fmaf(cJ[n * KA + kk], f[kk], s0);
        s1 = fmaf(cJ[n * KA + kk], fp[kk], s1);
      }
      rec[(R::G + n) * kWave + lane] = s0;
      rec[(R::GP + n) * kWave + lane] = s1;
    }
#pragma unroll
    for (int kk = 0; kk < KA; ++kk) {
      rec[(R::F + kk) * kWave + lane] = f[kk];
      rec[(R::FP + kk) * kWave + lane] = fp[kk];
    }
    rec[R::DX * kWave + lane] = q.dx;
    rec[R::DY * kWave + lane] = q.dy;
    rec[R::DZ * kWave + lane] = q.dz;
    rec[R::IR * kWave + lane] = q.inv_r;
    rec[R::J * kWave + lane] = (float)J;
    rec[R::K * kWave + lane] = (float)k;
    if constexpr (kTangent) {
      // t = (fbar_j - fbar_i) + Wbar d, as in the main adjoint
      const float tx = (a.fbar[q.j] - fbx) + gw[0] * q.dx + gw[3] * q.dy;
      const float ty = (a.fbar[a.N + q.j] - fby) + gw[1] * q.dy + gw[4] * q.dz;
      const float tz = (a.fbar[2 * a.N + q.j] - fbz) + gw[2] * q.dz + gw[5] * q.dx;
      const float ux = q.dx * q.inv_r, uy = q.dy * q.inv_r, uz = q.dz * q.inv_r;
      const float dt = ux * tx + uy * ty + uz * tz;
      rec[R::DT * kWave + lane] = dt;
      rec[R::WX * kWave + lane] = (tx - dt * ux) * q.inv_r;
      rec[R::WY * kWave + lane] = (ty - dt * uy) * q.inv_r;
      rec[R::WZ * kWave + lane] = (tz - dt * uz) * q.inv_r;
    }
  }
  lds_lane_exchange();
}

template <class C, bool kTri>
__device__ __forceinline__ bool high_atom(const HighArgs& a, int pa, HighAtom<C, kTri>& at) {
  const int iraw = a.order[pa];
  if (iraw < 0) return false;
  at.pa = pa;
  at.i = iraw;
  at.I = a.type[iraw];
  at.st = a.astruct[iraw];
  at.cell = load_cell<kTri>(a.box, a.tilt, at.st);
  at.xi = a.pos[iraw];
  at.yi = a.pos[a.N + iraw];
  at.zi = a.pos[2 * a.N + iraw];
  at.nA = min(a.nb.cntA[iraw], a.nb.capA);
  return true;
}

// descriptor row of q_nl
template <class C>
__device__ __forceinline__ int high_row(int l, int n) {
  return C::NR + (l - 1) * C::NA + n;
}

template <class C, bool kTri>
__global__ __launch_bounds__(256) void k_high_desc(HighArgs a) {
  constexpr int NA = C::NA, KA = C::KA, L3 = C::L3, YH = C::YH;
  using R = HighRec<NA, KA>;
  __shared__ float recs[4][R::W * kWave];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  float* rec = recs[wv];
  const HighLane h = high_lane(lane, L3);
  const float gw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int u = 0; u < kAPW; ++u) {
    HighAtom<C, kTri> at;
    if (!high_atom<C, kTri>(a, (blockIdx.x * 4 + wv) * kAPW + u, at)) continue;
    float S[NA];
#pragma unroll
    for (int n = 0; n < NA; ++n) S[n] = 0.f;
    for (int k0 = 0; k0 < at.nA; k0 += kWave) {
      high_stage<C, kTri, false>(a, at, k0, rec, 0.f, 0.f, 0.f, gw);
      const int np = min(kWave, at.nA - k0);
      for (int jj = 0; jj < np; ++jj) {
        const float ir = rec[R::IR * kWave + jj];
        float v, gx, gy, gz;
        high_harm(h, rec[R::DX * kWave + jj] * ir, rec[R::DY * kWave + jj] * ir, rec[R::DZ * kWave + jj] * ir, v, gx,
                  gy, gz);
#pragma unroll
        for (int n = 0; n < NA; ++n) S[n] = fmaf(rec[(R::G + n) * kWave + jj], v, S[n]);
      }
      lds_lane_exchange();
    }
    if (lane < YH)
#pragma unroll
      for (int n = 0; n < NA; ++n) a.Sh[((size_t)at.pa * NA + n) * YH + lane] = S[n];
#pragma unroll
    for (int l = 5; l <= L3; ++l)
#pragma unroll
      for (int n = 0; n < NA; ++n) {
        const float q = wave_total(h.l == l ? S[n] * S[n] : 0.f);
        if (lane == 0) a.G[(size_t)high_row<C>(l, n) * a.Npad + at.pa] = q;
      }
  }
}

// E' of this lane's q_nl, channel n
template <class C>
__device__ __forceinline__ float high_ep(const float* __restrict__ rows, int Npad, int pa, const HighLane& h, int n) {
  const float v = rows[(size_t)high_row<C>(h.l, n) * Npad + pa];
  return h.N != 0.f ? v : 0.f;
}

template <class C, bool kTri>
__global__ __launch_bounds__(256) void k_high_force(HighArgs a) {
  constexpr int NA = C::NA, KA = C::KA, L3 = C::L3, YH = C::YH;
  using R = HighRec<NA, KA>;
  __shared__ float recs[4][R::W * kWave];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  float* rec = recs[wv];
  const HighLane h = high_lane(lane, L3);
  const float gw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int u = 0; u < kAPW; ++u) {
    HighAtom<C, kTri> at;
    if (!high_atom<C, kTri>(a, (blockIdx.x * 4 + wv) * kAPW + u, at)) continue;
    // A = dE/dS~ = 2 E'_nl S~
    float A[NA];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      const float s = a.Sh[((size_t)at.pa * NA + n) * YH + (lane < YH ? lane : 0)];
      A[n] = 2.0f * high_ep<C>(a.Ep, a.Npad, at.pa, h, n) * (lane < YH ? s : 0.f);
    }
    float vir[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < at.nA; k0 += kWave) {
      high_stage<C, kTri, false>(a, at, k0, rec, 0.f, 0.f, 0.f, gw);
      const int np = min(kWave, at.nA - k0);
      for (int jj = 0; jj < np; ++jj) {
        const float ir = rec[R::IR * kWave + jj];
        const float dx = rec[R::DX * kWave + jj], dy = rec[R::DY * kWave + jj], dz = rec[R::DZ * kWave + jj];
        const float ux = dx * ir, uy = dy * ir, uz = dz * ir;
        float v, gx, gy, gz;
        high_harm(h, ux, uy, uz, v, gx, gy, gz);
        float su = 0.f, sv = 0.f;
#pragma unroll
        for (int n = 0; n < NA; ++n) {
          su = fmaf(A[n], rec[(R::G + n) * kWave + jj], su);
          sv = fmaf(A[n], rec[(R::GP + n) * kWave + jj], sv);
        }
        // f_ij = sum A (g'_n u Y + g_n grad Y), grad Y = (I - u u^T) grad p / r
        const float vv = wave_total(sv * v);
        const float Gx = wave_total(su * gx), Gy = wave_total(su * gy), Gz = wave_total(su * gz);
        const float rad = ux * Gx + uy * Gy + uz * Gz;
        const float fx = vv * ux + (Gx - rad * ux) * ir;
        const float fy = vv * uy + (Gy - rad * uy) * ir;
        const float fz = vv * uz + (Gz - rad * uz) * ir;
        if (lane == 0) {
          float* fo = a.fA + 3 * ((size_t)at.i * a.nb.capA + (int)rec[R::K * kWave + jj]);
          fo[0] += fx;
          fo[1] += fy;
          fo[2] += fz;
        }
        vir[0] -= fx * dx; vir[1] -= fy * dy; vir[2] -= fz * dz;
        vir[3] -= fx * dy; vir[4] -= fy * dz; vir[5] -= fz * dx;
      }
      lds_lane_exchange();
    }
    if (lane == 0)
#pragma unroll
      for (int c = 0; c < 6; ++c) a.wv[(size_t)c * a.N + at.i] += vir[c];
  }
}

template <class C, bool kTri>
__global__ __launch_bounds__(256) void k_high_tangent(HighArgs a) {
  constexpr int NA = C::NA, KA = C::KA, L3 = C::L3, YH = C::YH;
  using R = HighRec<NA, KA>;
  __shared__ float recs[4][R::W * kWave];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  float* rec = recs[wv];
  const HighLane h = high_lane(lane, L3);
  for (int u = 0; u < kAPW; ++u) {
    HighAtom<C, kTri> at;
    if (!high_atom<C, kTri>(a, (blockIdx.x * 4 + wv) * kAPW + u, at)) continue;
    const float* wb = a.wbar + 6 * at.st;
    const float gw[6] = {wb[0], wb[1], wb[2], wb[3], wb[4], wb[5]};
    const float fbx = a.fbar[at.i], fby = a.fbar[a.N + at.i], fbz = a.fbar[2 * a.N + at.i];
    float Sd[NA];
#pragma unroll
    for (int n = 0; n < NA; ++n) Sd[n] = 0.f;
    for (int k0 = 0; k0 < at.nA; k0 += kWave) {
      high_stage<C, kTri, true>(a, at, k0, rec, fbx, fby, fbz, gw);
      const int np = min(kWave, at.nA - k0);
      for (int jj = 0; jj < np; ++jj) {
        const float ir = rec[R::IR * kWave + jj];
        float v, gx, gy, gz;
        high_harm(h, rec[R::DX * kWave + jj] * ir, rec[R::DY * kWave + jj] * ir, rec[R::DZ * kWave + jj] * ir, v, gx,
                  gy, gz);
        // Sdot = sum_j g'_n (u.t) Y + g_n grad p . (t - (u.t) u) / r
        const float gwt = gx * rec[R::WX * kWave + jj] + gy * rec[R::WY * kWave + jj] + gz * rec[R::WZ * kWave + jj];
        const float vdt = v * rec[R::DT * kWave + jj];
#pragma unroll
        for (int n = 0; n < NA; ++n)
          Sd[n] = fmaf(rec[(R::GP + n) * kWave + jj], vdt, fmaf(rec[(R::G + n) * kWave + jj], gwt, Sd[n]));
      }
      lds_lane_exchange();
    }
    if (lane < YH)
#pragma unroll
      for (int n = 0; n < NA; ++n) a.Sdh[((size_t)at.pa * NA + n) * YH + lane] = Sd[n];
#pragma unroll
    for (int l = 5; l <= L3; ++l)
#pragma unroll
      for (int n = 0; n < NA; ++n) {
        const float s = a.Sh[((size_t)at.pa * NA + n) * YH + (lane < YH ? lane : 0)];
        const float q = wave_total(h.l == l ? 2.0f * s * Sd[n] : 0.f);
        if (lane == 0) a.Gd[(size_t)high_row<C>(l, n) * a.Npad + at.pa] = q;
      }
  }
}

template <class C, bool kTri>
__global__ __launch_bounds__(256) void k_high_coef(HighArgs a) {
  constexpr int T = C::T, NA = C::NA, KA = C::KA, L3 = C::L3, YH = C::YH;
  static_assert(NA * KA <= kWave, "one coefficient slot per lane");
  using R = HighRec<NA, KA>;
  __shared__ float recs[4][R::W * kWave];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int wave = blockIdx.x * 4 + wv;
  float* rec = recs[wv];
  const HighLane h = high_lane(lane, L3);
  const int ne = lane / KA, ke = lane % KA;   // this lane's coefficient slot (n, k)
  float cb[T];
#pragma unroll
  for (int t = 0; t < T; ++t) cb[t] = 0.f;
  for (int u = 0; u < kAPW; ++u) {
    HighAtom<C, kTri> at;
    if (!high_atom<C, kTri>(a, wave * kAPW + u, at)) continue;
    const float* wb = a.wbar + 6 * at.st;
    const float gw[6] = {wb[0], wb[1], wb[2], wb[3], wb[4], wb[5]};
    const float fbx = a.fbar[at.i], fby = a.fbar[a.N + at.i], fbz = a.fbar[2 * a.N + at.i];
    // Sbar = 2 (Gbar S~ - E' Sdot~), A = 2 E' S~ (signs as in the main adjoint)
    float Sb[NA], Av[NA];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      const size_t o = ((size_t)at.pa * NA + n) * YH + (lane < YH ? lane : 0);
      const float s = lane < YH ? a.Sh[o] : 0.f, sd = lane < YH ? a.Sdh[o] : 0.f;
      const float ep = high_ep<C>(a.Ep, a.Npad, at.pa, h, n), gb = high_ep<C>(a.Gb, a.Npad, at.pa, h, n);
      Sb[n] = 2.0f * (gb * s - ep * sd);
      Av[n] = 2.0f * ep * s;
    }
    for (int k0 = 0; k0 < at.nA; k0 += kWave) {
      high_stage<C, kTri, true>(a, at, k0, rec, fbx, fby, fbz, gw);
      const int np = min(kWave, at.nA - k0);
      for (int jj = 0; jj < np; ++jj) {
        const float ir = rec[R::IR * kWave + jj];
        float v, gx, gy, gz;
        high_harm(h, rec[R::DX * kWave + jj] * ir, rec[R::DY * kWave + jj] * ir, rec[R::DZ * kWave + jj] * ir, v, gx,
                  gy, gz);
        const float gwt = gx * rec[R::WX * kWave + jj] + gy * rec[R::WY * kWave + jj] + gz * rec[R::WZ * kWave + jj];
        float Xe = 0.f, Ye = 0.f;
#pragma unroll
        for (int n = 0; n < NA; ++n) {
          const float X = wave_total(fmaf(Sb[n], v, -Av[n] * gwt));
          const float Yv = wave_total(Av[n] * v);
          Xe = ne == n ? X : Xe;
          Ye = ne == n ? Yv : Ye;
        }
        const int J = (int)rec[R::J * kWave + jj];
        const float dt = rec[R::DT * kWave + jj];
        const float fk = rec[(R::F + ke) * kWave + jj], fpk = rec[(R::FP + ke) * kWave + jj];
        const float add = fmaf(Xe, fk, -Ye * dt * fpk);
#pragma unroll
        for (int t = 0; t < T; ++t) cb[t] += (T == 1 || J == t) ? add : 0.f;
      }
      lds_lane_exchange();
    }
  }
  if (lane < NA * KA) {
    float* part = a.part + (size_t)wave * a.PW;
#pragma unroll
    for (int t = 0; t < T; ++t) part[(t * NA + ne) * KA + ke] += cb[t];
  }
}

}  // namespace nep
