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
// One wavefront takes the 8 atoms of an atom group (the species-ordered
// positions of one wavefront of the main kernels) and their angular pairs as
// one stream.  Two mappings follow what each kernel sums over:
//
//  - k_high_desc and k_high_tangent sum over an atom's pairs.  Lane c holds
//    harmonic (l, m) number c of l = 5..L3 (at most 56) for every channel n;
//    chunks of 64 pairs are staged in LDS (direction, g_n, g'_n, tangent, the
//    powers (x + iy)^k) and every lane walks the chunk.
//  - k_high_force and k_high_coef need, per pair, sums over all harmonics.
//    Lane p takes pair p of a chunk and evaluates every harmonic of l = 5..L3
//    at it, so those sums stay in the lane; the per-atom coefficients they
//    contract with sit in LDS, one table per atom slot.
//
#pragma once
#include <type_traits>

#include "nep_device.h"
#include "nep_kernels.h"

namespace nep {

constexpr int kPwStride = 19;   // words per pair in the power table (odd: no bank conflicts)

constexpr double high_cx_sqrt(double x) {
  double r = x > 1.0 ? x : 1.0;   // Newton from above
  for (int it = 0; it < 100; ++it) r = 0.5 * (r + x / r);
  return r;
}

// N_lM^2 = (2l + 1) / (4 pi) (l - M)! / (l + M)!, times 2 for M > 0
constexpr double high_norm2(int l, int M) {
  double v = (2.0 * l + 1.0) / (4.0 * 3.141592653589793);
  for (int k = l - M + 1; k <= l + M; ++k) v /= (double)k;
  return M > 0 ? 2.0 * v : v;
}

struct HighLane {
  int l;
  bool on;
  bool par;                  // Q has odd degree
  float a[5], b[4];          // H(w) = sum a_k w^k, H'(w) = sum b_k w^k
  int iP, iD1, iD2;          // power-table words of P, and of the two derivative factors
  float sD1, sD2;            // dP/dx = sD1 pw[iD1], dP/dy = sD2 pw[iD2]
};

// The 56 harmonics of l = 5..8 in lane order (harmonic c = l^2 - 25 + m,
// M = (m + 1) / 2, sine for even m > 0), built at compile time: N Q_l^M as
// z^par H(z^2) with the coefficients of Q_l^M from the recurrence
//   Q_M^M = (2M-1)!!,  (l-M) Q_l = (2l-1) z Q_{l-1} - (l+M-1) Q_{l-2}.
struct HighLanes {
  HighLane h[56];
};

constexpr HighLanes make_high_lanes() {
  HighLanes t{};
  int c = 0;
  for (int l = 5; l <= 8; ++l)
    for (int mi = 0; mi <= 2 * l; ++mi, ++c) {
      HighLane& h = t.h[c];
      const int M = (mi + 1) >> 1;
      const bool sine = mi > 0 && (mi & 1) == 0;
      double q0[9] = {}, q1[9] = {};
      double df = 1.0;
      for (int k = 1; k <= M; ++k) df *= 2.0 * k - 1.0;
      q1[0] = df;
      for (int lp = M + 1; lp <= l; ++lp) {
        double qn[9] = {};
        for (int p = 0; p < 9; ++p)
          qn[p] = ((2.0 * lp - 1.0) * (p > 0 ? q1[p - 1] : 0.0) - (lp + M - 1.0) * q0[p]) / (double)(lp - M);
        for (int p = 0; p < 9; ++p) {
          q0[p] = q1[p];
          q1[p] = qn[p];
        }
      }
      const double nrm = high_cx_sqrt(high_norm2(l, M));
      h.l = l;
      h.on = true;
      h.par = ((l - M) & 1) != 0;
      for (int k = 0; k < 5; ++k) {
        const int p = 2 * k + (h.par ? 1 : 0);   // Q has degree l <= 8
        h.a[k] = p < 9 ? (float)(nrm * q1[p]) : 0.f;
      }
      for (int k = 0; k < 4; ++k) h.b[k] = (float)(k + 1) * h.a[k + 1];
      // d/dx (x+iy)^M = M (x+iy)^(M-1), d/dy (x+iy)^M = i M (x+iy)^(M-1)
      const int m1 = M > 0 ? M - 1 : 0;
      h.iP = (sine ? 9 : 0) + M;
      h.iD1 = (sine ? 9 : 0) + m1;
      h.iD2 = (sine ? 0 : 9) + m1;
      h.sD1 = (float)M;
      h.sD2 = sine ? (float)M : -(float)M;
    }
  return t;
}
__constant__ const HighLanes kHighLanes = make_high_lanes();

// Harmonic c of l = 5..L3 for lane c; lanes past the last harmonic are off
// (zero polynomial).
__device__ __forceinline__ HighLane high_lane(int c, int L3) {
  const bool on = c < (L3 + 1) * (L3 + 1) - 25;
  HighLane h = kHighLanes.h[on ? c : 0];
  h.on = on;
  if (!on) {
#pragma unroll
    for (int k = 0; k < 5; ++k) h.a[k] = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) h.b[k] = 0.f;
  }
  return h;
}

// Y(u) and the gradient of its polynomial extension at u (its tangential part
// is the surface gradient); pw: the pair's powers (x + iy)^k, k = 0..8, real
// parts then imaginary parts
__device__ __forceinline__ void high_eval(const HighLane& h, float z, const float* pw, float& v, float& gx, float& gy,
                                          float& gz) {
  const float w = z * z;
  float H = fmaf(h.a[4], w, h.a[3]);
  H = fmaf(H, w, h.a[2]);
  H = fmaf(H, w, h.a[1]);
  H = fmaf(H, w, h.a[0]);
  float Hp = fmaf(h.b[3], w, h.b[2]);
  Hp = fmaf(Hp, w, h.b[1]);
  Hp = fmaf(Hp, w, h.b[0]);
  const float zp = h.par ? z : 1.0f;
  const float Q = zp * H;
  const float dQ = fmaf(2.0f * z * zp, Hp, h.par ? H : 0.0f);
  const float P = pw[h.iP];
  v = Q * P;
  gx = Q * h.sD1 * pw[h.iD1];
  gy = Q * h.sD2 * pw[h.iD2];
  gz = dQ * P;
}

// Sums of 8 values over the 64 lanes, scattered: on return the lanes with
// (lane & 7) == v hold the total of value v.  A butterfly over lane bits 0,
// 1 and 2 halves the values a lane carries at each step, so the 8 sums take
// 7 lane exchanges before the sum over the 8 groups instead of 24.
__device__ __forceinline__ float wave_scatter_sum8(const float (&x)[8]) {
  const int lane = threadIdx.x & (kWave - 1);
  const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
  float y[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) {   // y[w]: value 2w + b0
    const float send = b0 ? x[2 * w] : x[2 * w + 1];
    y[w] = (b0 ? x[2 * w + 1] : x[2 * w]) + dpp<kDppXor1>(send);
  }
  float z[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {   // z[u]: value 4u + 2 b1 + b0
    const float send = b1 ? y[2 * u] : y[2 * u + 1];
    z[u] = (b1 ? y[2 * u + 1] : y[2 * u]) + dpp<kDppXor2>(send);
  }
  const float send = b2 ? z[0] : z[1];   // value lane & 7 over the 8-lane group
  return atoms8_sum((b2 ? z[1] : z[0]) + xor4_val(send));
}

// Per-wave LDS record of up to 64 pairs, pair-major: pair jj's W words at
// rec[jj W], read by every lane at once (one address, so 16-byte reads serve
// four fields each).  kTan: w_x, w_y, w_z, u.t first, then g_n and g'_n;
// otherwise g_n only.  The pair's direction cosine z sits in word kPwZ of its
// power-table row.
template <int NA, bool kTan>
struct HighRec {
  static constexpr int WX = 0, WY = 1, WZ = 2, DT = 3, G = kTan ? 4 : 0, GP = G + NA;
  static constexpr int W = kTan ? GP + NA : G + NA;
};
constexpr int kPwZ = 18;

// The 8 atom slots of a wavefront and their pair counts.
struct HighGroup {
  int pa0, total;
  int cum[kAPW + 1];   // pairs before slot u
  unsigned occ;        // bit u: slot u holds an atom
};

__device__ __forceinline__ HighGroup high_group(const HighArgs& a, int pa0) {
  HighGroup g;
  g.pa0 = pa0;
  g.cum[0] = 0;
  g.occ = 0;
#pragma unroll
  for (int u = 0; u < kAPW; ++u) {
    const int i = a.order[pa0 + u];
    const int n = i >= 0 ? min(a.nb.cntA[i], a.nb.capA) : 0;
    g.cum[u + 1] = g.cum[u] + n;
    g.occ |= i >= 0 ? 1u << u : 0u;
  }
  g.total = g.cum[kAPW];
  return g;
}

// Stages pairs [c0, c0 + 64) of the group's stream, one per lane.
template <class C, bool kTri, bool kTan>
__device__ __forceinline__ void high_stage(const HighArgs& a, const HighGroup& gr, int c0, float* rec, float* pw) {
  constexpr int T = C::T, NA = C::NA, KA = C::KA;
  using R = HighRec<NA, kTan>;
  const int lane = threadIdx.x & (kWave - 1);
  const int gidx = c0 + lane;
  if (gidx < gr.total) {
    int u = 0, base = 0;
#pragma unroll
    for (int v = 1; v < kAPW; ++v) {
      const bool past = gidx >= gr.cum[v];
      u = past ? v : u;
      base = past ? gr.cum[v] : base;
    }
    const int k = gidx - base;
    const int i = a.order[gr.pa0 + u];
    const int I = a.type[i], st = a.astruct[i];
    const Cell cell = load_cell<kTri>(a.box, a.tilt, st);
    const size_t off = (size_t)i * a.nb.capA + k;
    const PairGeom q = pair_geom<kTri>(a.nb.idxA[off], a.pos, a.N, a.pos[i], a.pos[a.N + i], a.pos[2 * a.N + i],
                                       cell);
    float f[KA], fp[KA];
    radial_basis_d<KA>(q.r, a.inv_rcA, f, fp);
    const int J = a.type[q.j];
    const float* cJ = a.cA + (size_t)(I * T + J) * NA * KA;
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int kk = 0; kk < KA; ++kk) {
        s0 = fmaf(cJ[n * KA + kk], f[kk], s0);
        s1 = fmaf(cJ[n * KA + kk], fp[kk], s1);
      }
      rec[lane * R::W + R::G + n] = s0;
      if constexpr (kTan) rec[lane * R::W + R::GP + n] = s1;
    }
    const float ux = q.dx * q.inv_r, uy = q.dy * q.inv_r, uz = q.dz * q.inv_r;
    float c = 1.f, s = 0.f;
    float* p = pw + lane * kPwStride;
    p[kPwZ] = uz;
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      p[m] = c;
      p[9 + m] = s;
      const float cn = c * ux - s * uy;
      s = fmaf(s, ux, c * uy);
      c = cn;
    }
    if constexpr (kTan) {
      // t = (fbar_j - fbar_i) + Wbar d, as in the main adjoint
      const float* wb = a.wbar + 6 * st;
      const float tx = (a.fbar[q.j] - a.fbar[i]) + wb[0] * q.dx + wb[3] * q.dy;
      const float ty = (a.fbar[a.N + q.j] - a.fbar[a.N + i]) + wb[1] * q.dy + wb[4] * q.dz;
      const float tz = (a.fbar[2 * a.N + q.j] - a.fbar[2 * a.N + i]) + wb[2] * q.dz + wb[5] * q.dx;
      const float dt = ux * tx + uy * ty + uz * tz;
      rec[lane * R::W + R::DT] = dt;
      rec[lane * R::W + R::WX] = (tx - dt * ux) * q.inv_r;
      rec[lane * R::W + R::WY] = (ty - dt * uy) * q.inv_r;
      rec[lane * R::W + R::WZ] = (tz - dt * uz) * q.inv_r;
    }
  }
  lds_lane_exchange();
}

// Walks the group's pair stream: start(u) before the first pair of slot u,
// pair(u, jj) for each staged pair jj of slot u, finish(u) after its last pair
// (also for slots without pairs).  Each slot's pairs in a chunk are a range
// known from the pair counts, so no per-pair test decides where a slot ends,
// and the loop over a range is unrolled to keep several pairs' LDS reads in
// flight.  A slot belongs to the chunk holding its first pair (start) and
// the one holding its last (finish); an empty slot to the chunk holding its
// position in the stream, or the last chunk.
template <class C, bool kTri, bool kTan, class Start, class Pair, class Finish>
__device__ __forceinline__ void high_walk(const HighArgs& a, const HighGroup& gr, float* rec, float* pw,
                                          Start&& start, Pair&& pair, Finish&& finish) {
  const int total = gr.total;
  for (int c0 = 0; c0 < (total > 0 ? total : 1); c0 += kWave) {
    high_stage<C, kTri, kTan>(a, gr, c0, rec, pw);
    const int c1 = min(c0 + kWave, total);
    const bool last = c1 == total;
#pragma unroll
    for (int u = 0; u < kAPW; ++u) {
      const int b = gr.cum[u], e = gr.cum[u + 1];
      const bool starts = b >= c0 && (b < c1 || (b == e && last));
      const bool ends = b == e ? starts : e > c0 && e <= c1;
      if (starts) start(u);
      const int j1 = min(e, c1) - c0;
#pragma unroll 4
      for (int jj = max(b, c0) - c0; jj < j1; ++jj) pair(u, jj);
      if (ends) finish(u);
    }
    lds_lane_exchange();
  }
}

// descriptor row of q_nl
template <class C>
__device__ __forceinline__ int high_row(int l, int n) {
  return C::NR + (l - 1) * C::NA + n;
}

// a descriptor-row value of this lane's degree, channel n
template <class C>
__device__ __forceinline__ float high_rowval(const float* __restrict__ rows, int Npad, int pa, const HighLane& h,
                                            int n) {
  const float v = rows[(size_t)high_row<C>(h.l, n) * Npad + pa];
  return h.on ? v : 0.f;
}

// Stores the wave totals of the per-lane values vals[(l - 5) NA + n] to the
// descriptor rows of (l, n), l = 5..L3 (row NR + (l - 1) NA + n), eight
// values per scattered sum.
template <class C>
__device__ __forceinline__ void high_rows_store(const float (&vals)[(C::L3 - 4) * C::NA], float* rows, int Npad,
                                                int pa) {
  constexpr int NV = (C::L3 - 4) * C::NA;
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int g0 = 0; g0 < NV; g0 += 8) {
    float xs[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) xs[v] = g0 + v < NV ? vals[g0 + v < NV ? g0 + v : 0] : 0.f;
    const float t = wave_scatter_sum8(xs);
    if (lane < 8 && g0 + lane < NV) rows[(size_t)(C::NR + 4 * C::NA + g0 + lane) * Npad + pa] = t;
  }
}

// word of S~_nc (and Sdot~_nc) of atom position pa: [Npad][YH][NA], so the
// rows of a group's 8 slots are one contiguous block in the order of the
// pair-per-lane kernels' LDS tables
template <class C>
__device__ __forceinline__ size_t high_slot(int pa, int n, int lane) {
  return ((size_t)pa * C::YH + (lane < C::YH ? lane : 0)) * C::NA + n;
}

#define NEP_HIGH_PROLOGUE(TAN)                                           \
  constexpr int NA = C::NA, L3 = C::L3, YH = C::YH;                      \
  using R = HighRec<NA, TAN>;                                            \
  __shared__ __align__(16) float recs[4][R::W * kWave];                  \
  __shared__ float pws[4][kWave * kPwStride];                            \
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;  \
  const int wave = blockIdx.x * 4 + wv;                                  \
  float* rec = recs[wv];                                                 \
  float* pw = pws[wv];                                                   \
  const HighLane h = high_lane(lane, L3);                                \
  const HighGroup gr = high_group(a, wave * kAPW);                       \
  (void)YH;

template <class C, bool kTri>
__global__ __launch_bounds__(256) void k_high_desc(HighArgs a) {
  NEP_HIGH_PROLOGUE(false)
  float S[NA];
  auto start = [&](int) {
#pragma unroll
    for (int n = 0; n < NA; ++n) S[n] = 0.f;
  };
  auto pair = [&](int, int jj) {
    float v, gx, gy, gz;
    const float* pj = pw + jj * kPwStride;
    const float* rj = rec + jj * R::W;
    high_eval(h, pj[kPwZ], pj, v, gx, gy, gz);
#pragma unroll
    for (int n = 0; n < NA; ++n) S[n] = fmaf(rj[R::G + n], v, S[n]);
  };
  auto finish = [&](int u) {
    const int pa = gr.pa0 + u;
    if (!((gr.occ >> u) & 1u)) return;
    if (lane < YH)
#pragma unroll
      for (int n = 0; n < NA; ++n) a.Sh[high_slot<C>(pa, n, lane)] = S[n];
    float q[(L3 - 4) * NA];
#pragma unroll
    for (int l = 5; l <= L3; ++l)
#pragma unroll
      for (int n = 0; n < NA; ++n) q[(l - 5) * NA + n] = h.l == l ? S[n] * S[n] : 0.f;
    high_rows_store<C>(q, a.G, a.Npad, pa);
  };
  high_walk<C, kTri, false>(a, gr, rec, pw, start, pair, finish);
}

template <class C, bool kTri>
__global__ __launch_bounds__(256) void k_high_tangent(HighArgs a) {
  NEP_HIGH_PROLOGUE(true)
  float Sd[NA];
  auto start = [&](int) {
#pragma unroll
    for (int n = 0; n < NA; ++n) Sd[n] = 0.f;
  };
  auto pair = [&](int, int jj) {
    float v, gx, gy, gz;
    const float* pj = pw + jj * kPwStride;
    const float* rj = rec + jj * R::W;
    high_eval(h, pj[kPwZ], pj, v, gx, gy, gz);
    // Sdot = sum_j g'_n (u.t) Y + g_n grad p . (t - (u.t) u) / r
    const float gwt = gx * rj[R::WX] + gy * rj[R::WY] + gz * rj[R::WZ];
    const float vdt = v * rj[R::DT];
#pragma unroll
    for (int n = 0; n < NA; ++n)
      Sd[n] = fmaf(rj[R::GP + n], vdt, fmaf(rj[R::G + n], gwt, Sd[n]));
  };
  auto finish = [&](int u) {
    const int pa = gr.pa0 + u;
    if (!((gr.occ >> u) & 1u)) return;
    if (lane < YH)
#pragma unroll
      for (int n = 0; n < NA; ++n) a.Sdh[high_slot<C>(pa, n, lane)] = Sd[n];
    float q[(L3 - 4) * NA];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      const float s = lane < YH ? a.Sh[high_slot<C>(pa, n, lane)] : 0.f;
#pragma unroll
      for (int l = 5; l <= L3; ++l) q[(l - 5) * NA + n] = h.l == l ? 2.0f * s * Sd[n] : 0.f;
    }
    high_rows_store<C>(q, a.Gd, a.Npad, pa);
  };
  high_walk<C, kTri, true>(a, gr, rec, pw, start, pair, finish);
}

#undef NEP_HIGH_PROLOGUE

// ===================================================== one pair per lane
// For each order M, Qhat_l^M = N_lM Q_l^M (the Q_l^M and N_lM of high_lane)
// follows from the recurrence in l, with Qhat_{M-1}^M = 0:
//   Qhat_M^M = N_MM (2M - 1)!!,
//   Qhat_l^M = A_lM z Qhat_{l-1}^M - B_lM Qhat_{l-2}^M,
//   A_lM = (2l - 1) / (l - M) N_lM / N_{l-1,M},
//   B_lM = (l + M - 1) / (l - M) N_lM / N_{l-2,M},
// and dQhat_l^M / dz from the derivative of the same recurrence.  Harmonic
// (l, M) is then Y = Qhat Re (x + iy)^M (m = 2M - 1, or m = 0) and
// Y = Qhat Im (x + iy)^M (m = 2M), number l^2 - 25 + m as in high_lane.

struct HighTab {
  float q0[9];     // Qhat_M^M
  float A[9][9];   // [l][M]
  float B[9][9];
};

constexpr HighTab make_high_tab() {
  HighTab t{};
  for (int M = 0; M <= 8; ++M) {
    double df = 1.0;
    for (int k = 1; k <= M; ++k) df *= 2.0 * k - 1.0;
    t.q0[M] = (float)(high_cx_sqrt(high_norm2(M, M)) * df);
    for (int l = M + 1; l <= 8; ++l) {
      t.A[l][M] = (float)((2.0 * l - 1.0) / (l - M) * high_cx_sqrt(high_norm2(l, M) / high_norm2(l - 1, M)));
      t.B[l][M] = l >= M + 2
                      ? (float)((l + M - 1.0) / (l - M) * high_cx_sqrt(high_norm2(l, M) / high_norm2(l - 2, M)))
                      : 0.f;
    }
  }
  return t;
}
constexpr HighTab kHighTab = make_high_tab();

// Calls f(integral_constant<M>, q, dq) for M = 0..L3 with q[l - 5] = Qhat_l^M(z)
// and dq[l - 5] = its z-derivative for l = max(M, 5)..L3.
template <int L3, int M = 0, class F>
__device__ __forceinline__ void high_orders(float z, F&& f) {
  if constexpr (M <= L3) {
    float q[L3 - 4] = {}, dq[L3 - 4] = {};
    float q2 = 0.f, q1 = kHighTab.q0[M], d2 = 0.f, d1 = 0.f;
    if constexpr (M >= 5) q[M - 5] = q1;
#pragma unroll
    for (int l = M + 1; l <= L3; ++l) {
      const float A = kHighTab.A[l][M], B = kHighTab.B[l][M];
      const float qn = fmaf(A * z, q1, -B * q2);
      const float dn = fmaf(A, fmaf(z, d1, q1), -B * d2);
      q2 = q1;
      q1 = qn;
      d2 = d1;
      d1 = dn;
      if (l >= 5) {
        q[l - 5] = qn;
        dq[l - 5] = dn;
      }
    }
    f(std::integral_constant<int, M>{}, q, dq);
    high_orders<L3, M + 1>(z, f);
  }
}

// Harmonic numbers in the order the pair-per-lane kernels visit them (order
// M = 0..L3, within it l = max(M, 5)..L3, cosine then sine) and where each
// order starts.
template <int L3>
struct HighVisit {
  int cc[(L3 + 1) * (L3 + 1) - 25];
  int base[L3 + 2];
};

template <int L3>
constexpr HighVisit<L3> make_high_visit() {
  HighVisit<L3> v{};
  int k = 0;
  for (int M = 0; M <= L3; ++M) {
    v.base[M] = k;
    for (int l = M > 5 ? M : 5; l <= L3; ++l) {
      const int c = l * l - 25 + (M > 0 ? 2 * M - 1 : 0);
      v.cc[k++] = c;
      if (M > 0) v.cc[k++] = c + 1;
    }
  }
  v.base[L3 + 1] = k;
  return v;
}

// W words of an LDS table row (16-byte loads when W is a multiple of 4)
template <int W>
struct HighRow {
  float v[W];
};

template <int W>
__device__ __forceinline__ HighRow<W> high_row_load(const float* p) {
  HighRow<W> r;
  if constexpr (W % 4 == 0) {
#pragma unroll
    for (int e = 0; e < W; e += 4) {
      const float4 c = *reinterpret_cast<const float4*>(p + e);
      r.v[e] = c.x;
      r.v[e + 1] = c.y;
      r.v[e + 2] = c.z;
      r.v[e + 3] = c.w;
    }
  } else {
#pragma unroll
    for (int e = 0; e < W; ++e) r.v[e] = p[e];
  }
  return r;
}

// Visits every harmonic of l = 5..L3 at direction cosine z in HighVisit
// order: start(Mc) before order M, f(Mc, Qhat, dQhat, sine, row) per harmonic
// with its table row (W words at row0 + c W), fin(Mc) after order M.  The
// rows are loaded D harmonics ahead of their use, so the LDS latency is
// covered by the arithmetic of the harmonics in between.
template <int L3, int W, int D, class Start, class F, class Fin>
__device__ __forceinline__ void high_visit(const float* row0, float z, Start&& start, F&& f, Fin&& fin) {
  constexpr int YH = (L3 + 1) * (L3 + 1) - 25;
  constexpr HighVisit<L3> hv = make_high_visit<L3>();
  HighRow<W> pf[D];
#pragma unroll
  for (int d = 0; d < D; ++d) pf[d] = high_row_load<W>(row0 + hv.cc[d] * W);
  high_orders<L3>(z, [&](auto Mc, const float (&q)[L3 - 4], const float (&dq)[L3 - 4]) {
    constexpr int M = decltype(Mc)::value;
    constexpr int l0 = M > 5 ? M : 5, NS = M > 0 ? 2 : 1;
    start(Mc);
#pragma unroll
    for (int l = l0; l <= L3; ++l) {
#pragma unroll
      for (int sn = 0; sn < NS; ++sn) {
        const int k = hv.base[M] + NS * (l - l0) + sn;
        const HighRow<W> cur = pf[k % D];
        if (k + D < YH) pf[k % D] = high_row_load<W>(row0 + hv.cc[k + D < YH ? k + D : 0] * W);
        f(Mc, q[l - 5], dq[l - 5], sn, cur);
      }
    }
    fin(Mc);
  });
}

// degree l of harmonic number c (c in [l^2 - 25, (l + 1)^2 - 25))
__device__ __forceinline__ int high_deg(int c) { return c < 11 ? 5 : c < 24 ? 6 : c < 39 ? 7 : 8; }

// Words per atom slot of a coefficient table of w words: a multiple of 64
// plus 8, so the 8 slots start in 8 different groups of banks.
constexpr int high_table_stride(int w) { return (w + 63) / 64 * 64 + 8; }

// Pair p of the group's stream: its atom slot u, list entry k, atom i,
// neighbor j, geometry and the powers (x + iy)^k = R[k] + i I[k] of its
// direction.
struct HighPair {
  int u, k, i, j, st;
  float dx, dy, dz, r, ir, ux, uy, uz;
  float R[9], I[9];
};

template <bool kTri>
__device__ __forceinline__ HighPair high_pair(const HighArgs& a, const HighGroup& gr, int p) {
  HighPair g;
  int u = 0, base = 0;
#pragma unroll
  for (int v = 1; v < kAPW; ++v) {
    const bool past = p >= gr.cum[v];
    u = past ? v : u;
    base = past ? gr.cum[v] : base;
  }
  g.u = u;
  g.k = p - base;
  g.i = a.order[gr.pa0 + u];
  g.st = a.astruct[g.i];
  const Cell cell = load_cell<kTri>(a.box, a.tilt, g.st);
  const PairGeom q = pair_geom<kTri>(a.nb.idxA[(size_t)g.i * a.nb.capA + g.k], a.pos, a.N, a.pos[g.i],
                                     a.pos[a.N + g.i], a.pos[2 * a.N + g.i], cell);
  g.j = q.j;
  g.dx = q.dx;
  g.dy = q.dy;
  g.dz = q.dz;
  g.r = q.r;
  g.ir = q.inv_r;
  g.ux = q.dx * q.inv_r;
  g.uy = q.dy * q.inv_r;
  g.uz = q.dz * q.inv_r;
  float c = 1.f, s = 0.f;
#pragma unroll
  for (int m = 0; m < 9; ++m) {
    g.R[m] = c;
    g.I[m] = s;
    const float cn = c * g.ux - s * g.uy;
    s = fmaf(s, g.ux, c * g.uy);
    c = cn;
  }
  return g;
}

// LDS words of the per-slot factors 2 E'_nl (and 2 Gbar_nl) staged with a
// coefficient table
template <class C, bool kSbar>
constexpr int high_factor_words() {
  return (kSbar ? 2 : 1) * kAPW * (C::L3 - 4) * C::NA;
}

// Coefficient table of the group's 8 atom slots for the pair-per-lane
// kernels: the row of harmonic c of slot u at tab[u AS + c W], with
// A_nc = 2 E'_nl S~_nc in words OA + n and, with kSbar, Sbar_nc =
// 2 (Gbar_nl S~_nc - E'_nl Sdot~_nc) in words n (W = 2 NA, OA = NA; without,
// W = NA, OA = 0).  The slots' S~ (and Sdot~) rows are one contiguous block,
// read 16 bytes per lane; the factors of each (slot, l, n) go through `fac`
// (high_factor_words words of LDS) first.  Rows of empty slots are left as
// read: no pair refers to them.
template <class C, bool kSbar>
__device__ __forceinline__ void high_table_stage(const HighArgs& a, const HighGroup& gr, float* tab, int AS,
                                                 float* fac) {
  constexpr int NA = C::NA, YH = C::YH, NL = C::L3 - 4, NF = kAPW * NL * NA;
  constexpr int W = kSbar ? 2 * NA : NA, OA = kSbar ? NA : 0;
  static_assert(NA % 4 == 0, "rows are staged 4 channels at a time");
  constexpr int Q = NA / 4, NQ = kAPW * YH * Q;   // 16-byte units of the block
  const int lane = threadIdx.x & (kWave - 1);
  for (int e = lane; e < NF; e += kWave) {
    const int u = e / (NL * NA), l = 5 + (e / NA) % NL, n = e % NA;
    const size_t ro = (size_t)high_row<C>(l, n) * a.Npad + gr.pa0 + u;
    fac[e] = 2.0f * a.Ep[ro];
    if constexpr (kSbar) fac[NF + e] = 2.0f * a.Gb[ro];
  }
  lds_lane_exchange();
  const float4* S4 = reinterpret_cast<const float4*>(a.Sh + (size_t)gr.pa0 * YH * NA);
  const float4* D4 = reinterpret_cast<const float4*>(a.Sdh + (size_t)gr.pa0 * YH * NA);
#pragma unroll
  for (int e0 = 0; e0 < NQ; e0 += kWave) {
    const int e = e0 + lane;
    if (e0 + kWave <= NQ || e < NQ) {
      const int u = e / (YH * Q), c = (e / Q) % YH, n0 = (e % Q) * 4;
      const float4 sv = S4[e];
      const int fo = (u * NL + high_deg(c) - 5) * NA + n0;
      const float4 ep = *reinterpret_cast<const float4*>(fac + fo);
      float* row = tab + u * AS + c * W + n0;
      *reinterpret_cast<float4*>(row + OA) = make_float4(ep.x * sv.x, ep.y * sv.y, ep.z * sv.z, ep.w * sv.w);
      if constexpr (kSbar) {
        const float4 dv = D4[e];
        const float4 gb = *reinterpret_cast<const float4*>(fac + NF + fo);
        *reinterpret_cast<float4*>(row) =
            make_float4(fmaf(gb.x, sv.x, -ep.x * dv.x), fmaf(gb.y, sv.y, -ep.y * dv.y),
                        fmaf(gb.z, sv.z, -ep.z * dv.z), fmaf(gb.w, sv.w, -ep.w * dv.w));
      }
    }
  }
}

// Pair forces and virial of the q_nl of l = 5..L3.  With A_nlm = dE/dS~_nlm
// = 2 E'_nl S~_nlm of the pair's atom, the pair's share of the force is
//   f_ij = sum_nlm A_nlm (g'_n Y u + g_n (I - u u^T) grad p_lm / r)
// (grad p: gradient of the harmonic's polynomial).  Per order M the sums
// over l of sum_n A g'_n Qhat, sum_n A g_n Qhat and sum_n A g_n dQhat are
// formed first, so the powers (x + iy)^M and their derivatives enter once per
// order.  The per-atom virial sums the pairs of each slot in list order.
template <class C, bool kTri>
__global__ __launch_bounds__(256) void k_high_force(HighArgs a) {
  constexpr int T = C::T, NA = C::NA, KA = C::KA, L3 = C::L3, YH = C::YH;
  constexpr int AS = high_table_stride(YH * NA);
  static_assert(high_factor_words<C, false>() <= 6 * kWave, "the factors are staged in the virial words");
  __shared__ __align__(16) float tabs[4][kAPW * AS];
  __shared__ __align__(16) float vrs[4][6 * kWave];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int wave = blockIdx.x * 4 + wv;
  float* tab = tabs[wv];
  float* vr = vrs[wv];
  const HighGroup gr = high_group(a, wave * kAPW);
  high_table_stage<C, false>(a, gr, tab, AS, vr);
  lds_lane_exchange();
  float vir[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};   // lanes u < 8: atom slot u
  int lo = 0, hi = 0;                              // slot lane's pairs in the stream
#pragma unroll
  for (int v = 0; v < kAPW; ++v) {
    lo = lane == v ? gr.cum[v] : lo;
    hi = lane == v ? gr.cum[v + 1] : hi;
  }
  for (int c0 = 0; c0 < gr.total; c0 += kWave) {
    const int p = c0 + lane;
    float fx = 0.f, fy = 0.f, fz = 0.f, dx = 0.f, dy = 0.f, dz = 0.f;
    if (p < gr.total) {
      const HighPair g = high_pair<kTri>(a, gr, p);
      float f[KA], fp[KA];
      radial_basis_d<KA>(g.r, a.inv_rcA, f, fp);
      const float* cJ = a.cA + (size_t)(a.type[g.i] * T + a.type[g.j]) * NA * KA;
      float gn[NA], gpn[NA];
#pragma unroll
      for (int n = 0; n < NA; ++n) {
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int kk = 0; kk < KA; ++kk) {
          s0 = fmaf(cJ[n * KA + kk], f[kk], s0);
          s1 = fmaf(cJ[n * KA + kk], fp[kk], s1);
        }
        gn[n] = s0;
        gpn[n] = s1;
      }
      float vv = 0.f, Gx = 0.f, Gy = 0.f, Gz = 0.f;
      float V[2], Tq[2], Z[2];   // per order: sums over l of sum_n A g'_n Qhat, A g_n Qhat, A g_n dQhat
      high_visit<L3, NA, 4>(
          tab + g.u * AS, g.uz,
          [&](auto) {
            V[0] = V[1] = Tq[0] = Tq[1] = Z[0] = Z[1] = 0.f;
          },
          [&](auto, float q, float dq, int sn, const HighRow<NA>& row) {
            float su = 0.f, sv = 0.f;
#pragma unroll
            for (int n = 0; n < NA; ++n) {
              su = fmaf(row.v[n], gn[n], su);
              sv = fmaf(row.v[n], gpn[n], sv);
            }
            V[sn] = fmaf(sv, q, V[sn]);
            Tq[sn] = fmaf(su, q, Tq[sn]);
            Z[sn] = fmaf(su, dq, Z[sn]);
          },
          [&](auto Mc) {
            // Y = Qhat P, grad p = (Qhat dP/dx, Qhat dP/dy, dQhat P) with
            // d/dx (x + iy)^M = M (x + iy)^(M-1), d/dy (x + iy)^M = i M (x + iy)^(M-1)
            constexpr int M = decltype(Mc)::value;
            vv = fmaf(V[0], g.R[M], vv);
            Gz = fmaf(Z[0], g.R[M], Gz);
            if constexpr (M > 0) {
              vv = fmaf(V[1], g.I[M], vv);
              Gz = fmaf(Z[1], g.I[M], Gz);
              Gx = fmaf((float)M, fmaf(Tq[0], g.R[M - 1], Tq[1] * g.I[M - 1]), Gx);
              Gy = fmaf((float)M, fmaf(Tq[1], g.R[M - 1], -Tq[0] * g.I[M - 1]), Gy);
            }
          });
      const float rad = g.ux * Gx + g.uy * Gy + g.uz * Gz;
      fx = vv * g.ux + (Gx - rad * g.ux) * g.ir;
      fy = vv * g.uy + (Gy - rad * g.uy) * g.ir;
      fz = vv * g.uz + (Gz - rad * g.uz) * g.ir;
      float* fo = a.fA + 3 * ((size_t)g.i * a.nb.capA + g.k);
      fo[0] += fx;
      fo[1] += fy;
      fo[2] += fz;
      dx = g.dx;
      dy = g.dy;
      dz = g.dz;
    }
    vr[0 * kWave + lane] = fx;
    vr[1 * kWave + lane] = fy;
    vr[2 * kWave + lane] = fz;
    vr[3 * kWave + lane] = dx;
    vr[4 * kWave + lane] = dy;
    vr[5 * kWave + lane] = dz;
    lds_lane_exchange();
    if (lane < kAPW) {
      const int j1 = min(hi - c0, kWave);
      for (int jj = max(lo - c0, 0); jj < j1; ++jj) {
        const float px = vr[jj], py = vr[kWave + jj], pz = vr[2 * kWave + jj];
        const float qx = vr[3 * kWave + jj], qy = vr[4 * kWave + jj], qz = vr[5 * kWave + jj];
        vir[0] -= px * qx;
        vir[1] -= py * qy;
        vir[2] -= pz * qz;
        vir[3] -= px * qy;
        vir[4] -= py * qz;
        vir[5] -= pz * qx;
      }
    }
    lds_lane_exchange();
  }
  if (lane < kAPW) {
    const int i = a.order[gr.pa0 + lane];
    if (i >= 0)
#pragma unroll
      for (int c = 0; c < 6; ++c) a.wv[(size_t)c * a.N + i] += vir[c];
  }
}

// LDS of k_high_coef: per atom slot the table (Sbar_nc, A_nc) of every
// harmonic c; per chunk the record of each pair's X_n, Y_n (u.t), f_k, f'_k
// and neighbor species, field stride 65 words so the lanes of the second
// phase, which read different fields of one pair, hit different banks.  The
// record reuses the table's words (the table is staged again for each chunk
// of 64 pairs), which keeps a wavefront's LDS to the table alone.
template <class C>
struct HighCoefShape {
  static constexpr int NA = C::NA, KA = C::KA;
  static constexpr int AS = high_table_stride(C::YH * 2 * NA);
  static constexpr int RS = kWave + 1;
  static constexpr int RX = 0, RY = NA, RF = 2 * NA, RFP = 2 * NA + KA, RJ = 2 * NA + 2 * KA, NF = RJ + 1;
  static constexpr int TW = kAPW * AS + high_factor_words<C, true>();   // table and its factors
  static constexpr int WORDS = TW > NF * RS ? TW : NF * RS;
  // second phase: lane (slot s = (n, k), phase ph) sums pairs jj = ph, ph + NPH, ...
  static constexpr int NS = NA * KA;
  static constexpr int NPH = NS <= kWave / 2 ? 2 : 1;
  static constexpr int SPL = (NS + kWave / NPH - 1) / (kWave / NPH);
};

// The c^A gradient of the q_nl of l = 5..L3.  With Sbar_nlm = 2 (Gbar_nl S~ -
// E'_nl Sdot~) and A_nlm = 2 E'_nl S~ of the pair's atom (signs as in the main
// adjoint), each pair gives
//   X_n = sum_lm (Sbar_nlm Y - A_nlm grad p . w),  Y_n = sum_lm A_nlm Y,
//   dL/dc_nk^{IJ} += X_n f_k - Y_n (u.t) f'_k,
// with t the pair's tangent and w = (t - (u.t) u) / r.  Phase one: lane p
// forms X_n, Y_n of pair p.  Phase two: lane (n, k) adds up the chunk's
// pairs for its coefficient slots, one register per neighbor species J.
// One wavefront per block: the LDS per wavefront is the occupancy limit.
// With n_ang <= 4 the table leaves room for about 10 wavefronts per CU, and
// the register budget is set to match (3 per SIMD); the wider classes' table
// allows fewer, and they keep the default budget.
template <class C, bool kTri>
__global__ __launch_bounds__(kWave, C::NA <= 4 ? 3 : 1) void k_high_coef(HighArgs a) {
  using S = HighCoefShape<C>;
  constexpr int T = C::T, NA = C::NA, KA = C::KA, L3 = C::L3, YH = C::YH, AS = S::AS, RS = S::RS;
  __shared__ __align__(16) float lds[S::WORDS];
  float* tab = lds;
  float* rec = lds;
  const int lane = threadIdx.x;
  const int wave = blockIdx.x;
  const HighGroup gr = high_group(a, wave * kAPW);
  const int ph = S::NPH == 2 ? lane / (kWave / 2) : 0;
  const int s0 = S::NPH == 2 ? lane % (kWave / 2) : lane;
  int sn[S::SPL], sk[S::SPL];
  float cb[S::SPL][T];
#pragma unroll
  for (int r = 0; r < S::SPL; ++r) {
    const int s = s0 + r * (kWave / S::NPH);
    const int sc = s < S::NS ? s : 0;
    sn[r] = sc / KA;
    sk[r] = sc % KA;
#pragma unroll
    for (int t = 0; t < T; ++t) cb[r][t] = 0.f;
  }
  for (int c0 = 0; c0 < gr.total; c0 += kWave) {
    const int p = c0 + lane;
    high_table_stage<C, true>(a, gr, tab, AS, tab + kAPW * AS);
    lds_lane_exchange();
    const HighPair g = high_pair<kTri>(a, gr, p < gr.total ? p : 0);   // lanes past the chunk: pair 0, unused
    float f[KA], fp[KA];
    radial_basis_d<KA>(g.r, a.inv_rcA, f, fp);
    // t = (fbar_j - fbar_i) + Wbar d, as in the main adjoint
    const float* wb = a.wbar + 6 * g.st;
    const float tx = (a.fbar[g.j] - a.fbar[g.i]) + wb[0] * g.dx + wb[3] * g.dy;
    const float ty = (a.fbar[a.N + g.j] - a.fbar[a.N + g.i]) + wb[1] * g.dy + wb[4] * g.dz;
    const float tz = (a.fbar[2 * a.N + g.j] - a.fbar[2 * a.N + g.i]) + wb[2] * g.dz + wb[5] * g.dx;
    const float dt = g.ux * tx + g.uy * ty + g.uz * tz;
    const float wx = (tx - dt * g.ux) * g.ir, wy = (ty - dt * g.uy) * g.ir, wz = (tz - dt * g.uz) * g.ir;
    float X[NA], Y[NA];
#pragma unroll
    for (int n = 0; n < NA; ++n) X[n] = Y[n] = 0.f;
    float CM[2], Pz[2];   // per order: w_x dP/dx + w_y dP/dy and P w_z, cosine and sine
    high_visit<L3, 2 * NA, 3>(
        tab + g.u * AS, g.uz,
        [&](auto Mc) {
          constexpr int M = decltype(Mc)::value;
          CM[0] = CM[1] = 0.f;
          if constexpr (M > 0) {
            CM[0] = (float)M * (wx * g.R[M - 1] - wy * g.I[M - 1]);
            CM[1] = (float)M * (wx * g.I[M - 1] + wy * g.R[M - 1]);
          }
          Pz[0] = g.R[M] * wz;
          Pz[1] = g.I[M] * wz;
        },
        [&](auto Mc, float q, float dq, int sn, const HighRow<2 * NA>& row) {
          constexpr int M = decltype(Mc)::value;
          // Y = Qhat P and grad p . w = Qhat CM + dQhat P w_z
          const float v = q * (sn ? g.I[M] : g.R[M]);
          const float gw = fmaf(q, CM[sn], dq * Pz[sn]);
#pragma unroll
          for (int n = 0; n < NA; ++n) {
            X[n] = fmaf(row.v[n], v, fmaf(-row.v[NA + n], gw, X[n]));
            Y[n] = fmaf(row.v[NA + n], v, Y[n]);
          }
        },
        [&](auto) {});
    lds_lane_exchange();   // every lane's table reads are issued before the record overwrites it
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      rec[(S::RX + n) * RS + lane] = X[n];
      rec[(S::RY + n) * RS + lane] = Y[n] * dt;
    }
#pragma unroll
    for (int kk = 0; kk < KA; ++kk) {
      rec[(S::RF + kk) * RS + lane] = f[kk];
      rec[(S::RFP + kk) * RS + lane] = fp[kk];
    }
    rec[S::RJ * RS + lane] = __int_as_float(a.type[g.j]);
    lds_lane_exchange();
    // four pairs per step, so their LDS reads are in flight together; pairs
    // past the chunk read pair 0 and add nothing
    const int np = min(kWave, gr.total - c0);
    for (int j0 = ph; j0 < np; j0 += 4 * S::NPH) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int jj = j0 + e * S::NPH;
        const bool in = jj < np;
        const int jr = in ? jj : 0;
        const int J = in ? __float_as_int(rec[S::RJ * RS + jr]) : -1;
#pragma unroll
        for (int r = 0; r < S::SPL; ++r) {
          const float val = fmaf(rec[(S::RX + sn[r]) * RS + jr], rec[(S::RF + sk[r]) * RS + jr],
                                 -rec[(S::RY + sn[r]) * RS + jr] * rec[(S::RFP + sk[r]) * RS + jr]);
#pragma unroll
          for (int t = 0; t < T; ++t) cb[r][t] += J == t ? val : 0.f;
        }
      }
    }
    lds_lane_exchange();   // the record is read before the next chunk stages the table
  }
  if constexpr (S::NPH == 2) {
#pragma unroll
    for (int r = 0; r < S::SPL; ++r)
#pragma unroll
      for (int t = 0; t < T; ++t) cb[r][t] = xor32_sum(cb[r][t]);
  }
#pragma unroll
  for (int r = 0; r < S::SPL; ++r) {
    const int s = s0 + r * (kWave / S::NPH);
    if (ph == 0 && s < S::NS)
#pragma unroll
      for (int t = 0; t < T; ++t) a.part[(size_t)wave * a.PW + (t * NA + sn[r]) * KA + sk[r]] += cb[r][t];
  }
}

}  // namespace nep
