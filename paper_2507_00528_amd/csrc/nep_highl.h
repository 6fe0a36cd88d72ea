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
// positions of one wavefront of the main kernels).  Their angular pairs form
// one stream; chunks of 64 pairs are staged in LDS, one lane per pair
// (direction, g_n, g'_n, tangent, the powers (x + iy)^k), and then every lane
// walks the chunk.  Lane c holds harmonic (l, m) number c of l = 5..L3 (at
// most 56) for every channel n.
//
// Harmonic basis.  q_nl = sum_m C_lm S_nlm^2 with C_lm = 1 / integral of b_lm^2
// equals sum_m S~_nlm^2 for the sums S~ of any orthonormal real harmonics of
// degree l (both are (2l+1)/(4 pi) sum_jk g_n g_n P_l(u_j . u_k), the addition
// theorem).  So these kernels use the orthonormal real harmonics
//   Y_lm = N_lM Q_l^M(z) Re (x + i y)^M   (m = 2M - 1, or m = 0 with M = 0)
//   Y_lm = N_lM Q_l^M(z) Im (x + i y)^M   (m = 2M)
// with Q_l^M the associated Legendre function over (1 - z^2)^(M/2) (a
// polynomial in z from the three-term recurrence in l) and N_lM^2 =
// (2l+1)/(4 pi) (l-M)!/(l+M)! (times 2 for M > 0).  With C = 1 in this basis,
// dq/dS~ = 2 S~.  Each lane keeps N Q_l^M as z^par H(z^2), H of degree <= 4, and
// evaluates it by Horner's rule.
#pragma once
#include "nep_device.h"
#include "nep_kernels.h"

namespace nep {

constexpr int kPwStride = 19;   // words per pair in the power table (odd: no bank conflicts)

struct HighLane {
  int l;
  bool on;
  bool par;                  // Q has odd degree
  float a[5], b[4];          // H(w) = sum a_k w^k, H'(w) = sum b_k w^k
  int iP, iD1, iD2;          // power-table words of P, and of the two derivative factors
  float sD1, sD2;            // dP/dx = sD1 pw[iD1], dP/dy = sD2 pw[iD2]
};

__device__ __forceinline__ HighLane high_lane(int c, int L3) {
  HighLane h;
  h.l = 5;
  h.on = false;
  int M = 0, off = 0;
  bool sine = false;
  for (int l = 5; l <= L3; ++l) {
    const int w = 2 * l + 1;
    if (c >= off && c < off + w) {
      const int mi = c - off;
      h.l = l;
      M = (mi + 1) >> 1;
      sine = mi > 0 && (mi & 1) == 0;
      h.on = true;
    }
    off += w;
  }
  // coefficients of Q_l^M in powers of z, by the recurrence
  //   Q_M^M = (2M-1)!!,  (l-M) Q_l = (2l-1) z Q_{l-1} - (l+M-1) Q_{l-2}
  double q0[9], q1[9];
#pragma unroll
  for (int p = 0; p < 9; ++p) q0[p] = q1[p] = 0.0;
  double df = 1.0;
  for (int k = 1; k <= M; ++k) df *= (double)(2 * k - 1);
  q1[0] = df;
  for (int lp = M + 1; lp <= h.l; ++lp) {
    double qn[9];
#pragma unroll
    for (int p = 0; p < 9; ++p)
      qn[p] = ((2.0 * lp - 1.0) * (p > 0 ? q1[p - 1] : 0.0) - (lp + M - 1.0) * q0[p]) / (double)(lp - M);
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      q0[p] = q1[p];
      q1[p] = qn[p];
    }
  }
  double nrm = (2.0 * h.l + 1.0) / (4.0 * 3.141592653589793);
  for (int k = h.l - M + 1; k <= h.l + M; ++k) nrm /= (double)k;
  if (M > 0) nrm *= 2.0;
  nrm = h.on ? sqrt(nrm) : 0.0;
  h.par = ((h.l - M) & 1) != 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double v = 0.0;
#pragma unroll
    for (int p = 0; p < 9; ++p) v = (p == 2 * k + (h.par ? 1 : 0)) ? q1[p] : v;
    h.a[k] = (float)(nrm * v);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) h.b[k] = (float)(k + 1) * h.a[k + 1];
  // d/dx (x+iy)^M = M (x+iy)^(M-1), d/dy (x+iy)^M = i M (x+iy)^(M-1)
  const int m1 = M > 0 ? M - 1 : 0;
  h.iP = (sine ? 9 : 0) + M;
  h.iD1 = (sine ? 9 : 0) + m1;
  h.iD2 = (sine ? 0 : 9) + m1;
  h.sD1 = (float)M;
  h.sD2 = sine ? (float)M : -(float)M;
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

// Sums of V = 4 or 8 values over the 64 lanes, scattered: on return the lanes
// with (lane & (V - 1)) == v hold the total of value v.  A butterfly over
// lane bits 0, 1 (and 2) halves the values a lane carries at each step, so the
// V sums take V - 1 lane exchanges before the sum over the 8 groups instead
// of 3 V.
template <int V>
__device__ __forceinline__ float wave_scatter_sum(const float (&x)[V]) {
  static_assert(V == 4 || V == 8, "4 or 8 values");
  const int lane = threadIdx.x & (kWave - 1);
  const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
  float y[V / 2];
#pragma unroll
  for (int w = 0; w < V / 2; ++w) {   // y[w]: value 2w + b0
    const float send = b0 ? x[2 * w] : x[2 * w + 1];
    y[w] = (b0 ? x[2 * w + 1] : x[2 * w]) + dpp<kDppXor1>(send);
  }
  float z[V / 4];
#pragma unroll
  for (int u = 0; u < V / 4; ++u) {   // z[u]: value 4u + 2 b1 + b0
    const float send = b1 ? y[2 * u] : y[2 * u + 1];
    z[u] = (b1 ? y[2 * u + 1] : y[2 * u]) + dpp<kDppXor2>(send);
  }
  float r;
  if constexpr (V == 8) {             // value lane & 7 over the 8-lane group
    const float send = b2 ? z[0] : z[1];
    r = (b2 ? z[1] : z[0]) + xor4_val(send);
  } else {                            // value lane & 3 over the quad, then the group
    r = z[0] + xor4_val(z[0]);
  }
  return atoms8_sum(r);
}

// Per-wave LDS record of up to 64 pairs, field-major: rec[f * 64 + slot].
// kTan: tangent fields; kF: the radial basis f_k, f'_k.
template <int NA, int KA, bool kTan, bool kF>
struct HighRec {
  static constexpr int DX = 0, DY = 1, DZ = 2, IR = 3, U = 4, AI = 5, KI = 6, J = 7, G = 8, GP = G + NA;
  static constexpr int DT = GP + NA, WX = DT + 1, WY = DT + 2, WZ = DT + 3;
  static constexpr int F = kTan ? WZ + 1 : DT;
  static constexpr int FP = F + (kF ? KA : 0);
  static constexpr int W = FP + (kF ? KA : 0);
};

// The 8 atom slots of a wavefront and their pair counts.
struct HighGroup {
  int pa0, total;
  int cum[kAPW + 1];   // pairs before slot u
};

__device__ __forceinline__ HighGroup high_group(const HighArgs& a, int pa0) {
  HighGroup g;
  g.pa0 = pa0;
  g.cum[0] = 0;
#pragma unroll
  for (int u = 0; u < kAPW; ++u) {
    const int i = a.order[pa0 + u];
    const int n = i >= 0 ? min(a.nb.cntA[i], a.nb.capA) : 0;
    g.cum[u + 1] = g.cum[u] + n;
  }
  g.total = g.cum[kAPW];
  return g;
}

// Stages pairs [c0, c0 + 64) of the group's stream, one per lane.
template <class C, bool kTri, bool kTan, bool kF>
__device__ __forceinline__ void high_stage(const HighArgs& a, const HighGroup& gr, int c0, float* rec, float* pw) {
  constexpr int T = C::T, NA = C::NA, KA = C::KA;
  using R = HighRec<NA, KA, kTan, kF>;
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
      rec[(R::G + n) * kWave + lane] = s0;
      rec[(R::GP + n) * kWave + lane] = s1;
    }
    if constexpr (kF) {
#pragma unroll
      for (int kk = 0; kk < KA; ++kk) {
        rec[(R::F + kk) * kWave + lane] = f[kk];
        rec[(R::FP + kk) * kWave + lane] = fp[kk];
      }
    }
    const float ux = q.dx * q.inv_r, uy = q.dy * q.inv_r, uz = q.dz * q.inv_r;
    rec[R::DX * kWave + lane] = q.dx;
    rec[R::DY * kWave + lane] = q.dy;
    rec[R::DZ * kWave + lane] = q.dz;
    rec[R::IR * kWave + lane] = q.inv_r;
    rec[R::U * kWave + lane] = __int_as_float(u);
    rec[R::AI * kWave + lane] = __int_as_float(i);
    rec[R::KI * kWave + lane] = __int_as_float(k);
    rec[R::J * kWave + lane] = __int_as_float(J);
    float c = 1.f, s = 0.f;
    float* p = pw + lane * kPwStride;
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
      rec[R::DT * kWave + lane] = dt;
      rec[R::WX * kWave + lane] = (tx - dt * ux) * q.inv_r;
      rec[R::WY * kWave + lane] = (ty - dt * uy) * q.inv_r;
      rec[R::WZ * kWave + lane] = (tz - dt * uz) * q.inv_r;
    }
  }
  lds_lane_exchange();
}

// Walks the group's pair stream: start(u) before the first pair of slot u,
// pair(u, jj) for each staged pair jj of slot u, finish(u) after its last pair
// (also for slots without pairs), flush(c0) after each chunk of 64 pairs.
struct NoFlush {
  __device__ void operator()(int) const {}
};

template <class C, bool kTri, bool kTan, bool kF, class Start, class Pair, class Finish, class Flush = NoFlush>
__device__ __forceinline__ void high_walk(const HighArgs& a, const HighGroup& gr, float* rec, float* pw,
                                          Start&& start, Pair&& pair, Finish&& finish, Flush&& flush = Flush{}) {
  using R = HighRec<C::NA, C::KA, kTan, kF>;
  int cur = 0;
  start(0);
  for (int c0 = 0; c0 < gr.total; c0 += kWave) {
    high_stage<C, kTri, kTan, kF>(a, gr, c0, rec, pw);
    const int np = min(kWave, gr.total - c0);
    for (int jj = 0; jj < np; ++jj) {
      const int u = __float_as_int(rec[R::U * kWave + jj]);
      while (cur < u) {
        finish(cur);
        ++cur;
        start(cur);
      }
      pair(cur, jj);
    }
    flush(c0);
    lds_lane_exchange();
  }
  for (;;) {
    finish(cur);
    if (++cur == kAPW) break;
    start(cur);
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
    const float t = wave_scatter_sum<8>(xs);
    if (lane < 8 && g0 + lane < NV) rows[(size_t)(C::NR + 4 * C::NA + g0 + lane) * Npad + pa] = t;
  }
}

template <class C>
__device__ __forceinline__ size_t high_slot(int pa, int n, int lane) {
  return ((size_t)pa * C::NA + n) * C::YH + (lane < C::YH ? lane : 0);
}

#define NEP_HIGH_PROLOGUE(TAN, F)                                        \
  constexpr int NA = C::NA, KA = C::KA, L3 = C::L3, YH = C::YH;         \
  using R = HighRec<NA, KA, TAN, F>;                                     \
  __shared__ float recs[4][R::W * kWave];                                \
  __shared__ float pws[4][kWave * kPwStride];                            \
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;  \
  const int wave = blockIdx.x * 4 + wv;                                  \
  float* rec = recs[wv];                                                 \
  float* pw = pws[wv];                                                   \
  const HighLane h = high_lane(lane, L3);                                \
  const HighGroup gr = high_group(a, wave * kAPW);                       \
  (void)KA;                                                              \
  (void)YH;

template <class C, bool kTri>
__global__ __launch_bounds__(256) void k_high_desc(HighArgs a) {
  NEP_HIGH_PROLOGUE(false, false)
  float S[NA];
  auto start = [&](int) {
#pragma unroll
    for (int n = 0; n < NA; ++n) S[n] = 0.f;
  };
  auto pair = [&](int, int jj) {
    float v, gx, gy, gz;
    high_eval(h, rec[R::DZ * kWave + jj] * rec[R::IR * kWave + jj], pw + jj * kPwStride, v, gx, gy, gz);
#pragma unroll
    for (int n = 0; n < NA; ++n) S[n] = fmaf(rec[(R::G + n) * kWave + jj], v, S[n]);
  };
  auto finish = [&](int u) {
    const int pa = gr.pa0 + u;
    if (a.order[pa] < 0) return;
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
  high_walk<C, kTri, false, false>(a, gr, rec, pw, start, pair, finish);
}

template <class C, bool kTri>
__global__ __launch_bounds__(256) void k_high_force(HighArgs a) {
  NEP_HIGH_PROLOGUE(false, false)
  float A[NA];
  float vir[6];
  float pfx = 0.f, pfy = 0.f, pfz = 0.f;   // this lane's staged pair
  auto start = [&](int u) {
    // A = dE/dS~ = 2 E'_nl S~
    const int pa = gr.pa0 + u;
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      const float s = a.Sh[high_slot<C>(pa, n, lane)];
      A[n] = 2.0f * high_rowval<C>(a.Ep, a.Npad, pa, h, n) * (lane < YH ? s : 0.f);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) vir[c] = 0.f;
  };
  auto pair = [&](int, int jj) {
    const float ir = rec[R::IR * kWave + jj];
    const float dx = rec[R::DX * kWave + jj], dy = rec[R::DY * kWave + jj], dz = rec[R::DZ * kWave + jj];
    const float ux = dx * ir, uy = dy * ir, uz = dz * ir;
    float v, gx, gy, gz;
    high_eval(h, uz, pw + jj * kPwStride, v, gx, gy, gz);
    float su = 0.f, sv = 0.f;
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      su = fmaf(A[n], rec[(R::G + n) * kWave + jj], su);
      sv = fmaf(A[n], rec[(R::GP + n) * kWave + jj], sv);
    }
    // f_ij = sum A (g'_n u Y + g_n grad Y), grad Y = (I - u u^T) grad p / r
    const float parts[4] = {sv * v, su * gx, su * gy, su * gz};
    const float tot = wave_scatter_sum<4>(parts);
    const float vv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tot), 0));
    const float Gx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tot), 1));
    const float Gy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tot), 2));
    const float Gz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tot), 3));
    const float rad = ux * Gx + uy * Gy + uz * Gz;
    const float fx = vv * ux + (Gx - rad * ux) * ir;
    const float fy = vv * uy + (Gy - rad * uy) * ir;
    const float fz = vv * uz + (Gz - rad * uz) * ir;
    // the lane that staged pair jj adds it to fA after the chunk
    const bool mine = lane == jj;
    pfx = mine ? fx : pfx;
    pfy = mine ? fy : pfy;
    pfz = mine ? fz : pfz;
    vir[0] -= fx * dx; vir[1] -= fy * dy; vir[2] -= fz * dz;
    vir[3] -= fx * dy; vir[4] -= fy * dz; vir[5] -= fz * dx;
  };
  auto finish = [&](int u) {
    const int i = a.order[gr.pa0 + u];
    if (i >= 0 && lane == 0)
#pragma unroll
      for (int c = 0; c < 6; ++c) a.wv[(size_t)c * a.N + i] += vir[c];
  };
  auto flush = [&](int c0) {
    if (c0 + lane < gr.total) {
      const size_t o = (size_t)__float_as_int(rec[R::AI * kWave + lane]) * a.nb.capA +
                       __float_as_int(rec[R::KI * kWave + lane]);
      float* fo = a.fA + 3 * o;
      fo[0] += pfx;
      fo[1] += pfy;
      fo[2] += pfz;
    }
  };
  high_walk<C, kTri, false, false>(a, gr, rec, pw, start, pair, finish, flush);
}

template <class C, bool kTri>
__global__ __launch_bounds__(256) void k_high_tangent(HighArgs a) {
  NEP_HIGH_PROLOGUE(true, false)
  float Sd[NA];
  auto start = [&](int) {
#pragma unroll
    for (int n = 0; n < NA; ++n) Sd[n] = 0.f;
  };
  auto pair = [&](int, int jj) {
    float v, gx, gy, gz;
    high_eval(h, rec[R::DZ * kWave + jj] * rec[R::IR * kWave + jj], pw + jj * kPwStride, v, gx, gy, gz);
    // Sdot = sum_j g'_n (u.t) Y + g_n grad p . (t - (u.t) u) / r
    const float gwt = gx * rec[R::WX * kWave + jj] + gy * rec[R::WY * kWave + jj] + gz * rec[R::WZ * kWave + jj];
    const float vdt = v * rec[R::DT * kWave + jj];
#pragma unroll
    for (int n = 0; n < NA; ++n)
      Sd[n] = fmaf(rec[(R::GP + n) * kWave + jj], vdt, fmaf(rec[(R::G + n) * kWave + jj], gwt, Sd[n]));
  };
  auto finish = [&](int u) {
    const int pa = gr.pa0 + u;
    if (a.order[pa] < 0) return;
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
  high_walk<C, kTri, true, false>(a, gr, rec, pw, start, pair, finish);
}

// The c^A gradient: for each pair, X_n = sum_lm (Sbar_nlm Y - A_nlm grad Y . w)
// and Y_n = sum_lm A_nlm Y (sums over the lanes), then
// dL/dc_nk^{IJ} += X_n f_k - Y_n (u.t) f'_k.  Channels go in groups of four:
// the 8 sums of a group (X of its channels, then Y) come out of one scattered
// sum, lanes with (lane & 7) = e holding X of channel e and 4 + e holding Y.
// Coefficient slots (channel, J, k) are dealt to the lanes: lane l takes
// channel 4 cg + (l & 3) of group cg and slot (J, k) = 16 sg + (l >> 2) of
// slot group sg, for every group pair (cg, sg).
template <class C, bool kTri>
__global__ __launch_bounds__(256) void k_high_coef(HighArgs a) {
  constexpr int T = C::T;
  NEP_HIGH_PROLOGUE(true, true)
  constexpr int NCG = (NA + 3) / 4, NSG = (T * KA + 15) / 16;
  const int ne = lane & 3, se = lane >> 2;
  float cb[NCG][NSG];
#pragma unroll
  for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
    for (int sg = 0; sg < NSG; ++sg) cb[cg][sg] = 0.f;
  float Sb[NA], Av[NA];
  auto start = [&](int u) {
    // Sbar = 2 (Gbar S~ - E' Sdot~), A = 2 E' S~ (signs as in the main adjoint)
    const int pa = gr.pa0 + u;
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      const size_t o = high_slot<C>(pa, n, lane);
      const float s = lane < YH ? a.Sh[o] : 0.f, sd = lane < YH ? a.Sdh[o] : 0.f;
      const float ep = high_rowval<C>(a.Ep, a.Npad, pa, h, n), gb = high_rowval<C>(a.Gb, a.Npad, pa, h, n);
      Sb[n] = 2.0f * (gb * s - ep * sd);
      Av[n] = 2.0f * ep * s;
    }
  };
  auto pair = [&](int, int jj) {
    float v, gx, gy, gz;
    high_eval(h, rec[R::DZ * kWave + jj] * rec[R::IR * kWave + jj], pw + jj * kPwStride, v, gx, gy, gz);
    const float gwt = gx * rec[R::WX * kWave + jj] + gy * rec[R::WY * kWave + jj] + gz * rec[R::WZ * kWave + jj];
    const int J = __float_as_int(rec[R::J * kWave + jj]);
    const float dt = rec[R::DT * kWave + jj];
    const bool lo = (lane & 4) == 0;
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) {
      float xs[8];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int n = 4 * cg + e;
        const int nc = n < NA ? n : 0;
        xs[e] = n < NA ? fmaf(Sb[nc], v, -Av[nc] * gwt) : 0.f;
        xs[4 + e] = n < NA ? Av[nc] * v : 0.f;
      }
      const float own = wave_scatter_sum<8>(xs);
      const float other = xor4_val(own);
      const float Xe = lo ? own : other, Ye = lo ? other : own;
#pragma unroll
      for (int sg = 0; sg < NSG; ++sg) {
        const int sl = 16 * sg + se;
        const int te = sl / KA, ke = sl % KA;
        const int kc = sl < T * KA ? ke : 0;
        const float fk = rec[(R::F + kc) * kWave + jj], fpk = rec[(R::FP + kc) * kWave + jj];
        cb[cg][sg] += (T == 1 || J == te) ? fmaf(Xe, fk, -Ye * dt * fpk) : 0.f;
      }
    }
  };
  auto finish = [&](int) {};
  high_walk<C, kTri, true, true>(a, gr, rec, pw, start, pair, finish);
#pragma unroll
  for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
    for (int sg = 0; sg < NSG; ++sg) {
      const int n = 4 * cg + ne, sl = 16 * sg + se;
      if (n < NA && sl < T * KA) {
        const int te = sl / KA, ke = sl % KA;
        a.part[(size_t)wave * a.PW + (te * NA + n) * KA + ke] += cb[cg][sg];
      }
    }
}

#undef NEP_HIGH_PROLOGUE

}  // namespace nep
