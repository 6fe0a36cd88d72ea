// Device-side arithmetic of the NEP descriptor, written for gfx950 (wave64).
//
// Radial basis: Eq. 6 with the Chebyshev recursion (A1.1, A1.5) and the cosine
// cutoff (A2.1-A2.2).  Angular basis: the Cartesian harmonics of Appendix B for
// l <= 4, evaluated on the unit vector u = d/|d| (on the unit sphere r^2 = 1, so
// the polynomials simplify), with their Cartesian gradients.  Because
// B_lm(d) = b_lm(d/|d|) has degree 0, grad_d B_lm = (I - u u^T) grad b(u) / |d|
// for any extension of b off the sphere.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nep {

constexpr int kWave = 64;

// Read-only parameter arrays are addressed through the constant address
// space: with a wave-uniform address the loads become scalar (s_load) and the
// values live in SGPRs, feeding VALU instructions as scalar operands.
template <class T>
using cptr = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)(p);
}

// FW_ = 0: the per-atom kernels are compiled for 2 and 3 wavefronts per SIMD
// (a launch choice); otherwise for FW_ only (the padded size classes).
template <int T_, int NR_, int NA_, int KR_, int KA_, int L3_, int L4_, int L5_, int FW_ = 0>
struct Cfg {
  static constexpr int FIXED_WAVES = FW_;
  static constexpr int T = T_, NR = NR_, NA = NA_, KR = KR_, KA = KA_;
  static constexpr int L3 = L3_, L4 = L4_, L5 = L5_;
  // the per-atom kernels hold the harmonics of l <= 4 (and of the 4-/5-body
  // terms); degrees 5..L3 run in separate kernels (nep_highl.h)
  static constexpr int L3LO = L3 < 4 ? L3 : 4;
  static constexpr int LMAX = (L3LO > L4 ? (L3LO > L5 ? L3LO : L5) : (L4 > L5 ? L4 : L5));
  static constexpr int Y = LMAX * (LMAX + 2);
  static constexpr int YH = L3 > 4 ? (L3 + 1) * (L3 + 1) - 25 : 0;   // harmonics of l = 5..L3
  // waves per SIMD the adjoint is compiled for: 3 (a few registers spill, and
  // the extra wave hides more latency than the spills cost), except with
  // degrees l > 4, whose larger descriptor would spill too much
  static constexpr int ADJ_WAVES = YH > 0 ? 2 : 3;
  static constexpr int D = NR + NA * L3 + (L4 ? NA : 0) + (L5 ? NA : 0);
  static constexpr int PS = T * NR * KR + T * NA * KA;  // c-grad slots of one center species
};

// --------------------------------------------------------- transcendentals
// Hardware instructions: v_cos_f32 / v_sin_f32 take the angle in turns
// (cos(2 pi t)), v_rsq_f32 is 1/sqrt, v_rcp_f32 is 1/x and v_exp_f32 is 2^x.
// Their errors (a few ulp over these arguments) sit far below the FP32 path's
// tolerances, and each is one instruction instead of a library sequence.
__device__ __forceinline__ float cos_turns(float t) { return __builtin_amdgcn_cosf(t); }
__device__ __forceinline__ float sin_turns(float t) { return __builtin_amdgcn_sinf(t); }
__device__ __forceinline__ float rsq_hw(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }

// tanh z = 1 - 2 / (e^{2z} + 1); saturates to +-1 through e^{2z} = inf or 0
__device__ __forceinline__ float tanh_hw(float z) {
  const float e = __builtin_amdgcn_exp2f(z * 2.8853900817779268f);   // 2 / ln 2
  return fmaf(-2.0f, rcp_hw(e + 1.0f), 1.0f);
}

// ------------------------------------------------------------------ radial
// f_k(r) = (T_k(xi) + 1)/2 * f_c(r), xi = 2 (r/rc - 1)^2 - 1, and df_k/dr;
// f_c(r) = (1 + cos(pi r / rc)) / 2.  Written as two FMAs per order (four
// with the derivative).
template <int K>
__device__ __forceinline__ void radial_basis(float r, float inv_rc, float (&f)[K]) {
  const float u = r * inv_rc;
  const float x = u - 1.0f;
  const float xi = fmaf(2.0f * x, x, -1.0f);
  const float xi2 = 2.0f * xi;
  const float hfc = fmaf(0.25f, cos_turns(0.5f * u), 0.25f);   // f_c / 2
  float t0 = 1.0f, t1 = xi;
  f[0] = 2.0f * hfc;
  if (K > 1) f[1] = fmaf(xi, hfc, hfc);
#pragma unroll
  for (int k = 2; k < K; ++k) {
    const float t2 = fmaf(xi2, t1, -t0);
    f[k] = fmaf(t2, hfc, hfc);
    t0 = t1;
    t1 = t2;
  }
}

template <int K>
__device__ __forceinline__ void radial_basis_d(float r, float inv_rc, float (&f)[K], float (&fp)[K]) {
  const float u = r * inv_rc;
  const float x = u - 1.0f;
  const float xi = fmaf(2.0f * x, x, -1.0f);
  const float xi2 = 2.0f * xi;
  const float dxi = 4.0f * x * inv_rc;
  const float hfc = fmaf(0.25f, cos_turns(0.5f * u), 0.25f);                     // f_c / 2
  const float hfcp = -0.25f * 3.14159265358979f * inv_rc * sin_turns(0.5f * u);  // f_c' / 2
  const float a = dxi * hfc;   // d(T_k)/dr coefficient of f_c / 2
  float t0 = 1.0f, t1 = xi, d0 = 0.0f, d1 = 1.0f;
  f[0] = 2.0f * hfc;
  fp[0] = 2.0f * hfcp;
  if (K > 1) {
    f[1] = fmaf(xi, hfc, hfc);
    fp[1] = fmaf(xi, hfcp, fmaf(d1, a, hfcp));
  }
#pragma unroll
  for (int k = 2; k < K; ++k) {
    const float t2 = fmaf(xi2, t1, -t0);
    const float d2 = fmaf(xi2, d1, fmaf(2.0f, t1, -d0));
    f[k] = fmaf(t2, hfc, hfc);
    fp[k] = fmaf(t2, hfcp, fmaf(d2, a, hfcp));
    t0 = t1;
    t1 = t2;
    d0 = d1;
    d1 = d2;
  }
}

// ---------------------------------------------------------------- angular
// C_lm * 4 pi for l = 1..4 in Appendix-B order.  C_lm = 1 / (integral over the
// unit sphere of b_lm^2), which makes sum_m C_lm B_lm(u) B_lm(v) equal to
// (2l+1)/(4 pi) P_l(u.v) (the addition theorem behind Eq. 7).
__device__ __forceinline__ float clm(int lm) {
  constexpr float inv4pi = 0.0795774715459477f;
  constexpr float c[24] = {3.f, 3.f, 3.f,
                           1.25f, 15.f, 15.f, 3.75f, 3.75f,
                           1.75f, 2.625f, 2.625f, 26.25f, 26.25f, 4.375f, 4.375f,
                           0.140625f, 5.625f, 5.625f, 2.8125f, 2.8125f, 39.375f, 39.375f,
                           4.921875f, 4.921875f};
  return c[lm] * inv4pi;
}

// b_lm(u) for |u| = 1, l = 1..LM (Appendix B with r = 1).
template <int LM>
__device__ __forceinline__ void harm_val(float x, float y, float z, float (&b)[LM * (LM + 2)]) {
  b[0] = z;
  b[1] = x;
  b[2] = y;
  if constexpr (LM >= 2) {
    b[3] = 3.0f * z * z - 1.0f;
    b[4] = x * z;
    b[5] = y * z;
    b[6] = x * x - y * y;
    b[7] = 2.0f * x * y;
  }
  if constexpr (LM >= 3) {
    const float z2 = z * z, x2 = x * x, y2 = y * y;
    b[8] = (5.0f * z2 - 3.0f) * z;
    b[9] = (5.0f * z2 - 1.0f) * x;
    b[10] = (5.0f * z2 - 1.0f) * y;
    b[11] = (x2 - y2) * z;
    b[12] = 2.0f * x * y * z;
    b[13] = (x2 - 3.0f * y2) * x;
    b[14] = (3.0f * x2 - y2) * y;
  }
  if constexpr (LM >= 4) {
    const float z2 = z * z, x2 = x * x, y2 = y * y;
    b[15] = (35.0f * z2 - 30.0f) * z2 + 3.0f;
    b[16] = (7.0f * z2 - 3.0f) * z * x;
    b[17] = (7.0f * z2 - 3.0f) * z * y;
    b[18] = (7.0f * z2 - 1.0f) * (x2 - y2);
    b[19] = (7.0f * z2 - 1.0f) * 2.0f * x * y;
    b[20] = (x2 - 3.0f * y2) * x * z;
    b[21] = (3.0f * x2 - y2) * y * z;
    b[22] = x2 * x2 - 6.0f * x2 * y2 + y2 * y2;
    b[23] = 4.0f * x * y * (x2 - y2);
  }
}

// Gradients of the b_lm at u, written out term by term so that components
// that vanish identically cost nothing (a multiply by a literal zero cannot be
// folded without fast-math).
//   harm_dir:      d[lm] = grad b_lm(u) . w
//   harm_grad_sum: g = sum_lm w[lm] grad b_lm(u)
template <int LM>
__device__ __forceinline__ void harm_dir(float x, float y, float z, float wx, float wy, float wz,
                                         float (&d)[LM * (LM + 2)]) {
  d[0] = wz;
  d[1] = wx;
  d[2] = wy;
  if constexpr (LM >= 2) {
    const float P = x * wx - y * wy, Q = y * wx + x * wy;
    d[3] = 6.0f * z * wz;
    d[4] = z * wx + x * wz;
    d[5] = z * wy + y * wz;
    d[6] = 2.0f * P;
    d[7] = 2.0f * Q;
    if constexpr (LM >= 3) {
      const float x2 = x * x, y2 = y * y, z2 = z * z;
      const float f5 = 5.0f * z2 - 1.0f, dxy = x2 - y2, xy = x * y;
      d[8] = (15.0f * z2 - 3.0f) * wz;
      d[9] = f5 * wx + 10.0f * x * z * wz;
      d[10] = f5 * wy + 10.0f * y * z * wz;
      d[11] = 2.0f * z * P + dxy * wz;
      d[12] = 2.0f * z * Q + 2.0f * xy * wz;
      d[13] = 3.0f * dxy * wx - 6.0f * xy * wy;
      d[14] = 6.0f * xy * wx + 3.0f * dxy * wy;
      if constexpr (LM >= 4) {
        const float a = 7.0f * z2 - 1.0f, c = (7.0f * z2 - 3.0f) * z, e = 21.0f * z2 - 3.0f;
        d[15] = (140.0f * z2 - 60.0f) * z * wz;
        d[16] = c * wx + e * x * wz;
        d[17] = c * wy + e * y * wz;
        d[18] = 2.0f * a * P + 14.0f * z * dxy * wz;
        d[19] = 2.0f * a * Q + 28.0f * xy * z * wz;
        d[20] = 3.0f * dxy * z * wx - 6.0f * xy * z * wy + (x2 - 3.0f * y2) * x * wz;
        d[21] = 6.0f * xy * z * wx + 3.0f * dxy * z * wy + (3.0f * x2 - y2) * y * wz;
        d[22] = 4.0f * x * (x2 - 3.0f * y2) * wx + 4.0f * y * (y2 - 3.0f * x2) * wy;
        d[23] = 4.0f * y * (3.0f * x2 - y2) * wx + 4.0f * x * (x2 - 3.0f * y2) * wy;
      }
    }
  }
}

template <int LM>
__device__ __forceinline__ void harm_grad_sum(float x, float y, float z, const float (&w)[LM * (LM + 2)], float& gx,
                                              float& gy, float& gz) {
  gx = w[1];
  gy = w[2];
  gz = w[0];
  if constexpr (LM >= 2) {
    gx = fmaf(z, w[4], fmaf(2.0f * x, w[6], fmaf(2.0f * y, w[7], gx)));
    gy = fmaf(z, w[5], fmaf(-2.0f * y, w[6], fmaf(2.0f * x, w[7], gy)));
    gz = fmaf(6.0f * z, w[3], fmaf(x, w[4], fmaf(y, w[5], gz)));
    if constexpr (LM >= 3) {
      const float x2 = x * x, y2 = y * y, z2 = z * z;
      const float f5 = 5.0f * z2 - 1.0f, dxy = x2 - y2, xy = x * y;
      gx = fmaf(f5, w[9], fmaf(2.0f * x * z, w[11], fmaf(2.0f * y * z, w[12],
           fmaf(3.0f * dxy, w[13], fmaf(6.0f * xy, w[14], gx)))));
      gy = fmaf(f5, w[10], fmaf(-2.0f * y * z, w[11], fmaf(2.0f * x * z, w[12],
           fmaf(-6.0f * xy, w[13], fmaf(3.0f * dxy, w[14], gy)))));
      gz = fmaf(15.0f * z2 - 3.0f, w[8], fmaf(10.0f * x * z, w[9], fmaf(10.0f * y * z, w[10],
           fmaf(dxy, w[11], fmaf(2.0f * xy, w[12], gz)))));
      if constexpr (LM >= 4) {
        const float a = 7.0f * z2 - 1.0f, c = (7.0f * z2 - 3.0f) * z, e = 21.0f * z2 - 3.0f;
        const float xyz = xy * z, t1 = x2 - 3.0f * y2, t2 = 3.0f * x2 - y2;
        gx = fmaf(c, w[16], fmaf(2.0f * x * a, w[18], fmaf(2.0f * y * a, w[19], fmaf(3.0f * dxy * z, w[20],
             fmaf(6.0f * xyz, w[21], fmaf(4.0f * x * t1, w[22], fmaf(4.0f * y * t2, w[23], gx)))))));
        gy = fmaf(c, w[17], fmaf(-2.0f * y * a, w[18], fmaf(2.0f * x * a, w[19], fmaf(-6.0f * xyz, w[20],
             fmaf(3.0f * dxy * z, w[21], fmaf(-4.0f * y * t2, w[22], fmaf(4.0f * x * t1, w[23], gy)))))));
        gz = fmaf((140.0f * z2 - 60.0f) * z, w[15], fmaf(e * x, w[16], fmaf(e * y, w[17],
             fmaf(14.0f * z * dxy, w[18], fmaf(28.0f * xyz, w[19], fmaf(t1 * x, w[20], fmaf(t2 * y, w[21], gz)))))));
      }
    }
  }
}

// ------------------------------------------------- 4-body and 5-body terms
// The l = 2 sums (S_20..S_24) are the components of a traceless symmetric
// matrix M: M_zz = S_20/3, M_xz = S_21, M_yz = S_22, M_xx - M_yy = S_23,
// M_xy = S_24/2.  q4 = tr(M^3); dq4/dS_m = tr(Q E_m) with Q = 3 M^2, where E_m
// is dM/dS_m, and the Hessian applied to a tangent is tr(Q' E_m) with
// Q' = 3 (Mdot M + M Mdot).
struct Sym3 {
  float xx, yy, zz, xy, xz, yz;
};

__device__ __forceinline__ Sym3 sym_of(float s0, float s1, float s2, float s3, float s4) {
  Sym3 m;
  m.zz = s0 * (1.0f / 3.0f);
  m.xx = -s0 * (1.0f / 6.0f) + 0.5f * s3;
  m.yy = -s0 * (1.0f / 6.0f) - 0.5f * s3;
  m.xy = 0.5f * s4;
  m.xz = s1;
  m.yz = s2;
  return m;
}

// symmetric part of A*B for symmetric A, B: (AB + BA)/2
__device__ __forceinline__ Sym3 sym_mul(const Sym3& a, const Sym3& b) {
  Sym3 c;
  c.xx = a.xx * b.xx + a.xy * b.xy + a.xz * b.xz;
  c.yy = a.xy * b.xy + a.yy * b.yy + a.yz * b.yz;
  c.zz = a.xz * b.xz + a.yz * b.yz + a.zz * b.zz;
  const float xy1 = a.xx * b.xy + a.xy * b.yy + a.xz * b.yz;
  const float xy2 = b.xx * a.xy + b.xy * a.yy + b.xz * a.yz;
  const float xz1 = a.xx * b.xz + a.xy * b.yz + a.xz * b.zz;
  const float xz2 = b.xx * a.xz + b.xy * a.yz + b.xz * a.zz;
  const float yz1 = a.xy * b.xz + a.yy * b.yz + a.yz * b.zz;
  const float yz2 = b.xy * a.xz + b.yy * a.yz + b.yz * a.zz;
  c.xy = 0.5f * (xy1 + xy2);
  c.xz = 0.5f * (xz1 + xz2);
  c.yz = 0.5f * (yz1 + yz2);
  return c;
}

// tr(A B) for symmetric A, B
__device__ __forceinline__ float sym_dot(const Sym3& a, const Sym3& b) {
  return a.xx * b.xx + a.yy * b.yy + a.zz * b.zz + 2.0f * (a.xy * b.xy + a.xz * b.xz + a.yz * b.yz);
}

// tr(Q E_m), m = 0..4, for symmetric Q
__device__ __forceinline__ void sym_proj(const Sym3& q, float (&o)[5]) {
  o[0] = (q.zz - 0.5f * (q.xx + q.yy)) * (1.0f / 3.0f);
  o[1] = 2.0f * q.xz;
  o[2] = 2.0f * q.yz;
  o[3] = 0.5f * (q.xx - q.yy);
  o[4] = q.xy;
}

// ----------------------------------------------------------- wave helpers
// Workgroups of one launch are dealt round-robin to the 8 XCDs, each with its
// own L2.  xcd_block() renumbers them so that XCD x runs a contiguous range
// of logical blocks (a bijection for any grid size): blocks that read the
// same structure's data then share one L2 instead of filling all eight.
constexpr int kXCD = 8;
__device__ __forceinline__ int xcd_block_of(int b, int nb) {
  const int q = nb / kXCD, r = nb % kXCD, x = b % kXCD;
  return x * q + min(x, r) + b / kXCD;
}
__device__ __forceinline__ int xcd_block() { return xcd_block_of(blockIdx.x, gridDim.x); }

// ----------------------------------------- groups of 8 lanes (one atom)
// Lane l of a wavefront works on atom l/8; DPP moves data inside the group
// without touching LDS.  DPP reads return 0 from inactive lanes, so these
// helpers are only called where every lane of the wavefront is active.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
constexpr int kDppXor1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppRowRor8 = 0x128;   // within 16-lane rows: lane l takes lane l^8

// sum over the 4 lanes of a quad
__device__ __forceinline__ float quad_sum(float v) {
  v += dpp<kDppXor1>(v);
  v += dpp<kDppXor2>(v);
  return v;
}
// v of lane l ^ 4 inside each row of 16: rotate the row by 12 (lanes with
// bit 2 clear) or by 4 (bit 2 set).  Only the partner lane is read, so this
// is valid in divergent code as long as that partner is active.
constexpr int kDppRowRor4 = 0x124, kDppRowRor12 = 0x12C;
__device__ __forceinline__ float xor4_val(float v) {
  const float hi = dpp<kDppRowRor12>(v), lo = dpp<kDppRowRor4>(v);
  return (threadIdx.x & 4) ? lo : hi;
}
// sum over the 8 lanes of an atom group
__device__ __forceinline__ float grp8_sum(float v) {
  v = quad_sum(v);
  v += dpp<kDppHalfMirror>(v);
  return v;
}
// v + v[lane ^ 16] and v + v[lane ^ 32] with gfx950's lane-swap instructions
// (no LDS): swapping a copy of v with itself leaves one half in each result,
// so every lane gets the same two operands in the same order.
__device__ __forceinline__ float xor16_sum(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xor32_sum(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// sum over the 8 lanes of the wavefront with the same (l & 7)
__device__ __forceinline__ float atoms8_sum(float v) {
  v += dpp<kDppRowRor8>(v);
  return xor32_sum(xor16_sum(v));
}

// ------------------------------------------- reduce-scatter over lane bits
// One butterfly step over a lane bit: values (2w, 2w+1) become one value per
// lane, the even one summed over the pair of lanes where the bit is clear and
// the odd one where it is set, so each step halves the values a lane carries.
template <int CTRL>
struct DppStep {   // lane bit reached by a DPP pattern (xor 1, xor 2, row_ror 8 = xor 8)
  int bit;
  __device__ __forceinline__ float operator()(float e, float o) const {
    const bool hi = (threadIdx.x >> bit) & 1;
    const float send = hi ? e : o;
    return (hi ? o : e) + dpp<CTRL>(send);
  }
};
// lane bit 4 / 5: v_permlane16_swap / v_permlane32_swap exchange the odd
// 16-lane rows (upper 32-lane half) of the first operand with the even rows
// (lower half) of the second, so swap(e, o) leaves every lane with its kept
// value and the partner's copy of it
struct Perm16Step {
  __device__ __forceinline__ float operator()(float e, float o) const {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(e), __float_as_uint(o), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
};
struct Perm32Step {
  __device__ __forceinline__ float operator()(float e, float o) const {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(e), __float_as_uint(o), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
};
template <int V, class Step>
__device__ __forceinline__ void rs_step(const float (&x)[V], float (&y)[(V + 1) / 2], Step st) {
#pragma unroll
  for (int w = 0; w < (V + 1) / 2; ++w) y[w] = st(x[2 * w], 2 * w + 1 < V ? x[2 * w + 1] : 0.f);
}

// Sums of V per-lane values over the 4 pair slots and the 8 atoms of a
// wavefront (lane bits 0, 1, 3, 4, 5; bit 2, the harmonic group, is kept
// apart), scattered: out[r] holds the sum of value 32 r + c, where
// c = b0 + 2 b1 + 4 b3 + 8 b4 + 16 b5 from the lane's bits.  Takes about V / 2
// lane exchanges in all instead of 5 V.
template <int V>
__device__ __forceinline__ void rs_slots_atoms(const float (&x)[V], float (&out)[(V + 31) / 32]) {
  constexpr int V1 = (V + 1) / 2, V2 = (V1 + 1) / 2, V3 = (V2 + 1) / 2, V4 = (V3 + 1) / 2;
  float y1[V1], y2[V2], y3[V3], y4[V4];
  rs_step(x, y1, DppStep<kDppXor1>{0});
  rs_step(y1, y2, DppStep<kDppXor2>{1});
  rs_step(y2, y3, DppStep<kDppRowRor8>{3});
  rs_step(y3, y4, Perm16Step{});
  rs_step(y4, out, Perm32Step{});
}
// Sums of V per-lane values over the 8 lanes of an atom group (lane bits 0,
// 1, 2), scattered: out[r] of lane s holds the sum of value 8 r + s.
struct Xor4Step {
  __device__ __forceinline__ float operator()(float e, float o) const {
    const bool hi = threadIdx.x & 4;
    const float send = hi ? e : o;
    return (hi ? o : e) + xor4_val(send);
  }
};
template <int V>
__device__ __forceinline__ void rs_group8(const float (&x)[V], float (&out)[(V + 7) / 8]) {
  constexpr int V1 = (V + 1) / 2, V2 = (V1 + 1) / 2;
  float y1[V1], y2[V2];
  rs_step(x, y1, DppStep<kDppXor1>{0});
  rs_step(y1, y2, DppStep<kDppXor2>{1});
  rs_step(y2, out, Xor4Step{});
}

// value index c of the lane's first output of rs_slots_atoms
__device__ __forceinline__ int rs_slots_atoms_code() {
  const int l = threadIdx.x;
  return (l & 1) | ((l >> 1) & 1) << 1 | ((l >> 3) & 1) << 2 | ((l >> 4) & 1) << 3 | ((l >> 5) & 1) << 4;
}

// Image shift of a neighbor code: code = 9(sx+1) + 3(sy+1) + (sz+1).
__device__ __forceinline__ void decode_shift(uint32_t code, float& sx, float& sy, float& sz) {
  const int c = (int)code;
  sx = (float)(c / 9 - 1);
  sy = (float)((c / 3) % 3 - 1);
  sz = (float)(c % 3 - 1);
}

}  // namespace nep
