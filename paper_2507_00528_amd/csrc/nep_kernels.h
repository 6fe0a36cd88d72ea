// HIP kernels of the NEP loss-and-gradient path (gfx950, wave64).
//
// Data flow of one loss-and-gradient evaluation:
//   neighbors -> species order -> forward (descriptors, network, partial forces)
//   -> force gather -> per-structure loss and cotangents -> adjoint (tangent
//   pass, network adjoint, parameter partials) -> W0 reduction -> final gradient
//   reduction -> Adam.
// Per-atom kernels run in "species order": atoms grouped by species, each
// group padded to a multiple of 8 atoms, and 8 lanes per atom, so every
// wavefront evaluates one species' network.  Padding atoms have no neighbors
// and write nothing.
#pragma once
#include "nep_device.h"

namespace nep {

enum : int { FL_OVERFLOW = 1, FL_NONFINITE = 2, FL_BOX = 4, FL_TYPE = 8, FL_POS = 16, FL_STEP = 32, FL_BARRIER = 64 };

// ---------------------------------------------------------------- arguments
struct NbrArgs {
  int N, S, T, capR, capA;
  float rcR, rcA;
  const int* aoff;
  const float* box;
  const float* tilt;  // [S][3] (xy, xz, yz), null: every cell orthorhombic
  const float* pos;
  const int* type;
  uint32_t* idxR;
  int* cntR;
  uint32_t* idxA;
  int* cntA;
  int* astruct;
  int* flags;
  // cell-list search of structures of at least cell_min atoms (cells = 0:
  // all-pairs only)
  int cells, cell_min;
  int4* grid;    // [S] bins per axis (na, nb, nc, na nb nc), zero: all-pairs
  int* cell;     // [N+1] bin counts, then bin start offsets; [N] = binned atoms
  int* cpart;    // [N / kScanChunk + 1] per-chunk counts
  int* acell;    // [N] bin id of the atom, -1: all-pairs
  int* aslot;    // [N] slot in the bin
  float4* cpos;  // [N] binned atoms bin by bin (x, y, z, j)
};

struct PairLists {
  const uint32_t* idxR;
  const int* cntR;
  const uint32_t* idxA;
  const int* cntA;
  const int* revR;
  const int* revA;
  int capR, capA;
};

struct FwdArgs {
  int N, Npad, H;
  float inv_rcR, inv_rcA;
  const int* order;
  const int* astruct;
  const float* box;
  const float* tilt;  // null: every cell orthorhombic
  const float* pos;
  const int* type;
  PairLists nb;
  const float* cR;
  const float* cA;
  const float* nn;  // per species block of H*D + 2H + 1
  int nn_stride;
  float* G;        // [D][Npad] species order (may be null)
  float* Guser;    // [D][N] atom order (may be null)
  float* Sst;      // [NA*Y][Npad] (may be null)
  float* Ep;       // [D][Npad] (may be null)
  float* X;        // [H][Npad] (may be null)
  float* eatom;    // [N] atom order (may be null)
  float* eatom2;   // second copy for the caller (may be null)
  float* fR;       // [3][capR][N]
  float* fA;       // [3][capA][N]
  float* wv;       // [6][N]
  int do_mlp, do_force;
};

struct AdjArgs {
  int N, Npad, H, S;
  float inv_rcR, inv_rcA;
  const int* order;
  const int* astruct;
  const float* box;
  const float* tilt;  // null: every cell orthorhombic
  const float* pos;
  const int* type;
  PairLists nb;
  const float* cR;
  const float* cA;
  const float* nn;
  int nn_stride;
  const float* Sst;   // [NA*Y][Npad]
  const float* Ep;    // [D][Npad]
  const float* X;     // [H][Npad]
  const float* eps;   // [S] dL/dE(n)
  const float* fbar;  // [3][N] dL/dF
  const float* wbar;  // [S][6] dL/dW(n)
  float* Gd;          // [D][Npad]
  float* FRst;        // [T*KR][Npad] radial sums F[J][k]
  float* FPst;        // [T*KR][Npad] tangent sums Fp[J][k]
  float* Gbr;         // [NR][Npad] Gbar of the radial descriptors
  float* beta;        // [H][Npad]
  float* w1s;         // [H][Npad]
  float* part;        // [n_waves][PW] wave partial sums
  int PW;
};

// Kernels of the angular degrees l = 5..L3 (nep_highl.h)
struct HighArgs {
  int N, Npad, PW;
  float inv_rcA;
  const int* order;
  const int* astruct;
  const float* box;
  const float* tilt;
  const float* pos;
  const int* type;
  PairLists nb;
  const float* cA;
  float* Sh;          // [Npad][YH][NA] sums S~ of the orthonormal harmonics
  float* Sdh;         // [Npad][YH][NA] their tangents
  float* G;           // [D][Npad] descriptor rows (q_nl of l > 4 written here)
  const float* Ep;    // [D][Npad] dE/dG
  float* Gd;          // [D][Npad] descriptor tangents
  const float* Gb;    // [D][Npad] Gbar (rows of l > 4)
  float* fA;          // [N][capA][3] angular pair forces (added to)
  float* wv;          // [6][N] per-atom virials (added to)
  const float* fbar;  // [3][N]
  const float* wbar;  // [S][6]
  float* part;        // [n_waves][PW] (c^A slots added to)
};

}  // namespace nep
