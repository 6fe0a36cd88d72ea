/*
 * nep.h — C ABI of libnep, an MI355X (gfx950) library for one loss-and-gradient
 * evaluation of a neuroevolution potential (NEP) over a batch of periodic
 * atomic structures, and the Adam step it feeds.
 *
 * Method: Huang, Peng, Li, Zhou, Sun, "Efficient GPU-Accelerated Training of a
 * Neuroevolution Potential with Analytical Gradients" (arXiv 2507.00528).
 * Section and equation numbers below refer to that paper.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Array arguments are DEVICE pointers owned by the caller.  The library never
 *    allocates device memory; scratch space is the caller's workspace `ws`,
 *    whose size comes from nep_workspace_bytes().  `ws` must be 256-byte
 *    aligned and is clobbered by every call that takes it.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  Host-side validation of sizes and pointers runs before any
 *    launch; on a validation error nothing is launched.
 *  - Return value: NEP_OK (0) or a negative NEP_ERR_* code.
 *  - Conditions only the device can see (neighbor overflow, box too small,
 *    a type out of range, a position outside its cell, a non-finite loss) are
 *    OR-ed as NEP_FLAG_* bits into the caller's device word `d_flags`
 *    (int32, may be NULL where the argument is optional).  The caller clears it
 *    and reads it after synchronising; nep_flags_status() maps it to a code.
 *  - Layouts: positions and forces are structure-of-arrays [3*N] (all x, then
 *    all y, then all z).  Virials are per structure, 6 floats in the order
 *    (xx, yy, zz, xy, yz, zx).  Atoms of structure s occupy
 *    [atom_offset[s], atom_offset[s+1]).
 *  - Calls are stateless.  Two calls may run concurrently only with distinct
 *    workspaces and outputs.
 */
#ifndef NEP_H
#define NEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  NEP_OK = 0,
  NEP_ERR_ARG = -1,          /* bad size, NULL pointer or unsupported model   */
  NEP_ERR_BOX = -2,          /* a cell narrower than rc_rad (device flag)     */
  NEP_ERR_NBR_OVERFLOW = -3, /* more neighbors than cap_rad / cap_ang         */
  NEP_ERR_NONFINITE = -4,    /* loss not finite                               */
  NEP_ERR_HIP = -5,          /* a HIP runtime call failed                     */
  NEP_ERR_WORKSPACE = -6,    /* workspace NULL or misaligned                  */
  NEP_ERR_TYPE = -7,         /* an atom type outside [0, n_types)             */
  NEP_ERR_POSITION = -8,     /* an atom outside its cell (device flag)        */
  NEP_ERR_SCRATCH = -9       /* batch too large for nep_loss_grad_noalloc     */
};

#define NEP_FLAG_NBR_OVERFLOW 1
#define NEP_FLAG_NONFINITE 2
#define NEP_FLAG_BOX 4
#define NEP_FLAG_TYPE 8
#define NEP_FLAG_POSITION 16
#define NEP_FLAG_STEP 32   /* a captured step replayed with a step counter below 1 */
#define NEP_FLAG_BARRIER 64   /* the persistent step's grid barrier timed out (its blocks were not all
                                 resident at once); the replay stopped early and wrote no update */

/* NEP hyper-parameters, as counts (Sec. II.B, Appendix A):
 *   n_rad radial channels q_n, n = 0..n_rad-1              (Eq. 5)
 *   k_rad Chebyshev terms per radial function, k = 0..k_rad-1 (Eq. 6)
 *   n_ang, k_ang: the same for the angular radial functions g_n of Eq. 8
 *   l3:  3-body degrees l = 1..l3 of Eq. 7 (0..8 supported)
 *   l4:  0, or 2 for the 4-body invariant tr(M_n^3) of the l = 2 sums
 *   l5:  0, or 1 for the 5-body invariant (sum_m S_n1m^2)^2
 *   hidden: hidden neurons of the per-species tanh network (D1.1)
 *   rc_rad, rc_ang: cutoff radii (Eq. 2, A2.1), rc_ang <= rc_rad
 *   cap_rad, cap_ang: neighbor-list capacity per atom
 * Supported: up to 4 species, n_rad <= 12, n_ang <= 8, k_rad and k_ang <= 12,
 * l3 <= 8, l4 and l5 on or off (and the LDS of the chosen kernels within a
 * gfx950 workgroup's 160 KiB, which bounds hidden).  A few shapes are
 * compiled exactly; any other runs in the smallest compiled size class that
 * holds it, with its parameters zero-padded on the device (exact: padded
 * quantities contribute zeros).  nep_model_supported() tells. */
typedef struct {
  int32_t n_types, n_rad, n_ang, k_rad, k_ang, l3, l4, l5, hidden;
  float rc_rad, rc_ang;
  int32_t cap_rad, cap_ang;
} nep_model;

/* A batch of periodic structures (device pointers).  Cell of structure n:
 * edge vectors a = (Lx, 0, 0), b = (xy, Ly, 0), c = (xz, yz, Lz), the
 * image shift s = (sa, sb, sc) moving an atom by sa a + sb b + sc c (Eq. 2).
 *   atom_offset [n_struct+1] int32, atom_offset[0] = 0, last = n_atom
 *   box   [n_struct*3] float edge lengths (Lx, Ly, Lz)
 *   pos   [3*n_atom] float SoA
 *   type  [n_atom] int32 species in [0, n_types)
 *   tilt  [n_struct*3] float (xy, xz, yz), or NULL when every cell is
 *         orthorhombic (all tilts zero).
 *   max_atoms  host value: 0, or an upper bound on the atoms of any one
 *         structure.  It only selects kernels: structures of at least 1024
 *         atoms in cells wide enough are searched through cell lists, and
 *         structures of at least 2048 atoms are summed per 1024-atom chunk; a
 *         bound below those sizes skips the corresponding kernels.  No result
 *         depends on it beyond the order of floating-point sums; a negative
 *         value is NEP_ERR_ARG.
 * Orthorhombic cell (all three tilts zero): each L >= rc_rad and each
 * coordinate in [0, L).  Triclinic cell: each perpendicular width (cell
 * volume over the area of the opposite face) >= rc_rad / (1 - 2e-5) and the
 * fractional coordinates of every atom in [-1e-5, 1 + 1e-5).  Cells that
 * break these raise NEP_FLAG_BOX / NEP_FLAG_POSITION (the image set
 * {-1,0,1}^3 then no longer covers every neighbor). */
typedef struct {
  int32_t n_struct, n_atom;
  const int32_t* atom_offset;
  const float* box;
  const float* pos;
  const int32_t* type;
  const float* tilt;
  int32_t max_atoms;
} nep_batch;

/* Neighbor lists (Eq. 2), one for rc_rad and one for rc_ang (device).
 *   idx_*  [n_atom*cap] uint32, entry k of atom i at [i*cap + k] (each atom's
 *          list contiguous):
 *          (j << 5) | code, j the global atom index (< 2^27) and
 *          code = 9(sx+1) + 3(sy+1) + (sz+1) for the image shift s in {-1,0,1}^3
 *   cnt_*  [n_atom] int32, number of neighbors (may exceed cap: overflow)
 * Each list is in canonical order: j ascending, then code ascending. */
typedef struct {
  uint32_t* idx_rad;
  int32_t* cnt_rad;
  uint32_t* idx_ang;
  int32_t* cnt_ang;
} nep_neighbors;

/* Training labels (device): per-structure total energies [n_struct], forces
 * SoA [3*n_atom], per-structure total virials [n_struct*6]. */
typedef struct {
  const float* energy;
  const float* force;
  const float* virial;
} nep_labels;

/* Number of trainable parameters.  Packing of the flat float vector:
 *   c_rad[I][J][n][k]  (T*T*n_rad*k_rad; I = type of the center, J = type of
 *                       the neighbor, Eq. 6)
 *   c_ang[I][J][n][k]  (T*T*n_ang*k_ang, Eq. 8)
 *   per species I: W0[hidden][n_desc] (row = hidden unit), b0[hidden],
 *                  w1[hidden], b1                     (D1.1)
 * Returns a negative code for an invalid model. */
int64_t nep_param_count(const nep_model* model);

/* Length of the descriptor vector G_i (Eqs. 5, 7): n_rad + n_ang*l3
 * (+ n_ang if l4) (+ n_ang if l5), in the order [q_n][q_nl, l outer, n inner]
 * [4-body q_n][5-body q_n]. */
int32_t nep_descriptor_count(const nep_model* model);

/* NEP_OK if the model runs (an exact compiled shape or a size class that
 * holds it, see nep_model), else NEP_ERR_ARG. */
int nep_model_supported(const nep_model* model);

/* Bytes of workspace needed for a batch of n_struct structures, n_atom atoms. */
int nep_workspace_bytes(const nep_model* model, int32_t n_struct, int32_t n_atom, size_t* bytes);

/* Neighbor lists of Eq. 2 under periodic boundaries: all (j, s) != (i, 0)
 * with |x_j + s*L - x_i| < rc, s in {-1,0,1}^3, for rc_rad and rc_ang.  The
 * predicate is evaluated in IEEE float64 as d = (x_j - x_i) + s*L and
 * d2 = (dx*dx + dy*dy) + dz*dz < rc*rc without fused multiply-add, so the
 * lists are bit-reproducible.  Sets NEP_FLAG_NBR_OVERFLOW, _BOX, _TYPE,
 * _POSITION in d_flags (required).  Also prepares workspace state that the
 * other calls on this batch read (species order, reverse entries).
 * Structures of at least 1024 atoms in cells at least 3 (rc_rad + 0.05)
 * wide are searched through cell lists (see nep_batch.max_atoms); the lists
 * are the same bit for bit. */
int nep_build_neighbors(const nep_model* model, const nep_batch* batch, nep_neighbors* out,
                        void* ws, int32_t* d_flags, void* stream);

/* Descriptors G [n_desc*n_atom], entry v of atom i at [v*n_atom + i]
 * (Eqs. 5-8, Appendices A-B), for lists from nep_build_neighbors on the same
 * workspace. */
int nep_descriptors(const nep_model* model, const nep_batch* batch, const nep_neighbors* nbrs,
                    const float* params, float* G, void* ws, void* stream);

/* Per-atom energies e_atom [n_atom] (Eq. 1), per-structure energies
 * e_struct [n_struct], forces [3*n_atom] (Eq. 3: F_i = sum_j dE_i/dr_ij -
 * dE_j/dr_ji, gathered without atomics) and per-structure virials
 * [n_struct*6] (Eq. 4 summed over atoms: W = -sum_pairs f_ij (x) r_ij).
 * Any output may be NULL. */
int nep_energy_force_virial(const nep_model* model, const nep_batch* batch, const nep_neighbors* nbrs,
                            const float* params, float* e_atom, float* e_struct, float* force,
                            float* virial, void* ws, void* stream);

/* Vector-Jacobian product: grad [P] (overwritten) = e_bar . dE(n)/dtheta
 * + f_bar . dF/dtheta + v_bar . dW(n)/dtheta, given cotangents e_bar
 * [n_struct], f_bar [3*n_atom] SoA and v_bar [n_struct*6] (the chain of
 * Eqs. 13-16 and D1.18-D1.21 with arbitrary cotangents).  Recomputes the
 * forward state it needs; nothing per pair is stored. */
int nep_vjp(const nep_model* model, const nep_batch* batch, const nep_neighbors* nbrs,
            const float* params, const float* e_bar, const float* f_bar, const float* v_bar,
            float* grad, void* ws, void* stream);

/* Loss of Eqs. 9-12 and its gradient (Eqs. 13-16, D1.18-D1.21):
 *   L = lambda[0]*Le + lambda[1]*Lf + lambda[2]*Lv,
 *   Le = 1/S sum_n ((E(n) - E_tar(n))/N_n)^2,
 *   Lf = 1/(3N) sum (F - F_tar)^2,
 *   Lv = 1/(6S) sum_n sum_c ((W_c(n) - W_tar_c(n))/N_n)^2.
 * loss [4] = (L, Le, Lf, Lv), zeros for an empty batch; grad [P] overwritten.  e_struct, force, virial
 * (may be NULL) receive the predictions.  Sets NEP_FLAG_NONFINITE. */
int nep_loss_grad(const nep_model* model, const nep_batch* batch, const nep_neighbors* nbrs,
                  const float* params, const nep_labels* labels, const float lambda[3],
                  float* loss, float* grad, float* e_struct, float* force, float* virial,
                  void* ws, int32_t* d_flags, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the neighbor build
 * and loss-and-gradient evaluation of nep_build_neighbors() followed by
 * nep_loss_grad() on one workspace, with the workspace replaced by a static
 * device array of NEP_STATIC_SCRATCH_BYTES that the library holds on each GPU
 * it runs on until the process ends.  Arguments and outputs as in those two
 * calls (nbrs receives the lists; d_flags is required).  No call allocates
 * memory.  NEP_ERR_SCRATCH when nep_workspace_bytes() of the batch exceeds
 * NEP_STATIC_SCRATCH_BYTES (64 MiB: about 18,000 atoms of the 3/4/5-body
 * model with hidden 50, or 21,000 of the 3-body model with hidden 30).  The
 * array is shared by every call on the same GPU and keeps the last call's
 * contents; calls that overlap on one GPU (other streams or threads) race and
 * must be serialised by the caller.  The stream must belong to the current
 * device. */
#define NEP_STATIC_SCRATCH_BYTES (64u << 20)
int nep_loss_grad_noalloc(const nep_model* model, const nep_batch* batch, nep_neighbors* nbrs,
                          const float* params, const nep_labels* labels, const float lambda[3],
                          float* loss, float* grad, float* e_struct, float* force, float* virial,
                          int32_t* d_flags, void* stream);

/* One bias-corrected Adam step on P parameters (the optimizer of Sec. I):
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   params -= lr * (m/(1-b1^step)) / (sqrt(v/(1-b2^step)) + eps);
 * step is 1-based.  NEP_ERR_ARG for step < 1, beta1 or beta2 outside [0, 1),
 * a negative or non-finite eps or a non-finite lr. */
int nep_adam_step(int64_t P, float* params, float* m, float* v, const float* grad, float lr,
                  float beta1, float beta2, float eps, int32_t step, void* stream);

/* Learning rate of Eq. 17 at step s (host scalar helper). */
float nep_lr_schedule(int64_t s, float lr_start, float lr_stop, int64_t n_warmup, int64_t n_total);

/* Inference path (outside the training step): n_steps of velocity Verlet
 * with the NEP forces, in eV, A, fs and amu.  Each step kicks the velocities
 * by half a step with `force`, moves and wraps the positions into the cell
 * (into [0, L) per axis when orthorhombic; by the lattice vector of the
 * floored fractional coordinates when triclinic), rebuilds the neighbor lists, evaluates E and F (Eqs. 1-3) and kicks again.
 *   pos     must be batch->pos; advanced in place (device, SoA [3*n_atom])
 *   mass    [n_types] atomic masses in amu (device)
 *   vel     [3*n_atom] SoA velocities in A/fs, updated (device)
 *   force   [3*n_atom] SoA forces at the current positions on entry (from
 *           nep_energy_force_virial or the previous call), at the final
 *           positions on return (device)
 *   e_pot   [n_struct] potential energies at the final positions (device)
 *   e_kin   [n_struct] kinetic energies at the final velocities, or NULL
 *   ws      a workspace that already holds this batch's neighbor build
 *   d_flags device flag word (required; see nep_build_neighbors)
 * Returns NEP_ERR_ARG for a NULL or mismatched pointer, n_steps < 0 or a
 * non-finite dt. */
int nep_md_step(const nep_model* model, const nep_batch* batch, float* pos, nep_neighbors* nbrs,
                const float* params, const float* mass, float* vel, float* force, float dt, int32_t n_steps,
                float* e_pot, float* e_kin, void* ws, int32_t* d_flags, void* stream);

/* A whole training step — neighbors, forward, loss, adjoint, gradient and
 * Adam — recorded once as a HIP graph and replayed by
 * nep_train_step_graph_launch().  All pointers are captured: their contents
 * may change between replays, their addresses may not.  The step counter
 * (1-based, for Adam's bias correction) lives in `d_step` [1] int32 on the
 * device and is advanced by each replay; the learning rate of each replay
 * follows Eq. 17 with (lr_start, lr_stop, n_warmup, n_total), or stays at
 * lr_start when n_total <= 0.  loss [4] and d_flags describe the latest replay.
 * A replay whose neighbor build or loss raised any flag (overflow, box, type,
 * position, non-finite loss) or whose step counter is below 1 (NEP_FLAG_STEP)
 * writes grad but leaves params, m and v unchanged; a non-finite gradient
 * entry raises NEP_FLAG_NONFINITE and leaves its own parameter unchanged.
 * Returns NEP_ERR_ARG for beta1 or beta2 outside [0, 1), a negative or
 * non-finite eps, a non-finite learning rate or n_warmup < 0.
 * Returns an opaque handle in *graph. */
typedef struct {
  float lr_start, lr_stop;
  int64_t n_warmup, n_total;
  float beta1, beta2, eps;
} nep_adam_config;

/* graph_flags bit NEP_GRAPH_CACHED_NEIGHBORS: the graph leaves out the neighbor
 * build (lists, reverse index and species order) and reuses what an earlier
 * nep_build_neighbors() call with the same nbrs and ws produced.  Training
 * positions never change, so this is the step with cached lists. */
#define NEP_GRAPH_CACHED_NEIGHBORS 1

/* graph_flags bit NEP_GRAPH_PERSISTENT: everything after the neighbor build
 * (species order, forward, force gather, per-structure sums and loss of
 * Eqs. 9-12, adjoint, gradient reductions and Adam) runs as one persistent
 * launch whose phases are separated by a software grid barrier, in place of
 * about ten separate launches.  The grid takes as many blocks as are resident
 * at once.  Same results as the separate launches up to the order of
 * floating-point sums.  NEP_ERR_ARG for triclinic batches (tilt != NULL),
 * empty batches and models with 3-body degrees l > 4; the caller then uses
 * the separate launches.  A barrier wait beyond 2 s raises NEP_FLAG_BARRIER. */
#define NEP_GRAPH_PERSISTENT 2

int nep_train_step_graph_create(const nep_model* model, const nep_batch* batch, nep_neighbors* nbrs,
                                const nep_labels* labels, const float lambda[3], float* params,
                                float* m, float* v, float* grad, float* loss, int32_t* d_step,
                                const nep_adam_config* adam, void* ws, int32_t* d_flags,
                                int32_t graph_flags, void* stream, void** graph);
/* Launch choices of the captured step, picked per batch size class by the
 * library's autotuner (paper_2507_00528_amd/tune.py) from timed replays; none
 * changes a result beyond the order of floating-point sums.  0 in a field
 * keeps the default (in brackets).
 *   persistent      1: the persistent form of NEP_GRAPH_PERSISTENT [0]
 *   outer_blocks_w  blocks per species of the W0 outer-product sum, 1..512 [192]
 *   outer_blocks_c  blocks per species of the c_rad outer-product sum, 1..256 [64]
 *   reduce_chunks   chunks per species of the first gradient-partial reduction, 1..512 [128]
 *   cell_min_atoms  smallest structure searched through cell lists, >= 64 [1024]
 *   gather_lanes    lanes per atom of the force gather, 8 or 16 [16]
 *   forward_waves   wavefronts per SIMD the forward kernel is compiled for, 2 or 3 [3]
 *   adjoint_waves   the same for the adjoint kernel [3; 2 with degrees l > 4]
 *   reverse_branch  where the reverse index of the lists runs: 1 in the launch
 *                   that also counts the species order, 2 on a branch of its
 *                   own that overlaps the species order and the forward pass
 *                   and joins before the force gather [1]
 * A value out of range is NEP_ERR_ARG. */
typedef struct {
  int32_t persistent, outer_blocks_w, outer_blocks_c, reduce_chunks, cell_min_atoms, gather_lanes,
      forward_waves, adjoint_waves, reverse_branch;
} nep_tuning;

/* nep_train_step_graph_create() with launch choices (tuning may be NULL). */
int nep_train_step_graph_create_tuned(const nep_model* model, const nep_batch* batch, nep_neighbors* nbrs,
                                      const nep_labels* labels, const float lambda[3], float* params,
                                      float* m, float* v, float* grad, float* loss, int32_t* d_step,
                                      const nep_adam_config* adam, void* ws, int32_t* d_flags,
                                      int32_t graph_flags, const nep_tuning* tuning, void* stream,
                                      void** graph);
int nep_train_step_graph_launch(void* graph, void* stream);
int nep_train_step_graph_destroy(void* graph);

/* Per-kernel timing of one unfused loss-and-gradient pass (the same launches
 * nep_loss_grad makes, each bracketed by HIP events on `stream`).  Writes up
 * to max_kernels durations in milliseconds into ms[] and the matching kernel
 * names (static strings) into names[]; *n_kernels receives the count.
 * Synchronises the stream. */
int nep_profile_loss_grad(const nep_model* model, const nep_batch* batch, nep_neighbors* nbrs,
                          const float* params, const nep_labels* labels, const float lambda[3],
                          float* loss, float* grad, void* ws, int32_t* d_flags, void* stream,
                          float* ms, const char** names, int32_t max_kernels, int32_t* n_kernels);

/* Map a flag word read back from the device to the first matching error code
 * (NEP_OK when clear). */
int nep_flags_status(int32_t flags);

/* Human-readable message for a status code. */
const char* nep_status_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* NEP_H */
