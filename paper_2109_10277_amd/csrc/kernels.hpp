// Argument blocks and launchers of the libqsp HIP kernels.
#pragma once

#include <vector>

#include "common.hpp"
#include "shape.hpp"

namespace qsp {

// ---------------------------------------------------------------- DST solve
template <typename T>
struct SrcPEZ {             // psi, Ez, Bz sources of slice k
  const double* rho_mjz;    // plasma + beam deposits (ions added here)
  const double* jx;
  const double* jy;
  double n0;
  const double* ionx;       // ion density n0 ionx[i] iony[j]; null: uniform n0
  const double* iony;
  T* out;                   // 3 planes [ny][nx]: psi, Ez, Bz (x-transformed)
};

template <typename T>
struct SrcBxBy {            // Bx, By corrector sources
  const double* jz;         // Jz of slice k (plasma + particle beam)
  const double* jx_prev;    // J_perp of slice k-1
  const double* jy_prev;
  const double* jx_next;    // trial J_perp of slice k+1 (owner planes)
  const double* jy_next;
  const double* sx_next;    // and their shared planes (DepOut::sh)
  const double* sy_next;
  const T* bx;              // current iterate
  const T* by;
  double shift, dzeta;
  double beam_amp;          // Gaussian beam amplitude of slice k (0 = none)
  const double* bgx;        // Gaussian profile factors at the nodes
  const double* bgy;
  T* out;                   // 2 planes: Bx, By (x-transformed)
};

// Planes of FP64 scratch a kernel clears on the side (spread over its grid)
// once their previous readers have finished.
struct ZeroJob {
  double* p[8];
  int count;
  size_t n;                 // elements per plane
};

template <typename T>
struct ColArgs {
  const T* in;              // nfield planes
  T* out;                   // nfield planes
  T* out_dy;                // optional: -d_y of field 0 (nullptr = none)
  double shift[4];          // per field
  int honor_done;           // skip when the P-C has converged
  int w;                    // columns per workgroup (power of two, >= 2)
  ZeroJob zero;
};

// B^(0) = 2 B_{k-1} - B_{k-2} and the opening of a slice's predictor-
// corrector, done on the side of a row pass.
template <typename T>
struct GuessJob {
  T* bx;
  T* by;
  const T* bx1;
  const T* by1;
  const T* bx2;
  const T* by2;
  DevCounters* ctr;         // nullptr = no guess job
  T* tape_bx;               // optional copy of B^0 for the adjoint
  T* tape_by;
};

template <typename T>
struct RowInvArgs {
  const T* in[4];
  T* out[4];
  T* out_dx[4];             // optional -d_x of the result
  GuessJob<T> guess;
  int in_strip, out_strip;  // in / out planes in the strip order of Geom::strip
};

template <typename T>
struct PCArgs {
  const T* in;              // 2 planes from the column pass
  T* bx;                    // iterate, updated in place
  T* by;
  double* partial;          // 2 doubles per workgroup
  double tol;
  T* tape_bx;               // optional copy of the new iterate for the adjoint
  T* tape_by;
};

template <typename T>
void launch_src_fwd_pez(const Geom&, const SrcPEZ<T>&, const AxisTables<T>&, hipStream_t);
template <typename T>
void launch_src_fwd_bxby(const Geom&, const SrcBxBy<T>&, const AxisTables<T>&,
                         const DevCounters*, hipStream_t);
template <typename T>
void launch_col_solve(const Geom&, const ColArgs<T>&, int nfield, const AxisTables<T>&,
                      const double* lamx, const DevCounters*, hipStream_t);
template <typename T>
void launch_row_inv(const Geom&, const RowInvArgs<T>&, int nfield, const AxisTables<T>&,
                    hipStream_t);
template <typename T>
void launch_row_inv_pc(const Geom&, const PCArgs<T>&, const AxisTables<T>&, DevCounters*,
                       hipStream_t);
int pc_partial_count(const Geom&);
// column-strip width of a column pass over nfield planes
template <typename T>
int col_width(const Geom&, int nfield);
// rows per workgroup of the transform row passes (Geom::rr)
template <typename T>
int row_rows(int nx, int ny);

// ---------------------------------------------------------------- particles
template <typename T>
struct Particles {          // SoA, lattice order
  T* xi_x;                  // displacement from the lattice site, in cells
  T* xi_y;
  T* ux;
  T* uy;
  T* psi;
  T* w;                     // density weight n0/(ppc_x ppc_y); 0 = absorbed
  T* hist;                  // [4][5][np], slot s holds f of a slice = s mod 4
  // [5][np] Adams-Bashforth history part ab5_history of the slice the state
  // belongs to (the real push leaves it for the next slice; the first trial
  // push reads it instead of the history).  Null in saved copies of the
  // state (checkpoints, tapes), which restore it from the history.
  T* pab;
};

template <typename T>
struct SliceFields {        // the six fields a particle sees
  const T* exmby;
  const T* eypbx;
  const T* ez;
  const T* bx;
  const T* by;
  const T* bz;
};

// Deposit planes.  With tile histograms and shared planes (sh non-null: the
// trial pushes), a workgroup stores the nodes of its own tile's cells into
// ch with plain stores (every node of the lattice belongs to exactly one
// tile, so ch needs no clearing) and adds its halo nodes and its
// far-travelled particles to sh with atomics; readers take ch + sh.
// Without tiles or shared planes every deposit is an atomic add to ch
// (cleared beforehand).
struct DepOut {
  double* ch[4];            // rho-Jz, Jx, Jy, Jz (rho is formed as (rho - Jz) + Jz)
  double* sh[4];            // shared planes of the same channels (nullable)
};

// kExplicitDep: no push; deposit the explicit Bx/By solver's chi, DJx, DJy
// (dep.ch[0..2]) from the slice-k state in the slice-k psi, Ez, Bz
// kTrialLater: trial push of a later predictor-corrector iteration of the
// slice, from the record the first trial push of the slice left (rec).
// kPushTrialTape: kPushTrial that also copies the slice-k particle state it
// reads into `tape` (slices the reverse pass starts from); a kernel of its
// own so that the untaped trial push keeps its register allocation.
enum PushMode { kPushReal = 0, kPushTrial = 1, kDepositOnly = 2, kExplicitDep = 3, kTrialLater = 4,
                kPushTrialTape = 5 };

// Beam work carried by a real push launch, as workgroups after the plasma
// tiles: the time step of the beam particles of slice k (the slice being
// left) in the push's fields (push_wgs workgroups, 0: none) and the deposit
// of slice k+1's beam particles into dep.ch[0] (rho - Jz) and dep.ch[3] (Jz)
// (dep_wgs workgroups).  Particle ranges come from off (BeamScratch::off).
struct BeamRide {
  float* soa;
  int64_t n;
  const int64_t* off;
  double dt;
  int push_wgs, dep_wgs;
};

template <typename T>
struct PushArgs {
  Particles<T> p;
  SliceFields<T> f;
  DepOut dep;
  int k;                    // slice being left (history ring position)
  double dzeta, hx, hy, psi_floor;
  int tiled;                // 1: LDS tile histograms, 0: direct global atomics
  int tile_rows;            // lattice rows per workgroup tile
  int tile_halo;            // cells of LDS histogram around the tile's own cells
  // end-of-slice bookkeeping of the predictor-corrector (real push only):
  // the slice's iteration count to iters_out (caller) and iters_own
  // (library), the residual to resid_out; pc_budgeted: fewer iterations
  // than pc_max_iter were launched for the slice (a slice left unconverged
  // by them is counted in DevCounters::budget_short)
  int32_t* iters_out;
  int32_t* iters_own;
  double* resid_out;
  int pc_budgeted;
  double pc_tol;
  int pc_max_iter;
  // partial records of the last corrector solve (null: nothing to test);
  // a trial push tests them from its second iteration of a slice on
  const double* pc_partial;
  int pc_nblk;
  int pc_iter;              // trial push: P-C iteration index within the slice
  // trial record (6 planes of np): position at k+1 (x and y offsets), the
  // momentum at k+1 without the Bx/By kick, -w/D at k+1 (0: no deposit),
  // Psi at k+1.  The first trial push of a slice writes it (if non-null),
  // later ones read it.
  T* rec;
  // kPushTrialTape: copy of the slice-k particle state the push reads, 26
  // planes of np in the order xi_x, xi_y, ux, uy, psi, w, hist[4][5]
  T* tape;
  BeamRide beam;            // kPushReal only
};

template <typename T>
void launch_init_plasma(const Lattice&, const Particles<T>&, double w0, hipStream_t);
template <typename T>
void launch_push(const Geom&, const Lattice&, const PushArgs<T>&, PushMode, DevCounters*,
                 hipStream_t);
template <typename T>
void launch_import_state(const Geom&, const Lattice&, const Particles<T>&, const double* x,
                         const double* y, const double* ux, const double* uy,
                         const double* psi, const double* w, const double* hist, int k,
                         double dzeta, hipStream_t);
template <typename T>
void launch_export_state(const Geom&, const Lattice&, const Particles<T>&, double* x,
                         double* y, double* ux, double* uy, double* psi, double* w,
                         double* hist, int k, hipStream_t);

// ------------------------------------------------- explicit Bx/By solver
// Device scalars of the preconditioned conjugate-gradient solve of
// (-lap + chi) B = -R (two systems: 0 Bx, 1 By), in alternating slots by
// iteration parity.
struct ExplicitScalars {
  double bnorm2;            // ||b||^2 of both systems
  double rho[2][2];         // z . r
  double alpha[2][2];
};

template <typename T>
struct ExplicitArgs {
  const double* jz;         // Jz of slice k (plasma + particle beam)
  double beam_amp;          // Gaussian beam Jz = -beam_amp bgx[i] bgy[j]
  const double* bgx;
  const double* bgy;
  const double* chi;        // explicit deposits of slice k
  const double* djx;
  const double* djy;
  T* b[2];                  // Bx, By: initial guess on entry, iterate after each update
  double* x;                // FP64 Krylov vectors, 2 planes each
  double* r;
  double* q;
  double* p[2];             // two buffers (iteration parity) of 2 planes
  const T* col;             // column-pass output, input of the inverse row pass
  T* fwd;                   // forward row-pass output, input of the column pass
  T* z;                     // preconditioned residual
  // per-workgroup partial sums, explicit_partial_count records each
  double* part_s;           // set-up: ||b||^2, ||r0||^2
  double* part_z;           // inverse row pass: z.r, z.q per system
  double* part_m;           // matvec: p.q per system
  double* part_u;           // update: ||r||^2
  ExplicitScalars* s;
  double tol;               // relative residual target (<= 0: run every iteration)
  int it;                   // 0 set-up, m >= 1 iteration m
};

enum ExplicitStep {
  kExplSetup = 0,
  kExplMatvec = 1,
  kExplUpdate = 2,
  kExplRowInv = 3,
  kExplClose = 4
};

template <typename T>
void launch_explicit(const Geom&, const ExplicitArgs<T>&, ExplicitStep, const AxisTables<T>&,
                     DevCounters*, hipStream_t);
int explicit_partial_count(const Geom&);

// ---------------------------------------------------------------- grid utils
void launch_zero(double* p, size_t n, hipStream_t);
template <typename T>
void launch_zero_t(T* p, size_t n, hipStream_t);
template <typename T>
void launch_guess(const Geom&, T* bx, T* by, const T* bx1, const T* by1, const T* bx2,
                  const T* by2, DevCounters*, hipStream_t);
void launch_slice_end(DevCounters*, int32_t* iters_out, int32_t* iters_own, double* resid_out,
                      double tol, int max_iter, int budgeted, const double* pc_partial, int pc_nblk,
                      hipStream_t);

// copy a stored [ny][nx] grid into an [ny+1][nx+1] node array
struct OutCopy {
  const void* src[kMaxOut];
  const double* src2[kMaxOut];  // FP64 plane added to an FP64 source, may be null
  void* dst[kMaxOut];
  int is_double[kMaxOut];   // source precision (the destination matches it)
  int add_beam[kMaxOut];    // add -n_b (Jz, rho outputs of a Gaussian beam)
  int add_ion[kMaxOut];     // add the ion density (rho-Jz, rho outputs)
  int kind[kMaxOut];        // 0 full plane, 1 row ny/2, 2 axis node
  int count;
  double beam_amp, n0;
  const double* ionx;       // ion profile factors (null: uniform n0)
  const double* iony;
  const double* bgx;
  const double* bgy;
};
void launch_out_copy(const Geom&, const OutCopy&, hipStream_t);
void launch_add_current(size_t n, const double* src, double* jz, double* rho, hipStream_t);

template <typename S, typename T>
void launch_from_nodes(const Geom&, const S* src, T* dst, hipStream_t);  // [ny+1][nx+1] -> stored
template <typename T>
void launch_to_nodes(const Geom&, const T* src, double* dst, hipStream_t);    // stored -> [ny+1][nx+1]
template <typename T>
void launch_to_nodes_t(const Geom&, const T* src, T* dst, hipStream_t);

// ---------------------------------------------------------------- beams
struct BeamScratch {
  int* hist;            // [nchunk][nzeta + 1] per-chunk key counts, then their prefixes
  int* total;           // [nzeta + 1] particles per key
  int64_t* off;         // [nzeta + 2] first particle of each key, then n
  int nchunk;           // chunks the scratch holds
};

// Largest key count (nzeta + 1) of the slice sort: its per-chunk counters
// live in 64 KiB of LDS.
constexpr int kMaxBeamKeys = 16384;

// Stable sort of a [7][n] float SoA beam by nearest slice; offsets[k] is the
// first sorted particle of slice k (offsets[nzeta] = particles inside the
// box, offsets[nzeta+1] = n).  Synchronises the stream.
void beam_sort(const float* in, float* out, int64_t n, double zeta_hi, double dzeta, int nzeta,
               BeamScratch& s, std::vector<int64_t>& offsets, hipStream_t st);
int beam_sort_chunks(int64_t n);
// threads of a captured beam launch (per-slice counts at the paper's beam
// sizes stay below this; larger slices are covered by the grid-stride loop)
constexpr int64_t kBeamGraphThreads = 65536;
// Deposit and time step of the particles of slice k: off[k] .. off[k+1]-1
// of the sorted beam (BeamScratch::off, read on the device); the grid is
// sized for grid_count particles and strides over the slice's range.
void launch_beam_deposit(const Geom&, const float* soa, int64_t n, const int64_t* off, int k,
                         int64_t grid_count, double dzeta, double* rho_mjz, double* jz,
                         double* rho, hipStream_t);
template <typename T>
void launch_beam_push(const Geom&, float* soa, int64_t n, const int64_t* off, int k,
                      int64_t grid_count, const SliceFields<T>& f, double dt, hipStream_t);
void launch_zero_int(int* p, size_t n, hipStream_t);

// ---------------------------------------------------------------- adjoint
template <typename T>
struct AdjPushArgs {
  Particles<T> p;           // taped state of slice k
  SliceFields<T> f;         // fields of the push being transposed
  T* lam_y;                 // [5][np]
  T* lam_ring;              // [4][5][np], slot s = adjoint of history slot s
  const T* lsb_x;           // trial: solved adjoint sources of the corrector
  const T* lsb_y;
  double* lam_F[6];         // scatter targets: Ex-By, Ey+Bx, Ez, Bx, By, Bz
  int k;
  double dzeta, hx, hy, psi_floor, inv2dz;
  int tile_rows, tile_halo;   // lattice tiles of the forward push
  // later predictor-corrector iterations: the slice's trial record and the
  // per-particle sums [7][np] of their adjoints that the first iteration's
  // transpose takes up (adjoints of the new x, y offsets, u_x, u_y, Psi and
  // of the slice-k offsets through their own Bx, By); acc_mode 1 stores, 2
  // adds (later iterations), 0 with acc set: the first iteration reads them
  const T* rec;
  T* acc;
  int acc_mode;
};

template <typename T>
struct AdjDepArgs {
  Particles<T> p;
  const double* lam_dep[4]; // rho-Jz, Jx, Jy, Jz
  T* lam_y;
  double psi_floor;
};

template <typename T>
struct AdjSeedArgs {
  const T* cot[7];          // node layout cotangents (QSP_PSI .. QSP_BZ), may be null
  const double* extra[7];   // stored-layout additions, may be null
  double* out[7];
  double* zero[3];          // planes cleared alongside, may be null
};

template <typename T>
struct AdjPCGridArgs {
  const T* lsb_x;
  const T* lsb_y;
  double* lam_jz;
  double* jp_x;
  double* jp_y;
  double* lam_bx;
  double* lam_by;
  double shift, inv2dz;
};

template <typename T>
struct AdjDepGridArgs {
  const T* lpsi;
  const T* lez;
  const T* lbz;
  const double* lam_jz;
  const double* carry_jx;
  const double* carry_jy;
  double* lam_r;
  double* lam_jx;
  double* lam_jy;
  const double* bgx;
  const double* bgy;
  const double* dbgx;
  const double* dbgy;
  double* grad_amp;
  double* grad_sigma;
  double amp;
  int k;
};

template <typename T>
struct AdjSrcArgs {
  const double* p0[3];
  const double* p1[3];
  const double* p2[3];
  double c0[3], c1[3], c2[3];
  T* out[3];
  int count;
};

template <typename T>
struct LossArgs {
  const T* cot[7];
  const T* field[7];
  double* loss;
};

template <typename T, typename U>
struct CopyPlanes {
  const T* src[8];
  U* dst[8];
};

template <typename T>
void launch_adj_push(const Geom&, const Lattice&, const AdjPushArgs<T>&, bool trial, hipStream_t);
template <typename T>
void launch_adj_trial_later(const Geom&, const Lattice&, const AdjPushArgs<T>&, hipStream_t);
template <typename T>
void launch_adj_deposit(const Geom&, const Lattice&, const AdjDepArgs<T>&, hipStream_t);
template <typename T>
void launch_adj_seed(const Geom&, const AdjSeedArgs<T>&, hipStream_t);
template <typename T>
void launch_adj_pc_grid(const Geom&, const AdjPCGridArgs<T>&, hipStream_t);
void launch_adj_guess(size_t n, const double* lam_b0x, const double* lam_b0y, const double* c2x,
                      const double* c2y, double* b1x, double* b1y, double* b2x, double* b2y,
                      hipStream_t);
template <typename T>
void launch_adj_dep_grid(const Geom&, const AdjDepGridArgs<T>&, hipStream_t);
template <typename T>
void launch_adj_source(const Geom&, const AdjSrcArgs<T>&, hipStream_t);
template <typename T>
void launch_loss(const Geom&, const LossArgs<T>&, hipStream_t);
template <typename T>
// copies state and history; where dst keeps the history part P (pab), it
// is formed from the copied state of slice k (step dzeta)
void launch_copy_particles(const Lattice&, const Particles<T>& src, const Particles<T>& dst,
                           int k, double dzeta, hipStream_t);
template <typename T, typename U>
void launch_copy_planes(size_t n, int count, const CopyPlanes<T, U>&, hipStream_t);

}  // namespace qsp
