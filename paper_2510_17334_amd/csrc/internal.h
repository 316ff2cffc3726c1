// Internal declarations shared by the host orchestrator and the HIP kernels.
//
// Block-vector layout ("panel layout"): the complex vectors of a batch of
// systems are grouped in panels of 16 systems; element (row i, slot t) lives at
// complex index ((t / 16) * n + i) * 16 + t % 16.  A 16-lane group of a wave
// reads one row of a panel as one contiguous segment (128 B for complex float,
// 256 B for complex double), so every gather of the shifted SpMM is a
// coalesced row read.
//
// Dense real blocks used by Rayleigh-Ritz are row-major n x ld internally (the
// ABI is column-major; entry points transpose once on the way in and out).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace slrf {

constexpr int kPanel = 16;      // systems per panel
constexpr int kMaxRestart = 32; // GCR(m) with m <= 32
constexpr int kMaxPoles = 64;   // poles per handle
constexpr int kThreads = 256;   // workgroup size of the block-vector kernels

// Device view of the pencil (shared CSR pattern).
struct DevPencil {
  int n = 0, nnz = 0;
  const int* rowptr = nullptr;
  const int* col = nullptr;
  const double* a = nullptr;  // FP64 values (caller-owned)
  const double* b = nullptr;
  const float* a32 = nullptr; // FP32 copies (library-owned)
  const float* b32 = nullptr;
  const double* da = nullptr; // diag(A), diag(B) (library-owned)
  const double* db = nullptr;
  int max_nnz_sub64 = 0;      // max nonzeros in an aligned block of 64 / 32 rows
  int max_nnz_sub32 = 0;      // (LDS staging plan of the shifted SpMM; 0 = unknown)
  // Row-group ("union") format: groups of 4 consecutive rows, the union of
  // their columns once per group and 4 coefficients of A and of B per union
  // entry ([entry][4]); optional (gptr == nullptr: CSR kernels only).
  const int* gptr = nullptr;  // [ngroups + 1]
  const int* gcol = nullptr;  // [nunion]
  const double* gca = nullptr;
  const double* gcb = nullptr;
  const float* gca32 = nullptr;
  const float* gcb32 = nullptr;
  int grp_lds_ent = 0;        // max union entries of 8 consecutive groups
  // Halo-tile format (optional, hx_ntile == 0: absent): rows cut into tiles of
  // whole 8-row slices whose referenced columns (the tile's halo, sorted)
  // number at most kHaloMaxH; entry j of row r is stored at
  // hx_sptr[r / 8] * 8 + (j / 4) * 32 + (r % 8) * 4 + j % 4 (groups of 4
  // entries per row) with its column as a halo position.
  int hx_ntile = 0, hx_hmax = 0, hx_emax = 0;  // tiles, largest halo, most entries of a pass
  const int* hx_trow = nullptr;   // [ntile + 1] first row of each tile
  const int* hx_hptr = nullptr;   // [ntile + 1] halo offsets
  const int* hx_halo = nullptr;   // halo rows of all tiles
  const int* hx_sptr = nullptr;   // [nslice + 1] slice offsets (steps of 8 entries)
  const int* hx_slen = nullptr;   // [nslice * 8] row lengths
  const unsigned short* hx_lcol = nullptr;
  const float2* hx_ab32 = nullptr;   // (a, b) per entry
  const double2* hx_ab64 = nullptr;
  // Row-group format of the wave-uniform sweep (ug_ngroups == 0: absent):
  // groups of ug_R consecutive rows, per group the sorted distinct columns
  // with the mask of the rows that use them and ug_R (a, b) pairs each
  int ug_R = 0, ug_ngroups = 0;
  const int* ug_gptr = nullptr;   // [ngroups + 1]
  const int* ug_ent = nullptr;    // column | mask << 28
  const float2* ug_ab32 = nullptr;
  const double2* ug_ab64 = nullptr;
  // SpMM kernel choice per sweep precision (kSpmm*; chosen by the autotuner)
  int var32 = 0, var64 = 0;
};
// SpMM variants: 0 = row-group format if present, else CSR staged in LDS;
// 1 = row-group format; 2, 4, 5 = CSR staged in LDS with 8, 16, 32 gathers in
// flight per lane; 3 = CSR read directly; 6 = halo tiles (gathered operand
// staged in LDS) for plain sweeps, CSR staged in LDS (16 in flight) for the
// sweeps fused with the CGS projections
constexpr int kSpmmAuto = 0, kSpmmGroup = 1, kSpmmCsrLds = 2, kSpmmCsrDirect = 3,
              kSpmmCsrLds16 = 4, kSpmmCsrLds32 = 5, kSpmmHalo = 6, kSpmmUGroup = 7;
constexpr int kSpmmVariants = 8;
// Largest halo of a tile (rows of 128 bytes in LDS; with the staged
// coefficients of the tile four workgroups fit a CU) and the rows of a tile
// (one 8-row slice per wave of a 256-thread workgroup: a tile is formed in one
// pass).
#ifndef SLRF_HALO_MAXH
#define SLRF_HALO_MAXH 224
#endif
constexpr int kHaloMaxH = SLRF_HALO_MAXH;
constexpr int kHaloTileRows = 32;
// Units (128-byte panel column slices) per workgroup: a tile's coefficients
// are staged once for all of them.  On the 3D Q1 benchmark pencil (80 panels)
// 16 to 40 units run the halo sweeps and the up-step 2-4 % faster than 8, 4
// units 12 % slower; 16 keeps workgroups for small pencils and batches.
#ifndef SLRF_HALO_G
#define SLRF_HALO_G 16
#endif
constexpr int kHaloMaxG = SLRF_HALO_G;

// A rectangular real CSR matrix on the device (AMG prolongation / restriction).
struct DevTransfer {
  int nrows = 0, ncols = 0, nnz = 0;
  int max_sub64 = 0;  // most entries in an aligned block of 64 rows
  const int* rowptr = nullptr;
  const int* col = nullptr;
  const double* v = nullptr;
  const float* v32 = nullptr;
};

// Launch geometry of the panel kernels: a grid of (row block, panel) tiles.
struct PanelGrid {
  int rpb = 512;   // rows per workgroup
  int nrb = 0;     // row blocks
  int npan = 0;    // panels covered by the launch
  int group = 8;   // panels that share a row block before moving on (CSR reuse)
  int C = 0;       // slot capacity (stride of per-slot arrays)
  int ND = 0;      // stride of the partial-sum buffer (values per row block)
  unsigned blocks() const {
    long total = (long)nrb * npan;
    long per = (total + 7) / 8;
    return (unsigned)(per * 8);
  }
};

// Per-slot tables of the resident systems.
struct SlotTables {
  const int* sys = nullptr;        // system id (c * N + j) or -1
  const double2* sigma = nullptr;  // pole of the slot
  const int* col = nullptr;        // column of X / F
  const double* theta = nullptr;   // warm-start Ritz value of the column
  const int* src = nullptr;        // compaction source slot (-1 = newly admitted)
  int* active = nullptr;           // 1 while the slot iterates in the current cycle
  // scratch of the coarsest-level solve: the active slots grouped by pole
  // (plist, C entries) and each group's start (poff, kMaxPoles + 1 entries)
  int* plist = nullptr;
  int* poff = nullptr;
};

// ----- shifted block kernels (inner precision T = float or double) -----
// Wave-uniform row-group sweep (variant 7): true when selected for T.
template <typename T>
bool ugroup_selected(const DevPencil& P);
// Operator sweep on the row-group format: epi 0 Out = M Z, 1 (kEpiResidOp)
// Out = Bin - M Z, 2 (kEpiJacobiOp) Out = Z + omega D^-1 (Bin - M Z); false
// when the pencil's kernel choice for T is another variant (nothing launched).
template <typename T>
bool launch_ugroup(const DevPencil& P, const PanelGrid& g, const SlotTables& st, int epi,
                   double omega, const void* Z, const void* Bin, void* Out, hipStream_t s,
                   hipError_t& err);
// True when the pencil's operator sweeps for T run on the halo-tile kernel
// (then the GCR apply is a plain sweep followed by a separate projection pass).
template <typename T>
bool sweep_is_halo(const DevPencil& P);
// Plain operator sweep Out = M Z of the active slots (no projections).
template <typename T>
hipError_t launch_sweep(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                        const void* Z, void* Out, hipStream_t s);
// CGS projections h_i = <q_i, q_k>, i < k, as partial sums per row block.
// hq: the stored q_i are complex bfloat16 (complex float, k <= 8): slot i at
// Qbase + i * vstride elements holds lane pair (panel, row, lane) at 8-byte
// index (panel * n + row) * 8 + lane.
template <typename T>
hipError_t launch_dots(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                       const void* Qk, const void* Qbase, size_t vstride, int k, double2* part,
                       hipStream_t s, bool hq = false);
template <typename T>
hipError_t launch_apply_dots(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                             const void* Z, void* Qk, const void* Qbase, size_t vstride, int k,
                             double2* part, bool precond, hipStream_t s);
// CGS update of the new image only, q_k -= sum_i beta_i q_i, with the partial
// sums of <q_k, q_k> and <q_k, r> (the directions p_i are never formed: the
// solution update combines the stored preconditioned vectors z_i instead)
// The image w is read from Qk; q_k goes to Qout (may be Qk) when store is set
// (a cycle's last q_k is never read again); hq as for launch_dots, with q_k
// rounded to complex bfloat16 before its partial sums are taken.
template <typename T>
hipError_t launch_orth(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                       const void* Qk, const void* R, const void* Qbase, size_t vstride, int k,
                       const double2* beta, double2* part, hipStream_t s, void* Qout,
                       bool store, bool hq);
template <typename T>
// precond: 0 = none (z = r), 1 = point Jacobi, 2 = leave z to the AMG V-cycle,
// 3 = Z receives omega D^-1 r, the level-0 pre-smoothing of the next V-cycle,
// 4 = the same stored as complex bfloat16 (complex-float sweeps);
// Z may be null (no z written: the last step of a cycle); hq: Qk holds q_k as
// complex bfloat16 (layout as for launch_dots)
hipError_t launch_step(const DevPencil& P, const PanelGrid& g, const SlotTables& st, void* R,
                       void* Z, const void* Qk, const double2* alpha_k, double2* part,
                       int precond, double omega, hipStream_t s, bool hq = false);
// FP64 solution update of a finished cycle: y += sum_j g_j z_j, where the
// coefficients g follow from alpha and the CGS history beta (p_k = z_k -
// sum_{i<k} beta_ik p_i); z_0 in Z0, z_j (j >= 1) at Zbase + j * vstride.
template <typename T>
hipError_t launch_yupdate(int n, const PanelGrid& g, const SlotTables& st, double2* Y,
                          const void* Z0, const void* Zbase, size_t vstride, int kk,
                          const double2* alpha, const double2* bhist, hipStream_t s);
template <typename T>
hipError_t launch_true_resid(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                             const double2* Y, const double* F, int ldf, void* R, void* Z,
                             double2* part, int precond, hipStream_t s);
template <typename T>
hipError_t launch_admit(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                        const double2* Yold, const void* Rold, const void* Zold, double2* Ynew,
                        void* Rnew, void* Znew, const double* F, const double* E,
                        const double* X, int ld, bool warm, double2* part, int precond,
                        hipStream_t s);
template <typename T>
hipError_t launch_spmm_panel(const DevPencil& P, const PanelGrid& g, const double2* sigma_slot,
                             const void* Z, void* Q, hipStream_t s);

// ----- AMG V-cycle pieces (level vectors in panel layout, rows = level size) -----
constexpr int kEpiResidOp = 1, kEpiJacobiOp = 2;  // level-operator epilogues
template <typename T>
hipError_t launch_lvl_op(const DevPencil& L, const PanelGrid& g, const SlotTables& st, int epi,
                         double omega, const void* X, const void* Bin, void* Out, hipStream_t s);
template <typename T>
hipError_t launch_lvl_jacobi0(const DevPencil& L, const PanelGrid& g, const SlotTables& st,
                              double omega, const void* Bin, void* Out, hipStream_t s,
                              bool out_bf16 = false);
template <typename T>
hipError_t launch_transfer(const DevTransfer& M, const PanelGrid& g, const SlotTables& st,
                           const void* In, void* Out, bool add, hipStream_t s);
template <typename T>
hipError_t launch_coarse_solve(int nc, const PanelGrid& g, const SlotTables& st, int npoles,
                               const void* Minv, const void* In, void* Out, hipStream_t s);

// Fine-level image of the level-0 prolongator P for the fused up-step of the
// V-cycle: (A P, B P) in the halo-tile format (rows: fine rows in 32-row
// tiles; halo: coarse rows) with P's values per entry (zero where P has none).
struct DevImage {
  int nc = 0;                                 // coarse rows (columns of P)
  int ntile = 0, hmax = 0, emax = 0;          // ntile == 0: not built
  const int* trow = nullptr;
  const int* hptr = nullptr;
  const int* halo = nullptr;
  const int* sptr = nullptr;
  const unsigned short* lcol = nullptr;
  const float2* ab32 = nullptr;
  const double2* ab64 = nullptr;
  // P's own entries on the image tiles (its nonzeros only, same halo positions)
  int pemax = 0;
  const int* psptr = nullptr;
  const unsigned short* plcol = nullptr;
  const float* p32 = nullptr;
  const double* p64 = nullptr;
};
constexpr int kImgMaxH = 64;    // coarse-halo cap of an image tile's first layout attempt
constexpr int kImgMaxH2 = 128;  // the cap of the second attempt (fewer, wider tiles fail less)

// Level-0 up-step in one pass: with x = x0 + P e (e the coarse correction),
// Out = x + omega D^-1 (r1 - (A P - sigma B P) e), where r1 = b - M x0 is the
// residual the down-step formed; equal (to rounding) to prolongation followed
// by the damped-Jacobi post-smoothing sweep.  Returns false (nothing
// launched) when the pencil has no image.
template <typename T>
bool launch_post_image(const DevImage& I, const DevPencil& P, const PanelGrid& g,
                       const SlotTables& st, double omega, const void* E, const void* X0,
                       const void* R1, void* Out, hipStream_t s, hipError_t& err,
                       bool r1_bf16 = false);
// Level-0 residual r1 = b - M x on the halo tiles stored as complex bfloat16
// (x_bf16: the iterate x is complex bfloat16 too)
// (4 bytes per entry, panel layout): r1 is only restricted and read by the
// up-step, where the preconditioner tolerates its rounding.  Complex-float
// sweeps only; returns false (nothing launched) otherwise.
template <typename T>
bool launch_resid_bf16(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                       const void* X, const void* Bin, void* Out, hipStream_t s,
                       hipError_t& err, bool x_bf16 = false);
// Restriction of a complex-bfloat16 panel vector (complex-float results).
template <typename T>
hipError_t launch_restrict_bf16(const DevTransfer& M, const PanelGrid& g, const SlotTables& st,
                                const void* In, void* Out, hipStream_t s);

hipError_t launch_retire(int n, const PanelGrid& g, const int* retire_sys, const double2* Y,
                         double2* Ystore, hipStream_t s);
hipError_t launch_filter_sum(int n, int ncols, int npoles, const double2* Ystore,
                             const double2* w, double* Ur, hipStream_t s);

// ----- second-stage reductions and per-slot scalar updates -----
hipError_t launch_reduce(const double2* part, int nrb, int ND, int C, int nd, int nslots,
                         double2* out, hipStream_t s);
struct SlotScalars {
  double2* beta = nullptr;   // [kMaxRestart][C]
  double2* bhist = nullptr;  // [kMaxRestart (step k)][kMaxRestart (i < k)][C] beta of the cycle
  double2* alpha = nullptr;  // [kMaxRestart][C]
  double* qq = nullptr;      // [kMaxRestart][C]
  double* target2 = nullptr; // [C] squared residual target of the current cycle
  double* fnorm2 = nullptr;  // [ncols] squared column norms of F
  int* sys_its = nullptr;    // [S]
  double* sys_rn2 = nullptr; // [S] last FP64 squared residual norm
  int* status = nullptr;     // [C] 0 continue, 1 converged, 2 capped, 3 numeric, -1 empty
};
hipError_t launch_fin_beta(const double2* red, int k, int C, int nslots, const SlotTables& st,
                           const SlotScalars& sc, hipStream_t s);
hipError_t launch_fin_alpha(const double2* red, int k, int C, int nslots, const SlotTables& st,
                            const SlotScalars& sc, hipStream_t s);
hipError_t launch_fin_rnorm(const double2* red, int nslots, const SlotTables& st,
                            const SlotScalars& sc, int itcap, hipStream_t s);
hipError_t launch_fin_true(const double2* red, int nslots, const SlotTables& st,
                           const SlotScalars& sc, double tol, double inner_rtol, double safety,
                           int itcap, hipStream_t s);

// ----- real dense / sparse kernels for Rayleigh-Ritz (row-major blocks) -----
// launch_spmm_real on the pencil's complex-double halo tiles; false (nothing
// launched) where the tiles are absent or nc, ld or the alignment of X do not fit.
bool launch_spmm_real_halo(const DevPencil& P, const double* X, int ld, int nc, double* AX,
                           double* BX, const double* theta, double* E, hipStream_t s,
                           hipError_t& err);
hipError_t launch_spmm_real(const DevPencil& P, const double* X, int ld, int nc, double* AX,
                            double* BX, const double* theta, double* E, hipStream_t s);
// out[c * ldout + omap(r)] = in[r * ldin + imap(c)]; maps optional (NULL = identity)
hipError_t launch_transpose(const double* in, int rows, int cols, int ldin, double* out,
                            int ldout, hipStream_t s, const int* imap = nullptr,
                            const int* omap = nullptr);
// G (p x q, row-major, ldg) = X^T Y; X: n x p (ldx), Y: n x q (ldy); part:
// scratch of gram_part_doubles(n, pq) doubles for any p, q <= pq
hipError_t launch_gram(int n, int p, int q, const double* X, int ldx, const double* Y, int ldy,
                       double* part, double* G, int ldg, hipStream_t s);
size_t gram_part_doubles(int n, int pq);
// Z (n x q, ldz) = alpha * X (n x p, ldx) * S (p x q, lds) + beta * Z
hipError_t launch_gemm_tall(int n, int p, int q, double alpha, const double* X, int ldx,
                            const double* S, int lds, double beta, double* Z, int ldz,
                            hipStream_t s);
// per column c: out[c] = sum_r (X - theta_c Y)[r,c]^2 (theta NULL => X only) and
// out2[c] = sum_r W[r,c] * Y[r,c] (W NULL => skipped)
hipError_t launch_colstats(int n, int nc, const double* X, const double* Y, int ld,
                           const double* theta, const double* W, double* part, int nchunk,
                           double* out, double* out2, hipStream_t s);
int colstat_chunks(int n);
// grad[e] = sum_i glam_i x_{i,e}^T (dA_e - lam_i dB_e) x_{i,e}; nd in {4, 8, 24}
hipError_t launch_eig_grad(int n, int k, const double* X, const double* lam, const double* glam,
                           int nelem, int nd, const int* dofs, const double* dA, int sa,
                           const double* dB, int sb, double* grad, hipStream_t s);
hipError_t launch_cast_f32(const double* in, float* out, size_t cnt, hipStream_t s);
hipError_t launch_diag(const DevPencil& P, double* da, double* db, int* missing, hipStream_t s);

}  // namespace slrf
