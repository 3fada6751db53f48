// Internal structures of libgbsmpo: the device-resident state of one
// simulation, the per-layer workspace, and the kernel launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "common.h"

namespace gbs {

// Sets the thread-local message returned by mpo_last_error; returns code.
int set_error(int code, const char *msg);

// Sweep limit of the one-sided Jacobi of every block SVD.
constexpr int JACOBI_MAX_SWEEPS = 60;

// One beam splitter of a batched layer.
struct GateParam {
  int site;        // acts on modes (site, site + 1)
  int inst;        // instance (index into Layer::states)
  double theta, phi;
  long long fock0; // first entry of the gate's Fock table
  long long mir0;  // first entry of the gate's mirror maps (chi of the instance)
  long long blk0;  // first block descriptor of the gate (set per chunk)
  long long lst0;  // first entry of the gate's list regions (set per chunk)
  long long ct0;   // first entry of the gate's centre-bond run table
};

// One charge sector Theta(q) of one gate (App. D, Eq. theta).
struct BlkDesc {
  int q;          // packed new centre charge
  int r, s;       // rows (left-bond indices), cols (right-bond indices)
  int m, n;       // stored SVD operand is m x n column-major, m = max(r, s)
  int t;          // 1 when the stored operand is Theta^T (r < s)
  int mirror;     // local index of the block of the mirrored charge, -1 if none
  int sweeps;     // Jacobi sweeps used
  int len;        // singular values >= rank cut
  int kq;         // singular vectors kept
  int boff;       // first new-bond index of this block
  int uoff;       // first unit (selection) index owned by this block
  long long eoff; // operand offset (local to the gate) in the A and A0 pools
  double fro2;    // squared Frobenius norm of the operand
  int big;        // 1: SVD by multi-workgroup panel rounds, 0: one workgroup in LDS
  int w, npan;    // panel width and panel count of a big block
  int bigi;       // index of a big block in its gate's big-block list
  int svoff;      // offset of the n singular values / permutation
  int roff, coff; // offsets of the row / column index lists
  int gate;       // gate index inside the layer
  int comp;       // 1: contracted and SVD'd here; 0: derived from its mirror block
  int qr;         // 1: Householder QR first, the Jacobi runs on X = R^H (n x n)
  int mj;         // rows of the Jacobi operand (n with QR, else m)
  long long joff; // offset of R (local to the gate) in the R pool
};

// Per-gate plan totals (device -> host).
struct GateTot {
  int nblk, sv, rows, cols, maxr, maxc, sym;
  int nbig, maxpp;    // big blocks, largest even panel count among them
  long long elems;
  long long relems;   // R factors of the QR'd blocks (sum of n^2)
  int c0lo, c0hi, c1hi;  // centre bond: range of n, largest n' (-1: empty bond)
  double svd_flops;   // sum over blocks of 16 m n^2 + 36 n^3 (complex SVD convention)
  double contr_flops; // algorithmic Theta contraction flops of the gate (no padding,
                      // no mirror saving): centre-charge sums + factorised Fock weights
};

// Per-gate global offsets (host -> device).
struct GateBase {
  long long e;        // first operand element of the gate in the A / A0 pools
  int blk;            // first block (flat over the layer)
  int big;            // first big block (flat over the layer)
  long long r;        // first element of the gate in the R pool
};

// Device-resident state of one simulation (App. D Vidal form with charges).
struct State {
  int M, d, chi;
  cd *gam;          // M site matrices chi x chi, row-major, leading dim chi
  double *lam;      // (M+1) x chi Schmidt values
  int *chg;         // (M+1) x chi packed charges, sorted, CHARGE_NONE padded
  int *dim;         // (M+1) bond sizes
  double *ee;       // (M+1) operator EE per bond (bits)
  unsigned long long *ee_max;  // running max of EE (double bits)
  int *err;         // latched error bits
  int max_sweeps;   // Jacobi sweep limit of this simulation (JACOBI_MAX_SWEEPS
                    // unless lowered by the failure-injection hook)
};

// Workspace of one chunk of a batched layer: gates of one or many instances.
struct Layer {
  int ngates;
  const State *states;   // device table of instance states
  GateParam *gates;
  cd *fock;          // ngates x (2d-1) x d x d, [n][i1][j1]
  BlkDesc *blk;      // per-gate regions at GateParam::blk0
  int box_cap;       // largest admissible charge box per gate
  GateTot *tot;      // ngates
  GateBase *base;    // ngates
  int *rows, *cols;  // per-gate row / column index lists (at lst0)
  int *mirL, *mirR;  // per gate: mirror index on the left / right bond, -1 if none (at mir0)
  int *runs;         // per block (at 64 x the flat block index): row / column runs by charge
  int *ctab;         // per gate (at ct0): first centre-bond index with charge >= (c0lo + x, y),
                     // [x][y] for x in [0, c0hi - c0lo + 2), y in [0, c1hi + 2)
  cd *A;             // sector operands (overwritten by U * Sigma)
  cd *A0;            // pristine copies of the operands (right-vector recovery)
  cd *R;             // X = R^H of QR'd blocks, n x n (rotated by the Jacobi)
  cd *tau;           // Householder scalars (n per computed block, at lst0 + svoff)
  int *piv;          // QR column pivots (n per computed block, at lst0 + svoff)
  cd *U;             // kept left singular vectors of QR'd blocks (at the A offset)
  cd *V;             // conjugated kept right singular vectors of QR'd blocks (at the R offset)
  int *bigl;         // per gate: local indices of its big blocks (at lst0)
  int *rotf;         // per big block: rotation flags of the two latest sweeps
  int *active;       // [0] big blocks still rotating at the latest check, [1] their tasks
  int *task_blk;     // flat indices of the still-rotating big blocks
  int *task_pre;     // first panel task of each (task_pre[nact] = all tasks)
  int *qr_order;     // total_blocks: launch order of the QR workgroups (largest first)
  int *big_order;    // total_big: big blocks by operand rows, largest first (panel tasks)
  int *pver;         // per big block: panel versions and pair verification records
                     // (panel_version_ints() each)
  int nact, ntask;   // host copies of active[0], active[1] for the panel launches
  int total_big;     // big blocks in the layer
  int maxpp;         // largest even panel count in the layer
  int panel_lds;     // LDS bytes of one panel workgroup
  int mixed;         // 1: FP32 Jacobi (mixed-precision path), FP64 elsewhere
  int esz;           // bytes per Jacobi operand element in LDS (16, or 8 when mixed)
  double *sv;        // singular values, sorted descending per block
  int *perm;         // rank -> operand column
  unsigned long long *uval;   // selection units: value bits
  unsigned long long *ukey;   // selection units: tie key
  int *usize;                 // selection units: size (1 or 2)
  int total_blocks;
};

// ---------------- launch wrappers (one translation unit each) ----------------
// initial state
hipError_t launch_init_rho(const double *r, const int *nint, double eta, int M, int d,
                           double *rho, hipStream_t s);
hipError_t launch_init_norms(const double *rho, int M, int d, double *A, hipStream_t s);
hipError_t launch_init_conv(const double *rho, int M, int d, int b, const long long *woff,
                            double *w, hipStream_t s);
// total photon cap K >= 0 (K < 0: none): left weights V (M+1) x (K+1)^2
hipError_t launch_init_left(const double *rho, int M, int d, int K, double *V, hipStream_t s);
hipError_t launch_init_select(State st, const double *w, const long long *woff,
                              const double *A, unsigned long long *uval,
                              unsigned long long *ukey, int *usize, long long ucap,
                              const double *V, int K, hipStream_t s);
hipError_t launch_init_gamma(State st, const double *rho, const double *A, const double *V, int K,
                             hipStream_t s);

// one batched layer (chunk)
hipError_t launch_fock(Layer ly, hipStream_t s);
hipError_t launch_plan_count(Layer ly, hipStream_t s);
hipError_t launch_plan_fill(Layer ly, hipStream_t s);
hipError_t launch_ctab(Layer ly, hipStream_t s);
hipError_t launch_contract(Layer ly, int max_chi, int max_d, hipStream_t s);
hipError_t launch_qr(Layer ly, int max_chi, hipStream_t s);
hipError_t launch_leftvec(Layer ly, int max_chi, hipStream_t s);
hipError_t launch_svd_small(Layer ly, hipStream_t s);
hipError_t launch_svd_big_prep(Layer ly, hipStream_t s);
hipError_t launch_svd_panel_step(Layer ly, int step, hipStream_t s);
int svd_max_steps(Layer ly);
int panel_version_ints();
int panel_lds_bytes(int max_chi);
hipError_t launch_svd_count(Layer ly, int last, int next_step, hipStream_t s);
hipError_t launch_svd_big_finish(Layer ly, int sweeps_run, int max_chi, hipStream_t s);
hipError_t launch_select(Layer ly, hipStream_t s);
hipError_t launch_scatter(Layer ly, int max_chi, hipStream_t s);
hipError_t launch_entropy_layer(Layer ly, hipStream_t s);
int svd_lds_bytes();
void set_svd_route(int lds_limit_bytes, int qr_enable);

// readouts
hipError_t launch_entropy_all(State st, hipStream_t s);
hipError_t launch_renyi(State st, double alpha, double *out, hipStream_t s);
hipError_t launch_asym(double r, double mu, int nmax, double theta, int n_inputs, double alpha,
                       double *X, double *spec, double *out, int *err, hipStream_t s);
hipError_t launch_phases(State st, const double *phase, hipStream_t s);
size_t marginals_scratch(int M, int d, int chi);   // doubles
hipError_t launch_marginals(State st, cd *envL, cd *envR, double *part, double *P,
                            double *trace, hipStream_t s);
// marginals on the library's static scratch array (no allocation)
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
size_t marginals_noalloc_bytes(int M, int d, int chi);
hipError_t noalloc_scratch_init();    // once per device, with that device current
// enqueues the marginal kernels on the scratch array; *P (M*d raw marginals)
// and *trace receive the device addresses of the results inside it
hipError_t launch_marginals_noalloc(State st, double **P, double **trace, hipStream_t s);

}  // namespace gbs
