// One layer of disjoint beam splitters on the U(1) Vidal MPO (App. D).
//
// For a gate on modes (j, j+1) the bonds are L = j, C = j+1, R = j+2.  A new
// centre charge q gives the sector block (App. D, Eq. theta)
//   Theta(q)[a, b] = lam_L[a] lam_R[b] sum_alpha W(c_a, c_alpha, c_b, q)
//                    Gamma_j[a, alpha] lam_C[alpha] Gamma_{j+1}[alpha, b],
// rows a with c_a - q in [0,d)^2, columns b with q - c_b in [0,d)^2, and
//   W = U[n][i][j] conj(U[n'][i'][j'])        (Sec. II, U (x) conj(U)),
// where (n, n') = c_a - c_b are the photons on the two modes, (i, i') =
// c_a - q the new and (j, j') = c_a - c_alpha the old photons of mode j.
// Every block is SVD'd (App. D: block-wise SVD of all Theta(c)), the chi
// largest singular values over all blocks are kept under the mirror-pair rule,
// and Gamma~_j = V / lam_L, Gamma~_{j+1} = W^dag / lam_R (App. D).
//
// Kernels, in launch order: k_fock (Fock tables), k_plan (sector planning),
// k_ctab + k_contract (Theta blocks), k_qr_panel / k_qr (pivoted QR),
// k_svd_small and the panel rounds (one-sided Jacobi: k_panel_gram in FP64,
// k_panel in the mixed mode), k_big_finish,
// k_select (truncation), k_leftvec (kept vectors of QR'd blocks), k_zero +
// k_scatter (new tensors), k_entropy_layer (EE of the new bonds).
#include <math.h>

#include "blockops.h"
#include "internal.h"

namespace gbs {

// ----------------------------------------------------------------------------
// Fock beam-splitter tables by the creation-operator recursion: with
// U a1^dag U^dag = T11 a1^dag + T21 a2^dag and U a2^dag U^dag = T12 a1^dag +
// T22 a2^dag, the block of total photon number n follows from block n-1:
//   B_n[i][j] = (T11 sqrt(i) B_{n-1}[i-1][j-1] + T21 sqrt(n-i) B_{n-1}[i][j-1]) / sqrt(j)
//   B_n[i][0] = (T12 sqrt(i) B_{n-1}[i-1][0]   + T22 sqrt(n-i) B_{n-1}[i][0])   / sqrt(n)
// where i, j count photons in mode 1 of the output / input.  Stored entries
// are those with both modes inside the cutoff: tab[n][i][j], i, j, n-i, n-j < d.
// ----------------------------------------------------------------------------
__global__ void k_fock(Layer ly) {
  const int g = blockIdx.x;
  const GateParam gp = ly.gates[g];
  const int d = ly.states[gp.inst].d;
  const int nmax = 2 * d - 2;
  const int W = nmax + 1;
  __shared__ cd s_b[2][32 * 32];
  const double ct = cos(gp.theta), st = sin(gp.theta);
  const cd T11 = cmk(cos(gp.phi) * ct, sin(gp.phi) * ct);
  const cd T21 = cmk(cos(gp.phi) * st, sin(gp.phi) * st);
  const cd T12 = cmk(-st, 0.0);
  const cd T22 = cmk(ct, 0.0);
  cd *tab = ly.fock + gp.fock0;
  for (int i = threadIdx.x; i < W * d * d; i += blockDim.x) tab[i] = cmk(0.0, 0.0);
  if (threadIdx.x == 0) s_b[0][0] = cmk(1.0, 0.0);
  __syncthreads();
  if (threadIdx.x == 0) tab[0] = cmk(1.0, 0.0);
  for (int n = 1; n <= nmax; ++n) {
    const cd *prev = s_b[(n - 1) & 1];
    cd *cur = s_b[n & 1];
    for (int idx = threadIdx.x; idx < (n + 1) * (n + 1); idx += blockDim.x) {
      const int i = idx / (n + 1), j = idx % (n + 1);
      cd acc = cmk(0.0, 0.0);
      if (j >= 1) {
        if (i >= 1) cfma(acc, cscale(T11, sqrt((double)i)), prev[(i - 1) * 32 + (j - 1)]);
        if (i <= n - 1) cfma(acc, cscale(T21, sqrt((double)(n - i))), prev[i * 32 + (j - 1)]);
        acc = cscale(acc, 1.0 / sqrt((double)j));
      } else {
        if (i >= 1) cfma(acc, cscale(T12, sqrt((double)i)), prev[(i - 1) * 32]);
        if (i <= n - 1) cfma(acc, cscale(T22, sqrt((double)(n - i))), prev[i * 32]);
        acc = cscale(acc, 1.0 / sqrt((double)n));
      }
      cur[i * 32 + j] = acc;
      if (i < d && n - i < d && j < d && n - j < d) tab[((size_t)n * d + i) * d + j] = acc;
    }
    __syncthreads();
  }
}

hipError_t launch_fock(Layer ly, hipStream_t s) {
  hipLaunchKernelGGL(k_fock, dim3(ly.ngates), dim3(256), 0, s, ly);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Sector planning: one workgroup per gate.  New centre charges q lie in the
// box [lo0, hi0] x [lo1, hi1] spanned by the outer bonds; for each q the
// block has r = #{a : c_a - q in [0,d)^2} rows and s = #{b : q - c_b in [0,d)^2}
// columns, counted with binary searches on the sorted bonds.  Non-empty
// blocks are compacted in charge order, offsets assigned, row / column index
// lists written and each block's mirror (n', n) located.
// ----------------------------------------------------------------------------
__device__ inline int count_window(const int *c, int D, int n, int lo, int hi) {
  if (hi < lo || n < 0) return 0;
  lo = max(lo, 0);
  if (hi < lo) return 0;
  return lower_bound(c, D, pack_charge(n, hi + 1)) - lower_bound(c, D, pack_charge(n, lo));
}

constexpr int RUNS_PER_BLOCK = 64;   // 4 tables of up to 16 (d <= 16) per block

// LDS bytes of the one-workgroup Jacobi (operand + column norms) and the
// widest panel whose pair (2 w columns of m rows) fits in LDS.
__host__ __device__ inline size_t svd_small_need(int m, int n, int esz) {
  return (size_t)esz * m * n + sizeof(double) * (size_t)n;
}
// Panel width of an n-column operand of m rows: the fewest panels (an even
// count when more than one, so that no panel idles in a round) whose pair
// (2 w columns of m elements of esz bytes) fits in lds_bytes, at most 32
// columns each, and then the narrowest width giving that count.
__host__ __device__ inline int panel_width(int m, int n, int lds_bytes, int esz) {
  int wmax = (int)min((size_t)32, (size_t)lds_bytes / (2 * (size_t)m * esz));
  if (wmax < 1) wmax = 1;
  int np = (n + wmax - 1) / wmax;
  if (np > 1 && (np & 1)) ++np;
  return (n + np - 1) / np;
}

// Panel width of the FP64 panel rounds (Gram form, k_panel_gram): the columns
// stream from global memory, so only the 32 columns of a panel pair's Gram
// bound the width: the fewest panels of at most 16 columns (even count when
// more than one), then the narrowest width giving that count.
__host__ __device__ inline int gram_panel_width(int n) {
  int np = (n + 15) / 16;
  if (np > 1 && (np & 1)) ++np;
  return (n + np - 1) / np;
}

// Route of a computed block's SVD.  A block with at least 16 columns, or
// whose operand does not fit in LDS, is first reduced by a Householder QR,
// A = Q R, and the Jacobi rotates the n x n operand X = R^H: its columns are
// far closer to orthogonal than those of A (the Jacobi needs about half the
// sweeps) and the work per sweep drops by m / n.  The Jacobi runs in one
// workgroup from LDS when its operand fits there, otherwise as
// multi-workgroup panel rounds.
#ifndef GBS_QR_MIN_COLS
#define GBS_QR_MIN_COLS 16
#endif
constexpr int QR_MIN_COLS = GBS_QR_MIN_COLS;

// In FP64 (esz 16) a block of at least GBS_GRAM_MIN_COLS columns also takes
// the panel rounds (in Gram form) even when it would fit the one-workgroup
// Jacobi: its many dependent rounds on one workgroup would otherwise form a
// chain of their own beside the panel rounds that run anyway.
#ifndef GBS_GRAM_MIN_COLS
#define GBS_GRAM_MIN_COLS 48
#endif
__host__ __device__ inline void svd_route(int m, int n, int lds_bytes, int qr_ok, int esz,
                                          int &qr, int &big, int &mj) {
  qr = 0;
  mj = m;
  if (qr_ok && (svd_small_need(m, n, esz) > (size_t)lds_bytes || n >= QR_MIN_COLS)) {
    qr = 1;
    mj = n;
  }
  big = (svd_small_need(mj, n, esz) > (size_t)lds_bytes || (esz == 16 && n >= GBS_GRAM_MIN_COLS))
            ? 1 : 0;
}

// Two passes over the charge box of every gate.  The count pass (FILL =
// false) builds the mirror maps, decides whether the gate may use Hermiticity
// and totals the sizes the fill pass needs; the host then places every gate's
// regions and the fill pass (FILL = true) writes the block descriptors, the
// offsets and the row / column lists.  With Hermiticity a block with n > n'
// is derived from its mirror (its mirror exists because both outer bonds are
// mirror symmetric).
template <bool FILL>
__global__ __launch_bounds__(1024) void k_plan(Layer ly, int lds_bytes, int qr_ok) {
  const int panel_lds = ly.panel_lds;
  const int g = blockIdx.x;
  const GateParam gp = ly.gates[g];
  const State st = ly.states[gp.inst];
  const int d = st.d, chi = st.chi;
  const int j = gp.site;
  const int *cL = st.chg + (size_t)j * chi;
  const int *cR = st.chg + (size_t)(j + 2) * chi;
  const int DL = st.dim[j], DR = st.dim[j + 2];
  int *mirL = ly.mirL + gp.mir0;
  int *mirR = ly.mirR + gp.mir0;
  const double *lamL = st.lam + (size_t)j * chi;
  const double *lamR = st.lam + (size_t)(j + 2) * chi;
  __shared__ int s_sym;
  __shared__ int s_min1L, s_max1L, s_min1R, s_max1R, s_max1C;
  __shared__ long long s_scan[17];
  __shared__ int s_iscan[17];
  if (threadIdx.x == 0) {
    s_min1L = 1 << 30; s_max1L = -1; s_min1R = 1 << 30; s_max1R = -1; s_max1C = -1;
    s_sym = 1;
  }
  __syncthreads();
  if (!FILL) {
    // Mirror index maps.  The mirror of index a (charge (n, n'), rank k inside
    // its charge run) is the index of charge (n', n) with the same rank.  The
    // gate uses Hermiticity only when both outer bonds are exactly mirror
    // symmetric (same charges, bitwise equal Schmidt values).
    for (int a = threadIdx.x; a < DL; a += blockDim.x) {
      const int c = cL[a];
      const int cm = pack_charge(charge_np(c), charge_n(c));
      const int am = lower_bound(cL, DL, cm) + (a - lower_bound(cL, DL, c));
      const bool ok = am < DL && cL[am] == cm && lamL[am] == lamL[a];
      mirL[a] = ok ? am : -1;
      if (!ok) s_sym = 0;
    }
    for (int b = threadIdx.x; b < DR; b += blockDim.x) {
      const int c = cR[b];
      const int cm = pack_charge(charge_np(c), charge_n(c));
      const int bm = lower_bound(cR, DR, cm) + (b - lower_bound(cR, DR, c));
      const bool ok = bm < DR && cR[bm] == cm && lamR[bm] == lamR[b];
      mirR[b] = ok ? bm : -1;
      if (!ok) s_sym = 0;
    }
  }
  {
    int mn = 1 << 30, mx = -1;
    for (int a = threadIdx.x; a < DL; a += blockDim.x) {
      mn = min(mn, charge_np(cL[a]));
      mx = max(mx, charge_np(cL[a]));
    }
    atomicMin(&s_min1L, mn);
    atomicMax(&s_max1L, mx);
    mn = 1 << 30; mx = -1;
    for (int b = threadIdx.x; b < DR; b += blockDim.x) {
      mn = min(mn, charge_np(cR[b]));
      mx = max(mx, charge_np(cR[b]));
    }
    atomicMin(&s_min1R, mn);
    atomicMax(&s_max1R, mx);
    if (!FILL) {
      const int DC = st.dim[j + 1];
      const int *cC = st.chg + (size_t)(j + 1) * chi;
      mx = -1;
      for (int c = threadIdx.x; c < DC; c += blockDim.x) mx = max(mx, charge_np(cC[c]));
      atomicMax(&s_max1C, mx);
    }
  }
  __syncthreads();
  const int sym = FILL ? ly.tot[g].sym : s_sym;
  GateTot tot = {};
  tot.sym = sym;
  {
    const int DC = st.dim[j + 1];
    const int *cC = st.chg + (size_t)(j + 1) * chi;
    tot.c0lo = DC > 0 ? charge_n(cC[0]) : 0;
    tot.c0hi = DC > 0 ? charge_n(cC[DC - 1]) : -1;
    tot.c1hi = DC > 0 ? s_max1C : -1;
  }
  if (DL == 0 || DR == 0) {
    if (!FILL && threadIdx.x == 0) ly.tot[g] = tot;
    return;
  }
  const int minL0 = charge_n(cL[0]), maxL0 = charge_n(cL[DL - 1]);
  const int minR0 = charge_n(cR[0]), maxR0 = charge_n(cR[DR - 1]);
  const int lo0 = max(max(minL0 - (d - 1), minR0), 0), hi0 = min(maxL0, maxR0 + d - 1);
  const int lo1 = max(max(s_min1L - (d - 1), s_min1R), 0), hi1 = min(s_max1L, s_max1R + d - 1);
  const int W0 = hi0 - lo0 + 1, W1 = hi1 - lo1 + 1;
  if (W0 <= 0 || W1 <= 0) {
    if (!FILL && threadIdx.x == 0) ly.tot[g] = tot;
    return;
  }
  const long long area = (long long)W0 * W1;
  if (area > (1LL << 26)) {
    if (!FILL && threadIdx.x == 0) {
      atomicOr(st.err, ERR_BOX_OVERFLOW);
      ly.tot[g] = tot;
    }
    return;
  }
  BlkDesc *blk = ly.blk + gp.blk0;
  // pass 1: the non-empty blocks in charge order (counted, or compacted)
  long long nb = 0, eb = 0, reb = 0;
  int svb = 0, rb = 0, cb = 0, bgb = 0, maxr = 0, maxc = 0, maxpp = 0;
  double fl = 0.0;
  for (long long c0 = 0; c0 < area; c0 += blockDim.x) {
    const long long cell = c0 + threadIdx.x;
    int r = 0, s = 0;
    int q0 = 0, q1 = 0;
    if (cell < area) {
      q0 = lo0 + (int)(cell / W1);
      q1 = lo1 + (int)(cell % W1);
      for (int n = q0; n <= q0 + d - 1; ++n) r += count_window(cL, DL, n, q1, q1 + d - 1);
      if (r > 0)
        for (int n = max(q0 - d + 1, 0); n <= q0; ++n)
          s += count_window(cR, DR, n, q1 - d + 1, q1);
    }
    const long long flag = (r > 0 && s > 0) ? 1 : 0;
    if (!FILL) {
      if (flag) {
        const bool comp = !(sym && q0 > q1);
        const int m = max(r, s), n = min(r, s);
        rb += r;
        cb += s;
        maxr = max(maxr, r);
        maxc = max(maxc, s);
        if (comp) {
          eb += (long long)r * s;
          svb += n;
          fl += 16.0 * m * (double)n * n + 36.0 * (double)n * n * n;
          int qr, big, mj;
          svd_route(m, n, lds_bytes, qr_ok, ly.esz, qr, big, mj);
          if (qr) reb += (long long)n * n;
          if (big && 2LL * mj * ly.esz > panel_lds) atomicOr(st.err, ERR_WORKSPACE);
          if (big) {
            ++bgb;
            const int w = ly.mixed ? panel_width(mj, n, min(lds_bytes, panel_lds), ly.esz)
                                   : gram_panel_width(n);
            const int np = (n + w - 1) / w;
            maxpp = max(maxpp, np + (np & 1));
          }
        }
      }
      nb += flag;
    } else {
      long long total;
      const long long pos = nb + block_exclusive_scan<long long>(flag, s_scan, total);
      if (flag) {
        BlkDesc B = {};
        B.q = pack_charge(q0, q1);
        B.r = r;
        B.s = s;
        B.t = r < s;
        B.m = max(r, s);
        B.n = min(r, s);
        B.gate = g;
        blk[pos] = B;
      }
      nb += total;
    }
  }
  if (!FILL) {
    // algorithmic contraction work of the gate: 8 flops per (a, alpha, b)
    // term of the centre-charge sums (c_a - c_alpha and c_alpha - c_b valid
    // local pairs), plus the Fock weights applied factorised per (a, b):
    // m_ket m_bra (m_ket + m_bra) complex MACs, m = valid splits of the
    // two-mode photon number
    double cf = 0.0;
    {
      const int DC = st.dim[j + 1];
      const int *cC = st.chg + (size_t)(j + 1) * chi;
      for (int al = threadIdx.x; al < DC; al += blockDim.x) {
        const int p0 = charge_n(cC[al]), p1 = charge_np(cC[al]);
        int nl = 0, nr = 0;
        for (int n = p0; n <= p0 + d - 1; ++n) nl += count_window(cL, DL, n, p1, p1 + d - 1);
        for (int n = max(p0 - d + 1, 0); n <= p0; ++n)
          nr += count_window(cR, DR, n, p1 - d + 1, p1);
        cf += 8.0 * nl * (double)nr;
      }
      for (int a = threadIdx.x; a < DL; a += blockDim.x) {
        // right indices with 0 <= c_a0 - c_b0 <= 2d - 2: one range of the sorted bond
        const int ca0 = charge_n(cL[a]), ca1 = charge_np(cL[a]);
        const int b0 = lower_bound(cR, DR, pack_charge(max(ca0 - 2 * d + 2, 0), 0));
        const int b1 = lower_bound(cR, DR, pack_charge(ca0 + 1, 0));
        for (int b = b0; b < b1; ++b) {
          const int n0 = ca0 - charge_n(cR[b]), n1 = ca1 - charge_np(cR[b]);
          if (n1 < 0 || n1 > 2 * d - 2) continue;
          const int mk = min(n0, 2 * d - 2 - n0) + 1, mb = min(n1, 2 * d - 2 - n1) + 1;
          cf += 8.0 * mk * mb * (double)(mk + mb);
        }
      }
    }
    // block-wide totals
    __shared__ long long s_nb, s_eb, s_re;
    __shared__ int s_sv, s_rb, s_cb, s_bg, s_mr, s_mc, s_pp;
    __shared__ double s_fl, s_cf;
    if (threadIdx.x == 0) {
      s_nb = 0; s_eb = 0; s_re = 0; s_sv = 0; s_rb = 0; s_cb = 0; s_bg = 0; s_mr = 0; s_mc = 0;
      s_pp = 0; s_fl = 0.0; s_cf = 0.0;
    }
    __syncthreads();
    atomicAdd((unsigned long long *)&s_nb, (unsigned long long)nb);
    atomicAdd((unsigned long long *)&s_eb, (unsigned long long)eb);
    atomicAdd((unsigned long long *)&s_re, (unsigned long long)reb);
    atomicAdd(&s_sv, svb);
    atomicAdd(&s_rb, rb);
    atomicAdd(&s_cb, cb);
    atomicAdd(&s_bg, bgb);
    atomicMax(&s_mr, maxr);
    atomicMax(&s_mc, maxc);
    atomicMax(&s_pp, maxpp);
    atomicAdd(&s_fl, fl);
    atomicAdd(&s_cf, cf);
    __syncthreads();
    if (threadIdx.x == 0) {
      tot.nblk = (int)s_nb;
      tot.sv = s_sv;
      tot.rows = s_rb;
      tot.cols = s_cb;
      tot.maxr = s_mr;
      tot.maxc = s_mc;
      tot.elems = s_eb;
      tot.relems = s_re;
      tot.nbig = s_bg;
      tot.maxpp = s_pp;
      tot.svd_flops = s_fl;
      tot.contr_flops = s_cf;
      ly.tot[g] = tot;
    }
    return;
  }
  __syncthreads();
  const int nblk = (int)nb;
  // mirror block by binary search on the sorted charges
  for (int bi = threadIdx.x; bi < nblk; bi += blockDim.x) {
    BlkDesc &B = blk[bi];
    const int qm = pack_charge(charge_np(B.q), charge_n(B.q));
    int lo = 0, hi = nblk;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (blk[mid].q < qm) lo = mid + 1; else hi = mid;
    }
    B.mirror = (lo < nblk && blk[lo].q == qm) ? lo : -1;
    B.comp = !(sym && charge_n(B.q) > charge_np(B.q));
  }
  __syncthreads();
  // pass 2: offsets; each computed block goes either to the one-workgroup LDS
  // Jacobi (operand fits in LDS) or to the multi-workgroup panel rounds
  int *bigl = ly.bigl + gp.lst0;
  eb = 0; reb = 0; svb = 0; rb = 0; cb = 0; bgb = 0;
  for (int b0 = 0; b0 < nblk; b0 += blockDim.x) {
    const int bi = b0 + threadIdx.x;
    long long e = 0, re = 0;
    int sv = 0, r = 0, c = 0, bg = 0, w = 0, npan = 0, qr = 0, mj = 0;
    if (bi < nblk) {
      const BlkDesc &B = blk[bi];
      mj = B.m;
      if (B.comp) {
        e = (long long)B.r * B.s;
        sv = B.n;
        svd_route(B.m, B.n, lds_bytes, qr_ok, ly.esz, qr, bg, mj);
        if (qr) re = (long long)B.n * B.n;
        if (bg) {
          w = ly.mixed ? panel_width(mj, B.n, min(lds_bytes, panel_lds), ly.esz)
                       : gram_panel_width(B.n);
          npan = (B.n + w - 1) / w;
        }
      }
      r = B.r;
      c = B.s;
    }
    long long te, tre;
    int tsv, tr, tc, tbg;
    const long long pe = eb + block_exclusive_scan<long long>(e, s_scan, te);
    const long long pre = reb + block_exclusive_scan<long long>(re, s_scan, tre);
    const int psv = svb + block_exclusive_scan<int>(sv, s_iscan, tsv);
    const int pr = rb + block_exclusive_scan<int>(r, s_iscan, tr);
    const int pc = cb + block_exclusive_scan<int>(c, s_iscan, tc);
    const int pbg = bgb + block_exclusive_scan<int>(bg, s_iscan, tbg);
    if (bi < nblk) {
      BlkDesc &B = blk[bi];
      B.eoff = pe;
      B.svoff = psv;
      B.roff = pr;
      B.coff = pc;
      B.big = bg;
      B.w = w;
      B.npan = npan;
      B.bigi = bg ? pbg : -1;
      B.qr = qr;
      B.mj = mj;
      B.joff = pre;
      B.sweeps = 0;
      if (bg) bigl[pbg] = bi;
    }
    eb += te; reb += tre; svb += tsv; rb += tr; cb += tc; bgb += tbg;
  }
  __syncthreads();
  // pass 3: row / column index lists (ascending) and, per block, the run
  // tables of the contraction: for k in [0, d), the rows with n = q0 + k start
  // at list position runs[k] and bond index runs[16 + k]; the columns with
  // n = q0 - k at list position runs[32 + k] and bond index runs[48 + k]
  int *rows = ly.rows + gp.lst0;
  int *cols = ly.cols + gp.lst0;
  for (int bi = threadIdx.x; bi < nblk; bi += blockDim.x) {
    const BlkDesc B = blk[bi];
    const int q0 = charge_n(B.q), q1 = charge_np(B.q);
    int *run = ly.runs + (size_t)(gp.blk0 + bi) * RUNS_PER_BLOCK;
    int k = 0;
    for (int n = q0; n <= q0 + d - 1; ++n) {
      const int a0 = lower_bound(cL, DL, pack_charge(n, q1));
      const int a1 = lower_bound(cL, DL, pack_charge(n, q1 + d));
      run[n - q0] = k;
      run[16 + n - q0] = a0;
      for (int a = a0; a < a1; ++a) rows[B.roff + k++] = a;
    }
    k = 0;
    for (int n = max(q0 - d + 1, 0); n <= q0; ++n) {
      const int b0 = lower_bound(cR, DR, pack_charge(n, max(q1 - d + 1, 0)));
      const int b1 = lower_bound(cR, DR, pack_charge(n, q1 + 1));
      run[32 + q0 - n] = k;
      run[48 + q0 - n] = b0;
      for (int b = b0; b < b1; ++b) cols[B.coff + k++] = b;
    }
  }
}

// Routing knobs (process-wide): an LDS budget below the device's for the
// one-workgroup Jacobi and the panel width, and whether rectangular large
// blocks are QR-reduced first.  They change only which kernels a block takes.
static int g_route_lds = 0;
static int g_qr_enable = 1;

void set_svd_route(int lds_limit_bytes, int qr_enable) {
  g_route_lds = lds_limit_bytes > 0 ? lds_limit_bytes : 0;
  g_qr_enable = qr_enable ? 1 : 0;
}

static int svd_route_bytes() {
  const int a = svd_lds_bytes();
  return g_route_lds > 0 && g_route_lds < a ? g_route_lds : a;
}

hipError_t launch_plan_count(Layer ly, hipStream_t s) {
  hipLaunchKernelGGL(k_plan<false>, dim3(ly.ngates), dim3(1024), 0, s, ly, svd_route_bytes(),
                     g_qr_enable);
  return hipGetLastError();
}

hipError_t launch_plan_fill(Layer ly, hipStream_t s) {
  hipLaunchKernelGGL(k_plan<true>, dim3(ly.ngates), dim3(1024), 0, s, ly, svd_route_bytes(),
                     g_qr_enable);
  return hipGetLastError();
}

// Locate the gate of a flat index given per-gate starts (ascending): the last
// gate whose start is <= flat (binary search; gates may own zero items).
__device__ inline int find_gate_blk(const GateBase *base, int ng, int flat) {
  int lo = 0, hi = ng;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid].blk <= flat) lo = mid; else hi = mid;
  }
  return lo;
}
__device__ inline int find_gate_big(const GateBase *base, int ng, int flat) {
  int lo = 0, hi = ng;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid].big <= flat) lo = mid; else hi = mid;
  }
  return lo;
}

// ----------------------------------------------------------------------------
// Theta(q) blocks in three steps.  For a pair (a, b) of outer indices the
// centre charges p that connect them form the box P(a, b) = [max(c_b,
// c_a - d + 1), min(c_b + d - 1, c_a)] (componentwise), and the new centre
// charges q of the blocks holding (a, b) form the same box.  The weight
// factorises into a ket and a bra part, W = K_q0[p0] conj(B_q1[p1]) with
// K = U[n0][c_a0 - q0][c_a0 - p0], B = U[n1][c_a1 - q1][c_a1 - p1],
// (n0, n1) = c_a - c_b.  So
//   G_p        = sum_{alpha of charge p} Gamma_j[a, alpha] lam_C[alpha] Gamma_{j+1}[alpha, b]
//   H_p0[q1]   = sum_{p1} conj(B_q1[p1]) G_(p0, p1)
//   Theta(q0, q1)[a, b] = lam_L[a] lam_R[b] sum_{p0} K_q0[p0] H_p0[q1]
// and every G_p and H_p0 is formed once per (a, b).  One workgroup per
// (gate, row a).  The columns b with charge n0 = c_b0 form one run of the
// right bond; a tile takes up to 256 / |box0| consecutive b of one run: its
// threads first form H for every (b, p0) into LDS, then the sums over p0
// for every (b, q0).
// ----------------------------------------------------------------------------
constexpr int CT_THREADS = 256;

template <int DMAX>
__global__ __launch_bounds__(CT_THREADS) void k_contract(Layer ly, int max_chi) {
  const int g = blockIdx.x / max_chi;
  const int a = blockIdx.x % max_chi;
  const GateParam gp = ly.gates[g];
  const State st = ly.states[gp.inst];
  const int d = st.d, chi = st.chi;
  const int j = gp.site;
  const int DL = st.dim[j], DR = st.dim[j + 2];
  if (a >= DL || DR == 0) return;
  const GateTot gt = ly.tot[g];
  if (gt.nblk == 0) return;
  const int *cL = st.chg + (size_t)j * chi;
  const int *cR = st.chg + (size_t)(j + 2) * chi;
  const int ca = cL[a];
  const int ca0 = charge_n(ca), ca1 = charge_np(ca);
  // row a of Gamma_j scaled by lam_C (shared by the whole row), then the
  // H values of one tile
  extern __shared__ __attribute__((aligned(16))) double s_dyn[];
  cd *sGa = reinterpret_cast<cd *>(s_dyn);
  cd *sH = sGa + max_chi;
  {
    const cd *Ga = st.gam + (size_t)j * chi * chi + (size_t)a * chi;
    const double *lC = st.lam + (size_t)(j + 1) * chi;
    const int DC = st.dim[j + 1];
    for (int al = threadIdx.x; al < DC; al += blockDim.x) sGa[al] = cscale(Ga[al], lC[al]);
  }
  // runs of b: for each c_b0 in [ca0 - 2d + 2, ca0], the indices with c_b1
  // in [ca1 - 2d + 2, ca1]
  __shared__ int s_b0[32], s_len[32];
  const int nrun = 2 * d - 1;
  if (threadIdx.x < nrun) {
    const int n0 = ca0 - 2 * d + 2 + (int)threadIdx.x;
    int b0 = 0, len = 0;
    if (n0 >= 0) {
      b0 = lower_bound(cR, DR, pack_charge(n0, max(ca1 - 2 * d + 2, 0)));
      len = lower_bound(cR, DR, pack_charge(n0, ca1 + 1)) - b0;
    }
    s_b0[threadIdx.x] = b0;
    s_len[threadIdx.x] = len;
  }
  __syncthreads();
  const cd *tab = ly.fock + gp.fock0;
  const double la = st.lam[(size_t)j * chi + a];
  const int W1 = gt.c1hi + 2;
  const int *T = ly.ctab + gp.ct0;
  const BlkDesc *blk = ly.blk + gp.blk0;
  const long long ebase = ly.base[g].e;
  const cd *G1 = st.gam + (size_t)(j + 1) * chi * chi;
  for (int r = 0; r < nrun; ++r) {
    const int len = s_len[r];
    if (len == 0) continue;
    const int n0b = ca0 - 2 * d + 2 + r;                       // c_b0 of the run
    const int base0 = max(n0b, ca0 - d + 1);                   // box0 = [base0, base0 + nq)
    const int nq = min(n0b + d - 1, ca0) - base0 + 1;
    const int n0 = ca0 - n0b;
    const int tb = CT_THREADS / nq;
    for (int bt = 0; bt < len; bt += tb) {
      const int nb = min(tb, len - bt);
      const int lt = threadIdx.x;
      const bool act = lt < nq * nb;
      const int k = act ? lt / nb : 0, bi = act ? lt % nb : 0;
      const int b = s_b0[r] + bt + bi;
      const int cb1 = act ? charge_np(cR[b]) : 0;
      const int n1 = ca1 - cb1;
      const int q1lo = max(cb1, ca1 - d + 1), q1hi = min(cb1 + d - 1, ca1);
      const int nq1 = q1hi - q1lo + 1;
      if (act) {
        // step 1 and 2 for (b, p0 = base0 + k)
        const int p0 = base0 + k;
        cd H[DMAX];
#pragma unroll
        for (int u = 0; u < DMAX; ++u) H[u] = cmk(0.0, 0.0);
        if (p0 >= gt.c0lo && p0 <= gt.c0hi) {
          const int *Tp = T + (size_t)(p0 - gt.c0lo) * W1;
          const cd *Gb = G1 + b;
          for (int p1 = q1lo; p1 <= q1hi && p1 <= gt.c1hi; ++p1) {
            const int al0 = Tp[p1], al1 = Tp[p1 + 1];
            if (al0 >= al1) continue;
            // four Gamma_{j+1} loads in flight per step
            cd G = cmk(0.0, 0.0);
            int al = al0;
            for (; al + 3 < al1; al += 4) {
              const cd b0 = Gb[(size_t)al * chi], b1 = Gb[(size_t)(al + 1) * chi];
              const cd b2 = Gb[(size_t)(al + 2) * chi], b3 = Gb[(size_t)(al + 3) * chi];
              cfma(G, sGa[al], b0);
              cfma(G, sGa[al + 1], b1);
              cfma(G, sGa[al + 2], b2);
              cfma(G, sGa[al + 3], b3);
            }
            for (; al < al1; ++al) cfma(G, sGa[al], Gb[(size_t)al * chi]);
            // H[q1] += conj(U[n1][ca1 - q1][ca1 - p1]) G
            const cd *Bcol = tab + (size_t)n1 * d * d + (ca1 - p1);
#pragma unroll
            for (int u = 0; u < DMAX; ++u)
              if (u < nq1) cfma(H[u], cconj(Bcol[(size_t)(ca1 - q1lo - u) * d]), G);
          }
        }
#pragma unroll
        for (int u = 0; u < DMAX; ++u)
          if (u < nq1) sH[(size_t)lt * DMAX + u] = H[u];
      }
      __syncthreads();
      if (act) {
        // step 3 for (b, q0 = base0 + k)
        const int q0 = base0 + k, i0 = ca0 - q0;
        cd acc[DMAX];
#pragma unroll
        for (int u = 0; u < DMAX; ++u) acc[u] = cmk(0.0, 0.0);
        for (int kp = 0; kp < nq; ++kp) {
          const cd K = tab[((size_t)n0 * d + i0) * d + (ca0 - base0 - kp)];
          const cd *Hr = sH + (size_t)(kp * nb + bi) * DMAX;
#pragma unroll
          for (int u = 0; u < DMAX; ++u)
            if (u < nq1) cfma(acc[u], K, Hr[u]);
        }
        // write Theta(q0, q1)[a, b] into every computed block (q0, q1)
        const double sc = la * st.lam[(size_t)(j + 2) * chi + b];
#pragma unroll
        for (int u = 0; u < DMAX; ++u) {
          if (u >= nq1) continue;
          const int q = pack_charge(q0, q1lo + u);
          int lo = 0, hi = gt.nblk;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (blk[mid].q < q) lo = mid + 1; else hi = mid;
          }
          if (lo >= gt.nblk || blk[lo].q != q) continue;
          const BlkDesc &B = blk[lo];
          if (!B.comp) continue;
          const int *run = ly.runs + (size_t)(gp.blk0 + lo) * RUNS_PER_BLOCK;
          const int ka = ca0 - q0, kb = q0 - n0b;
          const int ia = run[ka] + (a - run[16 + ka]);
          const int ib = run[32 + kb] + (b - run[48 + kb]);
          const size_t at = !B.t ? (size_t)ib * B.m + ia       // Theta, m = r rows
                                 : (size_t)ia * B.m + ib;      // Theta^T, m = s rows
          const cd v = cscale(acc[u], sc);
          ly.A[ebase + B.eoff + at] = v;
          ly.A0[ebase + B.eoff + at] = v;
        }
      }
      __syncthreads();
    }
  }
}

int svd_lds_bytes();

hipError_t launch_contract(Layer ly, int max_chi, int max_d, hipStream_t s) {
  if (ly.total_blocks == 0) return hipSuccess;
  svd_lds_bytes();   // dynamic LDS limits of the kernels (set once)
  const dim3 grid((unsigned)(ly.ngates * max_chi));
  // scaled Gamma row (max_chi) and one tile of H values (CT_THREADS x DMAX)
  const size_t row = sizeof(cd) * (size_t)max_chi, tile = sizeof(cd) * CT_THREADS;
  if (max_d <= 4)
    hipLaunchKernelGGL(k_contract<4>, grid, dim3(CT_THREADS), row + 4 * tile, s, ly, max_chi);
  else if (max_d <= 8)
    hipLaunchKernelGGL(k_contract<8>, grid, dim3(CT_THREADS), row + 8 * tile, s, ly, max_chi);
  else
    hipLaunchKernelGGL(k_contract<16>, grid, dim3(CT_THREADS), row + 16 * tile, s, ly, max_chi);
  return hipGetLastError();
}

// Centre-bond run table of every gate: T[x][y] = first index of the sorted
// centre bond with charge >= (c0lo + x, y).  The indices with charge (p0, p1)
// for p1 in [a, b) are then [T[p0 - c0lo][a], T[p0 - c0lo][b]).
__global__ __launch_bounds__(256) void k_ctab(Layer ly) {
  const int g = blockIdx.x;
  const GateParam gp = ly.gates[g];
  const GateTot gt = ly.tot[g];
  if (gt.c1hi < 0) return;
  const State st = ly.states[gp.inst];
  const int DC = st.dim[gp.site + 1];
  const int *cC = st.chg + (size_t)(gp.site + 1) * st.chi;
  const int W0 = gt.c0hi - gt.c0lo + 2, W1 = gt.c1hi + 2;
  int *T = ly.ctab + gp.ct0;
  for (int idx = threadIdx.x; idx < W0 * W1; idx += blockDim.x) {
    const int x = idx / W1, y = idx % W1;
    T[idx] = lower_bound(cC, DC, pack_charge(gt.c0lo + x, y));
  }
}

hipError_t launch_ctab(Layer ly, hipStream_t s) {
  hipLaunchKernelGGL(k_ctab, dim3(ly.ngates), dim3(256), 0, s, ly);
  return hipGetLastError();
}



// ----------------------------------------------------------------------------
// Householder QR with column pivoting of the large blocks: A P = Q R with
// Q = H_0 H_1 ... H_{n-1}, H_k = I - tau_k v_k v_k^H, v_k[0] = 1.  Step k
// brings the remaining column of largest norm (rows k..m-1; ties to the
// lowest index) to position k; for that column's part x below the diagonal,
// beta = -sign(Re x_0) |x|, tau = (beta - x_0) / beta and v = x / (x_0 - beta)
// give H_k^H x = beta e_1 with beta real, and the trailing columns are
// multiplied by H_k^H (their norms over rows k+1.. are recomputed exactly in
// the same pass).  One workgroup per block; the operand is overwritten (its
// pristine copy stays in A0), X = R^H (lower triangle) goes to the R pool
// and the pivot order to piv (piv[k] = original column at position k).
// The column pivoting grades R, so that the Jacobi on X needs few sweeps.
// ----------------------------------------------------------------------------
constexpr int QR_THREADS = 1024;

// Reflector of the column x = (al, rest), |rest|^2 = s2 (formulas above).
// Returns false (no reflection, H = I) when x is already a multiple of e_1,
// or when x is so small that |x|^2 underflows and the reflector cannot be
// formed in finite arithmetic: such a column is rounding noise (its
// entries below the diagonal, left in place, never reach X = R^H).
__device__ inline bool householder(cd al, double s2, cd &tau, cd &scale, double &beta) {
  if (s2 == 0.0 && al.im == 0.0) return false;
  const double nrm = sqrt(al.re * al.re + al.im * al.im + s2);
  beta = al.re >= 0.0 ? -nrm : nrm;
  tau = cmk((beta - al.re) / beta, -al.im / beta);
  const cd dn = cmk(al.re - beta, al.im);
  const double dd = cabs2(dn);
  scale = cmk(dn.re / dd, -dn.im / dd);
  return nrm > 0.0 && isfinite(tau.re) && isfinite(tau.im) && isfinite(scale.re) &&
         isfinite(scale.im);
}
constexpr int QC = 16;   // column elements per lane kept in registers (m - k <= 1024)

__device__ __forceinline__ double block_sum(double v, double *s_red);

// Workgroup sum without the trailing barrier of block_sum: for callers whose
// next write of s_red comes after another barrier.
__device__ __forceinline__ double block_sum_keep(double v, double *s_red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s_red[w];
  return t;
}

// Largest value over the 64 lanes of a wave with, among equal values, the
// lowest index; the same pair in every lane.  Each step merges a lane with
// its partner under one total order, so both end with the same pair.
__device__ __forceinline__ void amax_merge(double &bv, int &bi, double ov, int oi) {
  if (ov > bv || (ov == bv && oi < bi)) {
    bv = ov;
    bi = oi;
  }
}
template <int CTRL>
__device__ __forceinline__ void amax_dpp(double &bv, int &bi) {
  const double ov = dpp_d<CTRL>(bv);
  const int oi = __builtin_amdgcn_update_dpp(bi, bi, CTRL, 0xF, 0xF, false);
  amax_merge(bv, bi, ov, oi);
}
template <bool ROW16>
__device__ __forceinline__ void amax_swap(double &bv, int &bi) {
  const unsigned lo = __double2loint(bv), hi = __double2hiint(bv), ix = (unsigned)bi;
  double v0, v1;
  int i0, i1;
  if (ROW16) {
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const auto x = __builtin_amdgcn_permlane16_swap(ix, ix, false, false);
    v0 = __hiloint2double(h[0], l[0]);
    v1 = __hiloint2double(h[1], l[1]);
    i0 = (int)x[0];
    i1 = (int)x[1];
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    const auto x = __builtin_amdgcn_permlane32_swap(ix, ix, false, false);
    v0 = __hiloint2double(h[0], l[0]);
    v1 = __hiloint2double(h[1], l[1]);
    i0 = (int)x[0];
    i1 = (int)x[1];
  }
  bv = v0;
  bi = i0;
  amax_merge(bv, bi, v1, i1);
}
__device__ __forceinline__ void wave_argmax(double &bv, int &bi) {
  amax_dpp<0xB1>(bv, bi);
  amax_dpp<0x4E>(bv, bi);
  amax_dpp<0x140>(bv, bi);
  amax_dpp<0x141>(bv, bi);
  amax_swap<true>(bv, bi);
  amax_swap<false>(bv, bi);
}

// Trailing update of QR step k for the columns j > k: a_j -= conj(tau) v (v^H a_j)
// on rows k.., and the squared norm of a_j below row k.  Each wave takes CPW
// columns at a time (their loads in flight together), QCL elements per lane
// of each held in registers between the dot product and the update
// (len <= 64 QCL).
template <int QCL, int CPW>
__device__ __forceinline__ void qr_update(cd *A, int m, int n, int k, int len, const cd *v, cd ct,
                                          bool skip, double *cn, int wave, int nw, int lane) {
  for (int j0 = k + 1 + wave * CPW; j0 < n; j0 += nw * CPW) {
    cd ra[CPW][QCL];
    double wr[CPW], wi[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const cd *a = A + (size_t)(j0 + c) * m + k;
      const bool has = j0 + c < n;
#pragma unroll
      for (int u = 0; u < QCL; ++u) {
        const int y = lane + 64 * u;
        ra[c][u] = (has && y < len) ? a[y] : cmk(0.0, 0.0);
      }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      wr[c] = 0.0;
      wi[c] = 0.0;
      if (!skip) {
#pragma unroll
        for (int u = 0; u < QCL; ++u) {
          const int y = lane + 64 * u;
          if (y < len) {
            const cd q = cmulc(v[y], ra[c][u]);
            wr[c] += q.re;
            wi[c] += q.im;
          }
        }
      }
    }
    if (!skip) {
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        wr[c] = group_sum<64>(wr[c]);
        wi[c] = group_sum<64>(wi[c]);
      }
    }
    double nb[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int j = j0 + c;
      cd *a = A + (size_t)j * m + k;
      const cd f = cmul(ct, cmk(wr[c], wi[c]));    // conj(tau) v^H a
      nb[c] = 0.0;
#pragma unroll
      for (int u = 0; u < QCL; ++u) {
        const int y = lane + 64 * u;
        if (j < n && y < len) {
          const cd an = skip ? ra[c][u] : csub(ra[c][u], cmul(f, v[y]));
          if (!skip) a[y] = an;
          if (y >= 1) nb[c] += cabs2(an);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const double t = group_sum<64>(nb[c]);
      if (lane == 0 && j0 + c < n) cn[j0 + c] = t;
    }
  }
}

// Householder QR with column pivoting by panels of nb columns (delayed
// update, in the manner of LAPACK's xLAQPS): inside a panel the reflectors
// are not applied to the trailing columns; instead F = A^H V T collects them
// (A the trailing columns as they were when the panel started, V the panel's
// reflectors, T the triangular factor of Q = H_0 ... H_{nb-1} = I - V T V^H),
// so that Q^H A = A - V F^H.  Step k of the panel
//   brings the column of largest remaining norm to position k,
//   applies the panel's earlier reflectors to column k alone,
//   forms H_k from it,
//   appends column tau_k A^H v_k - tau_k F (V^H v_k) to F,
//   and updates row k of the trailing columns (it becomes a row of R), so
//   that their remaining norms drop by |R[k, j]|^2.
// At the end of the panel the trailing columns receive A -= V F^H in one
// pass, which also recomputes their norms exactly.  A panel ends early when
// a norm loses more than half of its digits to the downdate.  The trailing
// columns are read once per step (the product A^H v_k) and written once per
// panel instead of read and written once per step.
// LDS: v (m), remaining and reference norms (2 n doubles), F (n x nb, column
// stride n), per-wave partial norms (16 x 64 doubles).
constexpr int QR_NB = 8;

// X = R^H (n x n, column-major, lower triangle) from the factored operand.
__device__ __forceinline__ void qr_write_x(cd *X, const cd *A, int m, int n) {
  for (long long idx = threadIdx.x; idx < (long long)n * n; idx += blockDim.x) {
    const int c = (int)(idx / n), i = (int)(idx % n);
    X[idx] = c <= i ? cconj(A[(size_t)i * m + c]) : cmk(0.0, 0.0);
  }
}

#ifndef GBS_QR_PANELS
#define GBS_QR_PANELS 1
#endif

__host__ __device__ inline int qr_panel_width(int m, int n, int lds_bytes) {
  if (!GBS_QR_PANELS) return 1;
  const long long room = (long long)lds_bytes - 16LL * m - 16LL * n - 8 * 16 * 64 - 256;
  if (n <= 0 || room < 32LL * n) return 1;
  const long long w = room / (16LL * n);
  return w < QR_NB ? (int)w : QR_NB;
}

// LDS of one k_qr_panel workgroup given the device budget.
__host__ __device__ inline int svd_panel_half(int lds_bytes) { return lds_bytes / 2 - 1024; }

__device__ void qr_blocked(cd *A, int m, int n, cd *tau, int *piv, int nb, double *lds) {
  cd *v = reinterpret_cast<cd *>(lds);                    // reflector of the step (rows k..)
  double *cn = reinterpret_cast<double *>(v + m);          // remaining norms^2 (downdated)
  double *cr = cn + n;                                     // norms^2 at the last exact sum
  cd *F = reinterpret_cast<cd *>(cr + n);                  // F[j + c n]
  double *part = reinterpret_cast<double *>(F + (size_t)n * nb);   // [16][64]
  __shared__ double s_red[16];
  __shared__ double s_bv[16];
  __shared__ int s_bi[16];
  __shared__ cd s_aux[QR_NB];
  __shared__ int s_flag;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = wave; c < n; c += nw) {
    double acc = 0.0;
    for (int y = lane; y < m; y += 64) acc += cabs2(A[(size_t)c * m + y]);
    acc = wave_sum(acc);
    if (lane == 0) cn[c] = cr[c] = acc;
  }
  for (int c = threadIdx.x; c < n; c += blockDim.x) piv[c] = c;
  if (threadIdx.x == 0) s_flag = 0;
  __syncthreads();
  int k0 = 0;
  while (k0 < n) {
    const int nbk = min(nb, n - k0);
    int kb = nbk;
    for (int i = 0; i < nbk; ++i) {
      const int k = k0 + i;
      // pivot: largest remaining norm, lowest index on ties
      double bv = -1.0;
      int bi = n;
      for (int c = k + threadIdx.x; c < n; c += blockDim.x)
        if (cn[c] > bv) { bv = cn[c]; bi = c; }
      wave_argmax(bv, bi);
      if (lane == 0) { s_bv[wave] = bv; s_bi[wave] = bi; }
      __syncthreads();
      // every thread merges the waves' candidates in the same order (no
      // second barrier; s_bv / s_bi are next written after several more)
      int p;
      {
        double b = s_bv[0];
        int pp = s_bi[0];
        for (int w2 = 1; w2 < nw; ++w2)
          if (s_bv[w2] > b || (s_bv[w2] == b && s_bi[w2] < pp)) { b = s_bv[w2]; pp = s_bi[w2]; }
        p = pp < n ? pp : k;
      }
      if (p != k) {
        for (int y = threadIdx.x; y < m; y += blockDim.x) {
          const cd t = A[(size_t)k * m + y];
          A[(size_t)k * m + y] = A[(size_t)p * m + y];
          A[(size_t)p * m + y] = t;
        }
        for (int c = threadIdx.x; c < i; c += blockDim.x) {
          const cd t = F[k + (size_t)c * n];
          F[k + (size_t)c * n] = F[p + (size_t)c * n];
          F[p + (size_t)c * n] = t;
        }
        if (threadIdx.x == 0) {
          double t = cn[k]; cn[k] = cn[p]; cn[p] = t;
          t = cr[k]; cr[k] = cr[p]; cr[p] = t;
          const int ti = piv[k]; piv[k] = piv[p]; piv[p] = ti;
        }
        __syncthreads();
      }
      // column k: the panel's earlier reflectors, A[k:, k] -= V[k:, :i] F[k, :i]^H
      cd *x = A + (size_t)k * m + k;
      const int len = m - k;
      double s2 = 0.0;
      for (int y = threadIdx.x; y < len; y += blockDim.x) {
        cd a = x[y];
        for (int c = 0; c < i; ++c)
          a = csub(a, cmul(A[(size_t)(k0 + c) * m + k + y], cconj(F[k + (size_t)c * n])));
        if (i > 0) x[y] = a;
        if (y >= 1) s2 += cabs2(a);
      }
      s2 = block_sum_keep(s2, s_red);
      // every thread forms the same reflector from x[0] and s2 (no barrier);
      // thread 0 stores tau and the new diagonal after the next barrier, as
      // nothing reads x[0] before the following column
      cd h_tau, h_scale;
      double h_beta;
      const bool skip = !householder(x[0], s2, h_tau, h_scale, h_beta);
      for (int y = 1 + threadIdx.x; y < len; y += blockDim.x) {
        const cd t = skip ? x[y] : cmul(x[y], h_scale);
        if (!skip) x[y] = t;
        v[y] = t;
      }
      if (threadIdx.x == 0) v[0] = cmk(1.0, 0.0);
      __syncthreads();
      if (threadIdx.x == 0) {
        tau[k] = skip ? cmk(0.0, 0.0) : h_tau;
        if (!skip) x[0] = cmk(h_beta, 0.0);
      }
      // F[j, i] = tau_k A[k:, j]^H v (trailing j > k) and s_aux[c] = -tau_k V[k:, c]^H v
      const cd tk = skip ? cmk(0.0, 0.0) : h_tau;
      const int ntr = n - k - 1;
      for (int t = wave; t < ntr + i; t += nw) {
        const int col = t < ntr ? k + 1 + t : k0 + (t - ntr);
        const cd *a = A + (size_t)col * m + k;
        double wr = 0.0, wi = 0.0;
        int y = lane;
        // eight loads in flight per lane: one wave streams the whole trailing
        // column, so the loads in flight set the rate of the factorisation's
        // longest chain (the largest block's QR)
        for (; y + 448 < len; y += 512) {
          cd av[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) av[u] = a[y + 64 * u];
          double pr[8], pi[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const cd q = cmulc(av[u], v[y + 64 * u]);
            pr[u] = q.re;
            pi[u] = q.im;
          }
          wr += ((pr[0] + pr[1]) + (pr[2] + pr[3])) + ((pr[4] + pr[5]) + (pr[6] + pr[7]));
          wi += ((pi[0] + pi[1]) + (pi[2] + pi[3])) + ((pi[4] + pi[5]) + (pi[6] + pi[7]));
        }
        for (; y + 192 < len; y += 256) {
          const cd a0 = a[y], a1 = a[y + 64], a2 = a[y + 128], a3 = a[y + 192];
          const cd q0 = cmulc(a0, v[y]), q1 = cmulc(a1, v[y + 64]);
          const cd q2 = cmulc(a2, v[y + 128]), q3 = cmulc(a3, v[y + 192]);
          wr += (q0.re + q1.re) + (q2.re + q3.re);
          wi += (q0.im + q1.im) + (q2.im + q3.im);
        }
        for (; y < len; y += 64) {
          const cd q = cmulc(a[y], v[y]);
          wr += q.re;
          wi += q.im;
        }
        wr = group_sum<64>(wr);
        wi = group_sum<64>(wi);
        if (lane == 0) {
          const cd f = cmul(tk, cmk(wr, wi));
          if (t < ntr) F[col + (size_t)i * n] = f;
          else s_aux[t - ntr] = cmk(-f.re, -f.im);
        }
      }
      __syncthreads();
      // F[j, i] += F[j, :i] s_aux, then row k of the trailing columns and
      // their remaining norms
      for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) {
        cd f = F[j + (size_t)i * n];
        for (int c = 0; c < i; ++c) cfma(f, F[j + (size_t)c * n], s_aux[c]);
        F[j + (size_t)i * n] = f;
        cd a = A[(size_t)j * m + k];
        for (int c = 0; c < i; ++c)
          a = csub(a, cmul(A[(size_t)(k0 + c) * m + k], cconj(F[j + (size_t)c * n])));
        a = csub(a, cconj(f));                 // v_k[0] = 1
        A[(size_t)j * m + k] = a;
        const double rest = cn[j] - cabs2(a);
        if (cr[j] > 0.0 && !(rest > 1e-8 * cr[j])) s_flag = 1;
        cn[j] = fmax(rest, 0.0);
      }
      __syncthreads();
      if (s_flag) {
        kb = i + 1;
        break;
      }
    }
    // trailing columns j >= k1, rows y >= k1: A -= V F^H, exact norms.
    // Waves own 64-row chunks (their V rows in registers) and, when the
    // chunks are fewer than the waves, interleaved column groups.
    const int k1 = k0 + kb;
    const int R = m - k1, N2 = n - k1;
    if (R > 0 && N2 > 0) {
      const int nrc = (R + 63) / 64;
      const int ncg = nrc >= nw ? 1 : nw / nrc;
      const int nchunk_w = nrc >= nw ? nw : nrc;    // rows of part in use
      const int chunk0 = nrc >= nw ? wave : wave % nrc;
      const int grp = nrc >= nw ? 0 : wave / nrc;
      const bool active = grp < ncg;
      for (int jb = 0; jb < N2; jb += 64) {
        const int nj = min(64, N2 - jb);
        if (active) {
          // partial norms of this wave's columns over its chunks, in chunk order
          for (int jl = grp; jl < nj; jl += ncg)
            if (lane == 0) part[(size_t)(nrc >= nw ? wave : chunk0) * 64 + jl] = 0.0;
          for (int ch = chunk0; ch < nrc; ch += (nrc >= nw ? nw : nrc)) {
            const int y = k1 + ch * 64 + lane;
            const bool row = y < m;
            cd vr[QR_NB];
#pragma unroll
            for (int c = 0; c < QR_NB; ++c)
              vr[c] = (c < kb && row) ? A[(size_t)(k0 + c) * m + y] : cmk(0.0, 0.0);
            for (int jl = grp; jl < nj; jl += ncg) {
              const int j = k1 + jb + jl;
              cd a = row ? A[(size_t)j * m + y] : cmk(0.0, 0.0);
#pragma unroll
              for (int c = 0; c < QR_NB; ++c)
                if (c < kb) a = csub(a, cmul(vr[c], cconj(F[j + (size_t)c * n])));
              if (row) A[(size_t)j * m + y] = a;
              const double pn = group_sum<64>(row ? cabs2(a) : 0.0);
              if (lane == 0) part[(size_t)(nrc >= nw ? wave : chunk0) * 64 + jl] += pn;
            }
            if (nrc < nw) break;                    // one chunk per wave
          }
        }
        __syncthreads();
        for (int jl = threadIdx.x; jl < nj; jl += blockDim.x) {
          double t = 0.0;
          for (int r = 0; r < nchunk_w; ++r) t += part[(size_t)r * 64 + jl];
          cn[k1 + jb + jl] = cr[k1 + jb + jl] = t;
        }
        __syncthreads();
      }
    }
    if (threadIdx.x == 0) s_flag = 0;
    __syncthreads();
    k0 = k1;
  }
}

// Launch order of the QR workgroups: the QR'd blocks by decreasing work
// (m n^2, in quarter-octave buckets), then every other block (they exit at
// once).  A block's QR is one long chain on one workgroup, so starting the
// largest first shortens the launch's tail; the order changes no arithmetic.
constexpr int QR_ORDER_BUCKETS = 256;

__global__ __launch_bounds__(1024) void k_qr_order(Layer ly) {
  __shared__ int s_cnt[QR_ORDER_BUCKETS + 1];
  __shared__ int s_off[QR_ORDER_BUCKETS + 1];
  for (int i = threadIdx.x; i <= QR_ORDER_BUCKETS; i += blockDim.x) s_cnt[i] = 0;
  __syncthreads();
  auto bucket = [&](int flat) -> int {
    const int g = find_gate_blk(ly.base, ly.ngates, flat);
    const BlkDesc &B = ly.blk[ly.gates[g].blk0 + (flat - ly.base[g].blk)];
    if (!B.comp || !B.qr) return QR_ORDER_BUCKETS;          // last
    const double w = (double)B.m * B.n * B.n;
    const int k = (int)(4.0 * log2(fmax(w, 1.0)));
    return QR_ORDER_BUCKETS - 1 - min(k, QR_ORDER_BUCKETS - 1);   // heavy first
  };
  for (int f = threadIdx.x; f < ly.total_blocks; f += blockDim.x) atomicAdd(&s_cnt[bucket(f)], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int b = 0; b <= QR_ORDER_BUCKETS; ++b) {
      s_off[b] = acc;
      acc += s_cnt[b];
    }
  }
  __syncthreads();
  for (int f = threadIdx.x; f < ly.total_blocks; f += blockDim.x)
    ly.qr_order[atomicAdd(&s_off[bucket(f)], 1)] = f;
}

// QR of every block whose panel of F fits in LDS (the others: k_qr).
// A block's factorisation is one long chain on one workgroup, and the
// largest blocks' chains set the launch's length: 1024 threads per
// workgroup (one per CU, half of its LDS) stream each trailing column with
// twice the lanes of two 512-thread workgroups per CU.
#ifndef GBS_QRP_THREADS
#define GBS_QRP_THREADS 1024
#endif
constexpr int QRP_THREADS = GBS_QRP_THREADS;

// Blocks of the sketch-pivoted QR (defined below): one thread per column and
// the panel's reflectors in LDS beside the W tiles.
#ifndef GBS_QR_SKETCH
#define GBS_QR_SKETCH 0
#endif
constexpr int QS_NB = 8;             // panel width
constexpr int QS_THREADS = QRP_THREADS;   // one thread per block column (n <= 1024)
static_assert(QS_THREADS == 1024, "the sketch path holds one column per thread");
constexpr int QS_WBYTES = 16 * 16 * QS_NB * 16;   // per-wave W tiles (16 waves)
__host__ __device__ inline bool qs_fits(int m, int n, int lds_bytes) {
  return GBS_QR_SKETCH && n >= QS_NB + 4 && n <= QS_THREADS &&
         (long long)m * QS_NB * 16 + QS_WBYTES <= lds_bytes;
}

__device__ void qr_sketch(cd *A, int m, int n, cd *tau, int *piv, cd *S, double *s_dyn);

// lds_bytes: the column-pivoted path's budget; qs_lds: the sketch path's
// (the launch provides the larger of the two)
__global__ __launch_bounds__(QRP_THREADS) void k_qr_panel(Layer ly, int lds_bytes, int qs_lds) {
  const int flat = ly.qr_order[blockIdx.x];
  const int g = find_gate_blk(ly.base, ly.ngates, flat);
  const GateBase gb = ly.base[g];
  const GateParam gp = ly.gates[g];
  const BlkDesc B = ly.blk[gp.blk0 + (flat - gb.blk)];
  if (!B.comp || !B.qr) return;
  const int m = B.m, n = B.n;
  cd *A = ly.A + gb.e + B.eoff;
  cd *tau = ly.tau + gp.lst0 + B.svoff;
  int *piv = ly.piv + gp.lst0 + B.svoff;
  extern __shared__ __attribute__((aligned(16))) double s_dyn[];
  if (qs_fits(m, n, qs_lds)) {
    qr_sketch(A, m, n, tau, piv, ly.R + gb.r + B.joff, s_dyn);
  } else {
    const int nb = qr_panel_width(m, n, lds_bytes);
    if (nb < 2) return;
    qr_blocked(A, m, n, tau, piv, nb, s_dyn);
  }
  __syncthreads();
  qr_write_x(ly.R + gb.r + B.joff, A, m, n);
}

__global__ __launch_bounds__(QR_THREADS) void k_qr(Layer ly, int lds_bytes, int qs_lds) {
  const int flat = ly.qr_order[blockIdx.x];
  const int g = find_gate_blk(ly.base, ly.ngates, flat);
  const GateBase gb = ly.base[g];
  const GateParam gp = ly.gates[g];
  const BlkDesc B = ly.blk[gp.blk0 + (flat - gb.blk)];
  if (!B.comp || !B.qr) return;
  const int m = B.m, n = B.n;
  cd *A = ly.A + gb.e + B.eoff;
  cd *tau = ly.tau + gp.lst0 + B.svoff;
  int *piv = ly.piv + gp.lst0 + B.svoff;
  extern __shared__ __attribute__((aligned(16))) double s_dyn[];
  if (qr_panel_width(m, n, svd_panel_half(lds_bytes)) >= 2) return;   // k_qr_panel's block
  if (qs_fits(m, n, qs_lds)) return;                                   // sketch-pivoted in k_qr_panel
  // one column at a time (operands too large for a panel of F in LDS)
  cd *v = reinterpret_cast<cd *>(s_dyn);             // current reflector, m - k entries
  double *cn = reinterpret_cast<double *>(v + m);    // remaining column norms^2
  __shared__ double s_red[16];
  __shared__ double s_bv[16];
  __shared__ int s_bi[16];
  __shared__ cd s_tau, s_scale;
  __shared__ int s_skip, s_piv;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = wave; c < n; c += nw) {
    double acc = 0.0;
    for (int y = lane; y < m; y += 64) acc += cabs2(A[(size_t)c * m + y]);
    acc = wave_sum(acc);
    if (lane == 0) cn[c] = acc;
  }
  for (int c = threadIdx.x; c < n; c += blockDim.x) piv[c] = c;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot: largest remaining norm, lowest index on ties
    double bv = -1.0;
    int bi = n;
    for (int c = k + threadIdx.x; c < n; c += blockDim.x)
      if (cn[c] > bv) { bv = cn[c]; bi = c; }
    wave_argmax(bv, bi);
    if (lane == 0) { s_bv[wave] = bv; s_bi[wave] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double b = s_bv[0];
      int p = s_bi[0];
      for (int w2 = 1; w2 < nw; ++w2)
        if (s_bv[w2] > b || (s_bv[w2] == b && s_bi[w2] < p)) { b = s_bv[w2]; p = s_bi[w2]; }
      s_piv = p < n ? p : k;
    }
    __syncthreads();
    const int p = s_piv;
    if (p != k) {
      for (int y = threadIdx.x; y < m; y += blockDim.x) {
        const cd t = A[(size_t)k * m + y];
        A[(size_t)k * m + y] = A[(size_t)p * m + y];
        A[(size_t)p * m + y] = t;
      }
      if (threadIdx.x == 0) {
        const double t = cn[k]; cn[k] = cn[p]; cn[p] = t;
        const int ti = piv[k]; piv[k] = piv[p]; piv[p] = ti;
      }
      __syncthreads();
    }
    cd *x = A + (size_t)k * m + k;
    const int len = m - k;
    double s2 = 0.0;
    for (int y = 1 + threadIdx.x; y < len; y += blockDim.x) s2 += cabs2(x[y]);
    s2 = block_sum(s2, s_red);
    if (threadIdx.x == 0) {
      cd t, sc;
      double beta;
      if (!householder(x[0], s2, t, sc, beta)) {
        s_skip = 1;
        tau[k] = cmk(0.0, 0.0);
      } else {
        s_tau = t;
        s_scale = sc;
        tau[k] = t;
        x[0] = cmk(beta, 0.0);
        s_skip = 0;
      }
    }
    __syncthreads();
    const bool skip = s_skip != 0;
    if (!skip) {
      const cd sc = s_scale;
      for (int y = 1 + threadIdx.x; y < len; y += blockDim.x) {
        const cd t = cmul(x[y], sc);
        x[y] = t;
        v[y] = t;
      }
      if (threadIdx.x == 0) v[0] = cmk(1.0, 0.0);
    }
    __syncthreads();
    const cd ct = skip ? cmk(0.0, 0.0) : cconj(s_tau);
    if (len <= 64 * 4)
      qr_update<4, 4>(A, m, n, k, len, v, ct, skip, cn, wave, nw, lane);
    else if (len <= 64 * 8)
      qr_update<8, 2>(A, m, n, k, len, v, ct, skip, cn, wave, nw, lane);
    else if (len <= 64 * QC) {
      // column segment held in registers between the dot product and the update
      for (int j = k + 1 + wave; j < n; j += nw) {
        cd *a = A + (size_t)j * m + k;
        cd ra[QC];
        double wr = 0.0, wi = 0.0;
#pragma unroll
        for (int u = 0; u < QC; ++u) {
          const int y = lane + 64 * u;
          ra[u] = y < len ? a[y] : cmk(0.0, 0.0);
          if (y < len && !skip) {
            const cd q = cmulc(v[y], ra[u]);
            wr += q.re;
            wi += q.im;
          }
        }
        if (!skip) {
          wr = group_sum<64>(wr);
          wi = group_sum<64>(wi);
        }
        const cd f = cmul(ct, cmk(wr, wi));    // conj(tau) v^H a
        double nb = 0.0;
#pragma unroll
        for (int u = 0; u < QC; ++u) {
          const int y = lane + 64 * u;
          if (y < len) {
            const cd an = skip ? ra[u] : csub(ra[u], cmul(f, v[y]));
            if (!skip) a[y] = an;
            if (y >= 1) nb += cabs2(an);
          }
        }
        nb = group_sum<64>(nb);
        if (lane == 0) cn[j] = nb;
      }
    } else {
      for (int j = k + 1 + wave; j < n; j += nw) {
        cd *a = A + (size_t)j * m + k;
        double wr = 0.0, wi = 0.0;
        if (!skip) {
          for (int y = lane; y < len; y += 64) {
            const cd q = cmulc(v[y], a[y]);
            wr += q.re;
            wi += q.im;
          }
          wr = group_sum<64>(wr);
          wi = group_sum<64>(wi);
        }
        const cd f = cmul(ct, cmk(wr, wi));    // conj(tau) v^H a
        double nb = 0.0;
        for (int y = lane; y < len; y += 64) {
          const cd an = skip ? a[y] : csub(a[y], cmul(f, v[y]));
          if (!skip) a[y] = an;
          if (y >= 1) nb += cabs2(an);
        }
        nb = group_sum<64>(nb);
        if (lane == 0) cn[j] = nb;
      }
    }
    __syncthreads();
  }
  qr_write_x(ly.R + gb.r + B.joff, A, m, n);
}

// ----------------------------------------------------------------------------
// Householder QR with sketch pivoting, by panels of QS_NB columns (in place of
// the column pivoting above when GBS_QR_SKETCH is set).  A panel's pivots are
// the columns a column-pivoted QR of a small random sketch picks: the sketch
// S = Omega A[k0:, k0:] has QS_P = QS_NB + 4 rows of independent signs (a
// hash of the matrix row, the sketch row and the panel), and each of its
// column norms estimates the norm of the remaining column, so that the panel
// takes the columns of largest remaining norm without a pass over the
// trailing matrix per column.  The panel is then factored alone (unpivoted
// Householder: H = I - tau v v^H, v[0] = 1, H^H x = beta e_1 as above), its
// reflectors are gathered as Q = I - V T V^H (T upper triangular, forward
// accumulation) and the trailing columns receive Q^H in one step,
//   A_t <- A_t - V T^H (V^H A_t),
// computed on the FP64 matrix cores by tiles of 16 columns: the complex
// products run as real ones with the panel's 8 complex reflectors embedded
// as 16 real rows (W = V^H A_t: rows Re W, Im W; A_t -= V W': rows (y, re),
// (y, im)).  The trailing matrix is read three times and written once per
// panel (sketch, W, update) instead of read once per column.  One workgroup
// of 1024 threads per block, thread t holding the sketch column of column t.
// ----------------------------------------------------------------------------
constexpr int QS_P = QS_NB + 4;      // sketch rows

__device__ __forceinline__ uint32_t qs_mix(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}
// sign bits of the sketch drawn for the panel at column k0, for matrix row y:
// bit r set = entry (r, y) is -1
__device__ __forceinline__ uint32_t qs_signs(int y, int k0) {
  return qs_mix((uint32_t)y * 0x9e3779b9u + qs_mix((uint32_t)k0 + 0x632be5abu));
}

typedef double qs_d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ qs_d4 qs_mfma(double a, double b, qs_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ void qr_sketch(cd *A, int m, int n, cd *tau, int *piv, cd *S, double *s_dyn) {
  // S: the sketch (QS_P x n), in the block's R region
  cd *sW = reinterpret_cast<cd *>(s_dyn);               // [wave][16 columns][QS_NB]
  cd *sV = sW + 16 * 16 * QS_NB;                        // [row - k0][QS_NB]
  __shared__ cd s_T[QS_NB * QS_NB], s_vv[QS_NB * QS_NB];
  __shared__ cd s_x[QS_P], s_y[QS_P];
  __shared__ double s_bv[16], s_red[16];
  __shared__ int s_bi[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  if (tid < n) piv[tid] = tid;
  for (int k0 = 0; k0 < n; k0 += QS_NB) {
    const int b = min(QS_NB, n - k0), len0 = m - k0;
    // 0. sketch of the columns [k0, n) over rows [k0, m): S[r][j] = sum_y
    // Omega[r][y] A[y][j], by tiles of 16 columns (sketch rows in the real
    // A operand, the real and imaginary parts of A in two products)
    for (int j0 = k0 + 16 * wave; j0 < n; j0 += 16 * nw) {
      qs_d4 sr = {0.0, 0.0, 0.0, 0.0}, si = sr;
      const int j = j0 + lr;
      const cd *col = A + (size_t)min(j, n - 1) * m;
      for (int y0 = k0; y0 < m; y0 += 4) {
        const int y = y0 + lk;
        const bool in = y < m;
        const double om = (in && lr < QS_P) ? (((qs_signs(y, k0) >> lr) & 1u) ? -1.0 : 1.0) : 0.0;
        const cd a = (in && j < n) ? col[y] : cmk(0.0, 0.0);
        sr = qs_mfma(om, a.re, sr);
        si = qs_mfma(om, a.im, si);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * q + lk;
        if (r < QS_P && j < n) S[r + (size_t)QS_P * j] = cmk(sr[q], si[q]);
      }
    }
    __syncthreads();
    // 1. the panel's pivots: column-pivoted QR of the sketch columns [k0, n),
    // thread j holding column j
    cd sk[QS_P];
#pragma unroll
    for (int r = 0; r < QS_P; ++r)
      sk[r] = (tid >= k0 && tid < n) ? S[r + (size_t)QS_P * tid] : cmk(0.0, 0.0);
    for (int i = 0; i < b; ++i) {
      const int k = k0 + i;
      double bv = -1.0;
      int bi = n;
      if (tid >= k && tid < n) {
        double s2 = 0.0;
#pragma unroll
        for (int r = 0; r < QS_P; ++r)
          if (r >= i) s2 += cabs2(sk[r]);
        bv = s2;
        bi = tid;
      }
      wave_argmax(bv, bi);
      if (lane == 0) { s_bv[wave] = bv; s_bi[wave] = bi; }
      __syncthreads();
      int p;
      {
        double bb = s_bv[0];
        int pp = s_bi[0];
        for (int w2 = 1; w2 < nw; ++w2)
          if (s_bv[w2] > bb || (s_bv[w2] == bb && s_bi[w2] < pp)) { bb = s_bv[w2]; pp = s_bi[w2]; }
        p = pp < n ? pp : k;
      }
      if (p != k) {
        for (int y = tid; y < m; y += blockDim.x) {
          const cd t = A[(size_t)k * m + y];
          A[(size_t)k * m + y] = A[(size_t)p * m + y];
          A[(size_t)p * m + y] = t;
        }
        if (tid == p) {
#pragma unroll
          for (int r = 0; r < QS_P; ++r) s_x[r] = sk[r];
        }
        if (tid == k) {
#pragma unroll
          for (int r = 0; r < QS_P; ++r) s_y[r] = sk[r];
        }
        if (tid == 0) {
          const int t = piv[k];
          piv[k] = piv[p];
          piv[p] = t;
        }
        __syncthreads();
        if (tid == k) {
#pragma unroll
          for (int r = 0; r < QS_P; ++r) sk[r] = s_x[r];
        }
        if (tid == p) {
#pragma unroll
          for (int r = 0; r < QS_P; ++r) sk[r] = s_y[r];
        }
        __syncthreads();
      }
      if (tid == k) {
#pragma unroll
        for (int r = 0; r < QS_P; ++r) s_x[r] = sk[r];
      }
      __syncthreads();
      // reflector of the sketch column's rows i.. (every thread alike), applied
      // to the later sketch columns
      double s2 = 0.0;
#pragma unroll
      for (int r = 0; r < QS_P; ++r)
        if (r > i) s2 += cabs2(s_x[r]);
      cd ht, hs;
      double hb;
      const bool skip = !householder(s_x[i], s2, ht, hs, hb);
      if (!skip && tid > k && tid < n) {
        cd dv = sk[i];
#pragma unroll
        for (int r = 0; r < QS_P; ++r)
          if (r > i) cfma(dv, cconj(cmul(s_x[r], hs)), sk[r]);
        const cd f = cmul(cconj(ht), dv);             // conj(tau) v^H s
        sk[i] = csub(sk[i], f);
#pragma unroll
        for (int r = 0; r < QS_P; ++r)
          if (r > i) sk[r] = csub(sk[r], cmul(cmul(s_x[r], hs), f));
      }
      __syncthreads();
    }
    // 2. the panel: unpivoted Householder QR of A[k0:, k0:k0 + b]
    for (int i = 0; i < b; ++i) {
      const int k = k0 + i, len = m - k;
      cd *x = A + (size_t)k * m + k;
      double s2 = 0.0;
      for (int y = 1 + tid; y < len; y += blockDim.x) s2 += cabs2(x[y]);
      s2 = block_sum_keep(s2, s_red);
      cd h_tau, h_scale;
      double h_beta;
      const bool skip = !householder(x[0], s2, h_tau, h_scale, h_beta);
      if (!skip)
        for (int y = 1 + tid; y < len; y += blockDim.x) x[y] = cmul(x[y], h_scale);
      __syncthreads();
      if (tid == 0) {
        tau[k] = skip ? cmk(0.0, 0.0) : h_tau;
        if (!skip) x[0] = cmk(h_beta, 0.0);
      }
      const int c = k + 1 + wave;                     // one later panel column per wave
      if (!skip && c < k0 + b) {
        cd *a = A + (size_t)c * m + k;
        double dr = 0.0, di = 0.0;
        for (int y = lane; y < len; y += 64) {
          const cd v = y == 0 ? cmk(1.0, 0.0) : x[y];
          const cd q = cmulc(v, a[y]);
          dr += q.re;
          di += q.im;
        }
        dr = group_sum<64>(dr);
        di = group_sum<64>(di);
        const cd f = cmul(cconj(h_tau), cmk(dr, di));    // conj(tau) v^H a
        for (int y = lane; y < len; y += 64) {
          const cd v = y == 0 ? cmk(1.0, 0.0) : x[y];
          a[y] = csub(a[y], cmul(v, f));
        }
      }
      __syncthreads();
    }
    if (k0 + b >= n) break;
    // 3. V (rows k0.. of the panel's reflectors) into LDS, V^H V and T
    for (int idx = tid; idx < len0 * QS_NB; idx += blockDim.x) {
      const int yy = idx / QS_NB, c = idx - QS_NB * yy;
      cd v = cmk(0.0, 0.0);
      if (c < b) v = yy > c ? A[(size_t)(k0 + c) * m + k0 + yy] : (yy == c ? cmk(1.0, 0.0) : v);
      sV[idx] = v;
    }
    __syncthreads();
    for (int pi = wave; pi < b * (b - 1) / 2; pi += nw) {
      int c1 = 0, rem = pi;
      while (rem >= b - 1 - c1) { rem -= b - 1 - c1; ++c1; }
      const int c2 = c1 + 1 + rem;
      double vr = 0.0, vi = 0.0;
      for (int yy = c2 + lane; yy < len0; yy += 64) {
        const cd q = cmulc(sV[yy * QS_NB + c1], sV[yy * QS_NB + c2]);
        vr += q.re;
        vi += q.im;
      }
      vr = group_sum<64>(vr);
      vi = group_sum<64>(vi);
      if (lane == 0) s_vv[c1 * QS_NB + c2] = cmk(vr, vi);
    }
    __syncthreads();
    if (tid == 0) {
      for (int c = 0; c < QS_NB; ++c)
        for (int r = 0; r < QS_NB; ++r) s_T[r * QS_NB + c] = cmk(0.0, 0.0);
      for (int c = 0; c < b; ++c) {
        const cd tc = tau[k0 + c];
        for (int r = 0; r < c; ++r) {
          cd acc = cmk(0.0, 0.0);
          for (int q = r; q < c; ++q) cfma(acc, s_T[r * QS_NB + q], s_vv[q * QS_NB + c]);
          s_T[r * QS_NB + c] = cmk(-(tc.re * acc.re - tc.im * acc.im), -(tc.re * acc.im + tc.im * acc.re));
        }
        s_T[c * QS_NB + c] = tc;
      }
    }
    __syncthreads();
    // 4. the trailing columns [k0 + b, n) by tiles of 16 (one wave each)
    cd *wt = sW + (size_t)wave * 16 * QS_NB;
    for (int j0 = k0 + b + 16 * wave; j0 < n; j0 += 16 * nw) {
      const int j = j0 + lr;
      const bool cj = j < n;
      cd *col = A + (size_t)min(j, n - 1) * m + k0;
      // W = V^H A_t: rows c (Re W[c]) and 8 + c (Im W[c]); a step takes rows
      // yy = y0, y0 + 1 (k = lk: row y0 + lk / 2, real part when lk is even)
      qs_d4 wd = {0.0, 0.0, 0.0, 0.0};
      const int cv = lr & 7;
      const bool imrow = lr >= 8;
      for (int y0 = 0; y0 < len0; y0 += 2) {
        const int yy = y0 + (lk >> 1);
        const bool part = lk & 1;
        const bool in = yy < len0;
        const cd v = in ? sV[yy * QS_NB + cv] : cmk(0.0, 0.0);
        const double av = !imrow ? (part ? v.im : v.re) : (part ? v.re : -v.im);
        const cd a = (in && cj) ? col[yy] : cmk(0.0, 0.0);
        wd = qs_mfma(av, part ? a.im : a.re, wd);
      }
      // lane (lr, lk) holds Re W[lk], Re W[4 + lk], Im W[lk], Im W[4 + lk] of
      // column j; W' = T^H W per column through the wave's LDS tile
      wt[lr * QS_NB + lk] = cmk(wd[0], wd[2]);
      wt[lr * QS_NB + 4 + lk] = cmk(wd[1], wd[3]);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // the wave's LDS writes before its reads
      cd w2[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = lk + 4 * h;
        cd acc = cmk(0.0, 0.0);
        for (int c2 = 0; c2 <= c; ++c2) cfma(acc, cconj(s_T[c2 * QS_NB + c]), wt[lr * QS_NB + c2]);
        w2[h] = acc;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      wt[lr * QS_NB + lk] = w2[0];
      wt[lr * QS_NB + 4 + lk] = w2[1];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      // A_t -= V W' by 8-row tiles: output row R = 2 (yy - yb) + part; step s
      // takes reflectors 2 s, 2 s + 1 (k = lk: reflector 2 s + lk / 2, the
      // real part of W' when lk is even)
      for (int yb = 0; yb < len0; yb += 8) {
        qs_d4 d;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int R = 4 * q + lk, yy = yb + (R >> 1);
          const cd a = (yy < len0 && cj) ? col[yy] : cmk(0.0, 0.0);
          d[q] = (R & 1) ? a.im : a.re;
        }
        const int yy = yb + (lr >> 1);
        const bool opart = lr & 1;
#pragma unroll
        for (int s4 = 0; s4 < QS_NB / 2; ++s4) {
          const int c = 2 * s4 + (lk >> 1);
          const bool wpart = lk & 1;
          const cd v = yy < len0 ? sV[yy * QS_NB + c] : cmk(0.0, 0.0);
          // coefficient of W'[c].(wpart) in output (yy, opart), negated
          const double av = !opart ? (!wpart ? -v.re : v.im) : (!wpart ? -v.im : -v.re);
          const cd wv = wt[lr * QS_NB + c];             // B operand: W'[c][column lr]
          d = qs_mfma(av, wpart ? wv.im : wv.re, d);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int R = 4 * q + lk, yo = yb + (R >> 1);
          if (yo < len0 && cj) {
            double *dst = reinterpret_cast<double *>(col + yo);
            dst[R & 1] = d[q];
          }
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_qr(Layer ly, int max_chi, hipStream_t s) {
  if (ly.total_blocks == 0) return hipSuccess;
  (void)max_chi;
  const int lb = svd_lds_bytes();
  const int half = svd_panel_half(lb);
  hipLaunchKernelGGL(k_qr_order, dim3(1), dim3(1024), 0, s, ly);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the sketch path's static LDS exceeds the 2 KB the others leave
  const int qs_lds = lb - 2048;
  hipLaunchKernelGGL(k_qr_panel, dim3(ly.total_blocks), dim3(QRP_THREADS),
                     (size_t)(GBS_QR_SKETCH ? qs_lds : half), s, ly, half, qs_lds);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_qr, dim3(ly.total_blocks), dim3(QR_THREADS), (size_t)lb, s, ly, lb, qs_lds);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of every computed block.  For columns x, y of
// the operand with x^H y = |g| e^{i psi}:
//   zeta = (|y|^2 - |x|^2) / (2 |g|),  t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
//   c = 1 / sqrt(1 + t^2), s = c t,
//   x <- c x - s e^{-i psi} y,  y <- s x + c e^{-i psi} y.
// At convergence the operand is U Sigma with orthogonal columns.  The right
// factor is not accumulated: the kept right singular vectors are recovered in
// the scatter from the pristine operand, V[:, i] = A0^H u_i / sigma_i.
// Pairs with a column at the rounding floor are left alone (jacobi_floor).
//   * k_svd_small: the whole operand in LDS, one workgroup, round-robin pairs;
//   * big blocks: column panels of width w; each sweep is a round-robin
//     tournament of panel pairs, one launch per round, one workgroup per panel
//     pair holding its 2w columns in LDS (round 0 also rotates the pairs inside
//     each panel, later rounds only the cross pairs).
// ----------------------------------------------------------------------------
constexpr int SVD_THREADS = 512;
constexpr int MAX_SWEEPS = JACOBI_MAX_SWEEPS;
constexpr int RPL = 8;          // column rows cached per lane (m <= 512)

// Column pairs are rotated by groups of L lanes (L = 16: one DPP row, four
// pairs per wavefront; 32 or 64 when a round has too few pairs to keep every
// group busy).  Dot products reduce with DPP steps inside a row, plus one or
// two cross-row butterflies for L = 32, 64.
#ifndef GBS_CE
#define GBS_CE 8
#endif
constexpr int CE = GBS_CE;   // elements per lane kept in registers (m <= L * CE)

// One rotation of the column pair (x, y) by one group of L lanes (gl = lane
// in the group).  The squared norms al = |x|^2, be = |y|^2 are tracked in
// LDS: a rotation with tangent t changes them exactly to al - t |g| and
// be + t |g|; when either loses more than half it is recomputed from the
// rotated column.
// T is the complex type of the LDS operand (cd: FP64; cf: the FP32 Jacobi of
// the mixed-precision path); dot products and rotations run in its precision,
// the tracked norms and the rotation parameters in FP64.
// NC: row chunks of L per lane when the columns are cached in registers.  With
// NC = ceil(m / L) (the dispatched form) every chunk but the last is full and
// is loaded without a bound check; the default NC = CE serves any m <= L CE.
template <int L, typename T, int NC = CE>
__device__ __forceinline__ void jacobi_pair(T *xp, T *xq, double *nx, double *ny, int m,
                                            int gl, double tol, double tiny, int &rot) {
  using R = typename real_of<T>::type;
  const double al = *nx, be = *ny;
  if (fmin(al, be) <= tiny) return;
  R gr = 0, gi = 0;
  const bool exact = m > L * (NC - 1);
  const bool cached = m <= L * NC;
  T rx[NC], ry[NC];
  if (cached) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int i = gl + L * k;
      const bool in = (exact && k < NC - 1) || i < m;
      rx[k] = in ? xp[i] : T{0, 0};
      ry[k] = in ? xq[i] : T{0, 0};
      gr = fma(rx[k].re, ry[k].re, fma(rx[k].im, ry[k].im, gr));
      gi = fma(rx[k].re, ry[k].im, fma(-rx[k].im, ry[k].re, gi));
    }
  } else {
    for (int i = gl; i < m; i += L) {
      const T x = xp[i], y = xq[i];
      gr = fma(x.re, y.re, fma(x.im, y.im, gr));
      gi = fma(x.re, y.im, fma(-x.im, y.re, gi));
    }
  }
  const double grd = group_sum<L>(gr), gid = group_sum<L>(gi);
  const double ga2 = grd * grd + gid * gid;
  if (!(ga2 > tol * tol * (al * be)) || !(ga2 > 1e-300)) return;
  const double rga = rsqrt(ga2), ga = ga2 * rga;
  const double zeta = (be - al) * (0.5 * rga);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cd_ = rsqrt(1.0 + t * t);
  const double er = grd * rga, ei = -gid * rga;      // e^{-i psi}
  // x' = c x - (s e) y,  y' = s x + (c e) y
  const R c = (R)cd_, s = (R)(cd_ * t);
  const R ser = (R)(cd_ * t * er), sei = (R)(cd_ * t * ei);
  const R cer = (R)(cd_ * er), cei = (R)(cd_ * ei);
  double al2 = al - t * ga, be2 = be + t * ga;
  // the tracked norms lose accuracy when a column loses more than half of
  // its weight; then both are summed afresh from the rotated columns
  const bool renorm = !(al2 >= 0.5 * al) || !(be2 >= 0.5 * be);
  R na = 0, nb = 0;
  auto rotate = [&](const T x, const T y, T &x2, T &y2) {
    x2.re = fma(-ser, y.re, fma(sei, y.im, c * x.re));
    x2.im = fma(-ser, y.im, fma(-sei, y.re, c * x.im));
    y2.re = fma(cer, y.re, fma(-cei, y.im, s * x.re));
    y2.im = fma(cer, y.im, fma(cei, y.re, s * x.im));
  };
  if (cached) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int i = gl + L * k;
      if ((exact && k < NC - 1) || i < m) {
        T x2, y2;
        rotate(rx[k], ry[k], x2, y2);
        xp[i] = x2;
        xq[i] = y2;
        if (renorm) {
          na += cabs2(x2);
          nb += cabs2(y2);
        }
      }
    }
  } else {
    for (int i = gl; i < m; i += L) {
      T x2, y2;
      rotate(xp[i], xq[i], x2, y2);
      xp[i] = x2;
      xq[i] = y2;
      if (renorm) {
        na += cabs2(x2);
        nb += cabs2(y2);
      }
    }
  }
  if (renorm) {              // uniform over the group
    al2 = group_sum<L>(na);
    be2 = group_sum<L>(nb);
  }
  if (gl == 0) {
    *nx = al2;
    *ny = be2;
  }
  rot = 1;
}

// Squared norms of the nc columns at A (column stride m) into nrm.
template <typename T>
__device__ __forceinline__ void column_norms(const T *A, int m, int nc, double *nrm) {
  using R = typename real_of<T>::type;
  const int gl = threadIdx.x & 15, slot = threadIdx.x >> 4;
  const int ns = blockDim.x >> 4;
  for (int c = slot; c < nc; c += ns) {
    R acc = 0;
    for (int i = gl; i < m; i += 16) acc += cabs2(A[(size_t)c * m + i]);
    acc = group_sum<16>(acc);
    if (gl == 0) nrm[c] = acc;
  }
  __syncthreads();
}

// Unit roundoff of the Jacobi's working precision.
template <typename T> __device__ __forceinline__ double unit_eps();
template <> __device__ __forceinline__ double unit_eps<cd>() { return 1.11e-16; }
template <> __device__ __forceinline__ double unit_eps<cf>() { return 5.96e-8; }

// Relative orthogonality tolerance: max(9 eps, 2.07 eps m) (1e-15 and
// 2.3e-16 m in FP64).
template <typename T = cd>
__device__ __forceinline__ double jacobi_tol(int m) {
  return fmax(9.0 * unit_eps<T>(), 2.07 * unit_eps<T>() * m);
}

// Rounding floor of a column's squared norm: a column of an operand with
// squared Frobenius norm fro2 whose own squared norm is below 16 m eps^2 fro2
// holds nothing but rounding noise, and its orthogonality to any other column
// cannot be resolved to the relative tolerance (rotating such pairs never
// settles).  Pairs with either column below the floor are left alone; their
// singular values lie far below the 1e-14 rank cut.
template <typename T = cd>
__device__ __forceinline__ double jacobi_floor(int m, double fro2) {
  return 16.0 * m * (unit_eps<T>() * unit_eps<T>()) * fro2;
}

// The Jacobi operand of a computed block: R of a QR'd block, else the block.
__device__ __forceinline__ cd *jacobi_operand(const Layer &ly, const GateBase &gb,
                                              const BlkDesc &B) {
  return B.qr ? ly.R + gb.r + B.joff : ly.A + gb.e + B.eoff;
}

// One round-robin pass over all pairs of the nc columns at A (column stride m,
// squared norms in nrm), L lanes per pair.
template <int L, typename T, int NC = CE>
__device__ __forceinline__ void round_robin_pass_l(T *A, double *nrm, int m, int nc, double tol,
                                                   double tiny, int &rot) {
  const int gl = threadIdx.x & (L - 1), slot = threadIdx.x / L;
  const int ns = blockDim.x / L;
  const int np = nc + (nc & 1);
  for (int round = 0; round < np - 1; ++round) {
    for (int k = slot; k < np / 2; k += ns) {
      int p, q;
      if (k == 0) {
        p = round;
        q = np - 1;
      } else {
        p = (round + k) % (np - 1);
        q = (round - k + np - 1) % (np - 1);
      }
      if (p >= nc || q >= nc) continue;
      jacobi_pair<L, T, NC>(A + (size_t)p * m, A + (size_t)q * m, nrm + p, nrm + q, m, gl, tol,
                            tiny, rot);
    }
    __syncthreads();
  }
}

// Lanes per column pair in the one-workgroup Jacobi and in the panel rounds.
#ifndef GBS_SMALL_LANES
#define GBS_SMALL_LANES 16
#endif
#ifndef GBS_PANEL_LANES
#define GBS_PANEL_LANES 32
#endif
#ifndef GBS_PANEL_WIDE
#define GBS_PANEL_WIDE 1
#endif

// Cross pairs of two panels held in LDS (wI columns then wJ columns, panel
// width w): w sub-rounds, column t of the first panel with (t + sr) mod w of
// the second; L lanes per pair.
template <int L, typename T>
__device__ __forceinline__ void cross_pass_l(T *sA, double *nrm, int m, int w, int wI, int wJ,
                                             double tol, double tiny, int &rot) {
  const int gl = threadIdx.x & (L - 1), slot = threadIdx.x / L;
  const int ns = blockDim.x / L;
  for (int sr = 0; sr < w; ++sr) {
    for (int t = slot; t < wI; t += ns) {
      const int u = (t + sr) % w;
      if (u >= wJ) continue;
      jacobi_pair<L>(sA + (size_t)t * m, sA + (size_t)(wI + u) * m, nrm + t, nrm + wI + u, m, gl,
                     tol, tiny, rot);
    }
    __syncthreads();
  }
}

// The same cross pairs when every pair takes a whole wavefront and the
// columns fit in registers (m <= 64 CE): column t of the first panel stays
// with wave t for all w sub-rounds, so only the second panel's columns pass
// through LDS.  Every rotation is computed exactly as jacobi_pair<64> does
// (same operands, same operation order), so the result is bitwise the same;
// only the first panel's LDS loads and stores per sub-round are saved.
// NC = ceil(m / 64) row chunks per lane (m <= 64 NC): all but the last are
// full and carry no bound check.
template <typename T, int NC>
__device__ __forceinline__ void cross_pass_stationary(T *sA, double *nrm, int m, int w, int wI,
                                                      int wJ, double tol, double tiny, int &rot) {
  using R = typename real_of<T>::type;
  const int gl = threadIdx.x & 63, t = threadIdx.x >> 6;
  const bool own = t < wI;
  T rx[NC];
  double nx = 0.0;
  if (own) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int i = gl + 64 * k;
      rx[k] = (k < NC - 1 || i < m) ? sA[(size_t)t * m + i] : T{0, 0};
    }
    nx = nrm[t];
  }
  int u = t;                   // (t + sr) mod w, stepped per sub-round
  for (int sr = 0; sr < w; ++sr, u = (u + 1 == w) ? 0 : u + 1) {
    if (own && u < wJ) {
      T *yq = sA + (size_t)(wI + u) * m;
      double *ny = nrm + wI + u;
      const double al = nx, be = *ny;
      if (fmin(al, be) > tiny) {
        R gr = 0, gi = 0;
        T ry[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          const int i = gl + 64 * k;
          ry[k] = (k < NC - 1 || i < m) ? yq[i] : T{0, 0};
          gr = fma(rx[k].re, ry[k].re, fma(rx[k].im, ry[k].im, gr));
          gi = fma(rx[k].re, ry[k].im, fma(-rx[k].im, ry[k].re, gi));
        }
        const double grd = group_sum<64>(gr), gid = group_sum<64>(gi);
        const double ga2 = grd * grd + gid * gid;
        if ((ga2 > tol * tol * (al * be)) && (ga2 > 1e-300)) {
          const double rga = rsqrt(ga2), ga = ga2 * rga;
          const double zeta = (be - al) * (0.5 * rga);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cd_ = rsqrt(1.0 + tt * tt);
          const double er = grd * rga, ei = -gid * rga;
          const R c = (R)cd_, s = (R)(cd_ * tt);
          const R ser = (R)(cd_ * tt * er), sei = (R)(cd_ * tt * ei);
          const R cer = (R)(cd_ * er), cei = (R)(cd_ * ei);
          double al2 = al - tt * ga, be2 = be + tt * ga;
          const bool renorm = !(al2 >= 0.5 * al) || !(be2 >= 0.5 * be);
          R na = 0, nb = 0;
#pragma unroll
          for (int k = 0; k < NC; ++k) {
            const int i = gl + 64 * k;
            if (k < NC - 1 || i < m) {
              const T x = rx[k], y = ry[k];
              T x2, y2;
              x2.re = fma(-ser, y.re, fma(sei, y.im, c * x.re));
              x2.im = fma(-ser, y.im, fma(-sei, y.re, c * x.im));
              y2.re = fma(cer, y.re, fma(-cei, y.im, s * x.re));
              y2.im = fma(cer, y.im, fma(cei, y.re, s * x.im));
              rx[k] = x2;
              yq[i] = y2;
              if (renorm) {
                na += cabs2(x2);
                nb += cabs2(y2);
              }
            }
          }
          if (renorm) {
            al2 = group_sum<64>(na);
            be2 = group_sum<64>(nb);
          }
          nx = al2;
          if (gl == 0) *ny = be2;
          rot = 1;
        }
      }
    }
    __syncthreads();
  }
  if (own) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int i = gl + 64 * k;
      if (k < NC - 1 || i < m) sA[(size_t)t * m + i] = rx[k];
    }
    if (gl == 0) nrm[t] = nx;
  }
  __syncthreads();
}

// Calls F.template operator()<NC>() with NC = ceil(m / L) for m <= L CE
// (register-cached columns, exact chunk count), else with NC = CE.
template <int L, typename F>
__device__ __forceinline__ void with_chunks(int m, F &&f) {
  static_assert(CE == 8, "chunk dispatch written for eight chunks");
  switch ((m + L - 1) / L) {
    case 1: f.template operator()<1>(); break;
    case 2: f.template operator()<2>(); break;
    case 3: f.template operator()<3>(); break;
    case 4: f.template operator()<4>(); break;
    case 5: f.template operator()<5>(); break;
    case 6: f.template operator()<6>(); break;
    case 7: f.template operator()<7>(); break;
    default: f.template operator()<CE>(); break;
  }
}

__device__ __forceinline__ double block_sum(double v, double *s_red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s_red[w];
  __syncthreads();
  return t;
}

// Workgroup copies between global memory and LDS with eight loads in flight
// per thread (a plain loop waits for each load before the next).
// (scaled by sc on the way in and by 1 / sc on the way out: the FP32 Jacobi
// works on the operand normalised to unit Frobenius norm, so that sectors of
// tiny weight do not underflow in single precision)
template <typename T>
__device__ __forceinline__ void copy_in(T *dst, const cd *src, int count, double sc = 1.0) {
  const int step = blockDim.x;
  for (int base = threadIdx.x; base < count; base += 8 * step) {
    cd r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * step;
      if (idx < count) r[u] = src[idx];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * step;
      if (idx < count) dst[idx] = to_c<T>(sc == 1.0 ? r[u] : cscale(r[u], sc));
    }
  }
}

template <typename T>
__device__ __forceinline__ void copy_out(cd *dst, const T *src, int count, double isc = 1.0) {
  for (int idx = threadIdx.x; idx < count; idx += blockDim.x)
    dst[idx] = isc == 1.0 ? to_cd(src[idx]) : cscale(to_cd(src[idx]), isc);
}

// Scale applied to an operand of squared Frobenius norm fro2 before its
// Jacobi: 1 in FP64, 1 / |A|_F in FP32.
template <typename T> __device__ __forceinline__ double jacobi_scale(double fro2);
template <> __device__ __forceinline__ double jacobi_scale<cd>(double) { return 1.0; }
template <> __device__ __forceinline__ double jacobi_scale<cf>(double fro2) {
  return fro2 > 0.0 ? 1.0 / sqrt(fro2) : 1.0;
}

// Self-mirror block (q = (n, n)) of a Hermitian state: the block obeys
// Theta[a~, b~] = conj(Theta[a, b]) (a~ the mirror index), so each
// non-degenerate singular vector is J-real up to a phase: u[y~] = e^{i phi}
// conj(u[y]) on the operand's rows.  The bilinear sum s = sum_y u[y] u[y~] =
// e^{i phi} |u|^2 gives the phase and the column is multiplied by e^{-i phi/2}.
template <typename T>
__device__ __forceinline__ void self_mirror_phase(const Layer &ly, const GateParam &gp,
                                                  const BlkDesc &B, T *A) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int m = B.m, n = B.n;
  // operand rows: left-bond indices (stored Theta) or right-bond indices (Theta^T)
  const int *lst = !B.t ? ly.rows + gp.lst0 + B.roff : ly.cols + gp.lst0 + B.coff;
  const int *my = (!B.t ? ly.mirL : ly.mirR) + gp.mir0;
  for (int c = wave; c < n; c += nw) {
    double sr = 0.0, si = 0.0, nr = 0.0;
    for (int y = lane; y < m; y += 64) {
      const int ym = lower_bound(lst, m, my[lst[y]]);
      const cd x = to_cd(A[(size_t)c * m + y]), z = to_cd(A[(size_t)c * m + ym]);
      const cd p = cmul(x, z);
      sr += p.re;
      si += p.im;
      nr += cabs2(x);
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    nr = wave_sum(nr);
    const double sa = sqrt(sr * sr + si * si);
    if (sa > 0.5 * nr && sa > 0.0) {
      const double ang = -0.5 * atan2(si, sr);
      const cd f = cmk(cos(ang), sin(ang));
      for (int i = lane; i < m; i += 64)
        A[(size_t)c * m + i] = to_c<T>(cmul(to_cd(A[(size_t)c * m + i]), f));
    }
  }
  __syncthreads();
}

// Singular values = column norms, sorted descending (ties by column).
template <typename T>
__device__ __forceinline__ void sort_values(int *err, const T *A, int m, int n, double *sig,
                                            double *sv, int *perm, double vscale = 1.0) {
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < m; ++i) acc += cabs2(to_cd(A[(size_t)c * m + i]));
    sig[c] = sqrt(acc) * vscale;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const double v = sig[c];
    int rank = 0;
    for (int o = 0; o < n; ++o) {
      const double w = sig[o];
      rank += (w > v) || (w == v && o < c);
    }
    sv[rank] = v;
    perm[rank] = c;
    if (!isfinite(v)) atomicOr(err, ERR_NONFINITE);
  }
}

__device__ inline void big_block_of(const Layer &ly, int flat_big, int &g, int &bi) {
  g = find_gate_big(ly.base, ly.ngates, flat_big);
  bi = ly.bigl[ly.gates[g].lst0 + (flat_big - ly.base[g].big)];
}

// One workgroup per block whose LDS need lies in (lo, hi] (the launches are
// split by size so that small blocks do not reserve a whole CU's LDS).
template <typename T>
__global__ __launch_bounds__(SVD_THREADS) void k_svd_small(Layer ly, int lo, int hi) {
  const int flat = blockIdx.x;
  const int g = find_gate_blk(ly.base, ly.ngates, flat);
  const GateBase gb = ly.base[g];
  const GateParam gp = ly.gates[g];
  const State st = ly.states[gp.inst];
  BlkDesc *Bp = ly.blk + gp.blk0 + (flat - gb.blk);
  const BlkDesc B = *Bp;
  if (!B.comp || B.big) return;
  {
    const long long need = (long long)svd_small_need(B.mj, B.n, (int)sizeof(T));
    if (need <= lo || need > hi) return;
  }
  const int m = B.mj, n = B.n;
  extern __shared__ __attribute__((aligned(16))) double s_dyn[];
  T *sA = reinterpret_cast<T *>(s_dyn);                  // m x n operand
  double *sig = reinterpret_cast<double *>(sA + (size_t)m * n);   // n column norms^2
  __shared__ int s_rot;
  __shared__ double s_red[16];
  cd *A = jacobi_operand(ly, gb, B);
  double f2 = 0.0;
  for (int i = threadIdx.x; i < m * n; i += blockDim.x) f2 += cabs2(A[i]);
  f2 = block_sum(f2, s_red);
  const double sc = jacobi_scale<T>(f2);
  copy_in(sA, A, m * n, sc);
  __syncthreads();
  const double tol = jacobi_tol<T>(m), tiny = jacobi_floor<T>(m, f2 * sc * sc);
  int sweep = 0;
  const int msw = min(MAX_SWEEPS, st.max_sweeps);
  if (n > 1) {
    for (sweep = 0; sweep < msw; ++sweep) {
      if (threadIdx.x == 0) s_rot = 0;
      column_norms(sA, m, n, sig);
      int rot = 0;
      with_chunks<GBS_SMALL_LANES>(m, [&]<int NC>() {
        round_robin_pass_l<GBS_SMALL_LANES, T, NC>(sA, sig, m, n, tol, tiny, rot);
      });
      if (rot) s_rot = 1;
      __syncthreads();
      const int any = s_rot;
      __syncthreads();
      if (!any) break;
    }
    if (sweep == msw && threadIdx.x == 0) atomicOr(st.err, ERR_SVD_NOT_CONVERGED);
  }
  if (!B.qr && charge_n(B.q) == charge_np(B.q) && ly.tot[g].sym) self_mirror_phase(ly, gp, B, sA);
  sort_values(st.err, sA, m, n, sig, ly.sv + gp.lst0 + B.svoff, ly.perm + gp.lst0 + B.svoff,
              1.0 / sc);
  copy_out(A, sA, m * n, 1.0 / sc);
  if (threadIdx.x == 0) {
    Bp->sweeps = sweep;
    Bp->fro2 = f2;
  }
}

// Blocks with at most PANEL_VERSION_MAX panels (after rounding up to even)
// keep panel versions and per-pair verification records (see k_panel):
// PVER_STRIDE ints per big block, versions first, then the pair table.
constexpr int PANEL_VERSION_MAX = 64;
constexpr int PVER_STRIDE = PANEL_VERSION_MAX + PANEL_VERSION_MAX * PANEL_VERSION_MAX;

// Big blocks: squared Frobenius norm and cleared convergence flags.
// rotf[4k + (s % 3)]: a rotation happened in sweep s; rotf[4k + 3]: converged
// at that sweep (0 while running).
__global__ __launch_bounds__(256) void k_big_prep(Layer ly) {
  int g, bi;
  big_block_of(ly, blockIdx.x, g, bi);
  BlkDesc *Bp = ly.blk + ly.gates[g].blk0 + bi;
  const GateBase gb = ly.base[g];
  const cd *A = jacobi_operand(ly, gb, *Bp);
  __shared__ double s_red[16];
  double f2 = 0.0;
  for (long long i = threadIdx.x; i < (long long)Bp->mj * Bp->n; i += blockDim.x) f2 += cabs2(A[i]);
  f2 = block_sum(f2, s_red);
  if (threadIdx.x == 0) {
    Bp->fro2 = f2;
    int *rf = ly.rotf + 4 * (size_t)blockIdx.x;
    rf[0] = rf[1] = rf[2] = rf[3] = 0;
  }
  // panel versions 0, no pair verified yet
  int *pv = ly.pver + (size_t)blockIdx.x * PVER_STRIDE;
  for (int i = threadIdx.x; i < PVER_STRIDE; i += blockDim.x) pv[i] = i < PANEL_VERSION_MAX ? 0 : -1;
}

#ifndef GBS_PANEL_THREADS
#define GBS_PANEL_THREADS 1024
#endif

constexpr int PANEL_THREADS = GBS_PANEL_THREADS;

// Launch t of the panel rounds: every big block runs its own sequence of
// sweeps, Pp - 1 rounds each (Pp = panel count rounded up to even), so block
// b is at sweep t / (Pp_b - 1), round t mod (Pp_b - 1): blocks with few
// panels do not wait for the rounds of the largest ones.
template <typename T>
__global__ __launch_bounds__(PANEL_THREADS) void k_panel(Layer ly, int step) {
  // task -> (still-rotating big block, panel pair) through the compacted list
  const int task = blockIdx.x;
  int lo = 0, hi = ly.nact;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ly.task_pre[mid] <= task) lo = mid; else hi = mid;
  }
  const int kbig = ly.task_blk[lo];
  const int kpair = task - ly.task_pre[lo];
  int g, bi;
  big_block_of(ly, kbig, g, bi);
  const BlkDesc B = ly.blk[ly.gates[g].blk0 + bi];
  const int P = B.npan, Pp = P + (P & 1);
  if (kpair >= Pp / 2) return;
  const int sweep = step / (Pp - 1), round = step % (Pp - 1);
  if (sweep >= min(MAX_SWEEPS, ly.states[ly.gates[g].inst].max_sweeps)) return;
  int *rf = ly.rotf + 4 * (size_t)kbig;
  if (rf[3]) return;
  if (round == 0 && sweep > 0 && rf[(sweep - 1) % 3] == 0) {   // previous sweep: no rotation
    if (threadIdx.x == 0) rf[3] = sweep;
    return;
  }
  if (round == 0 && kpair == 0 && threadIdx.x == 0) rf[(sweep + 1) % 3] = 0;
  const int k = kpair;
  int I, J;
  if (k == 0) {
    I = round;
    J = Pp - 1;
  } else {
    I = (round + k) % (Pp - 1);
    J = (round - k + Pp - 1) % (Pp - 1);
  }
  const int m = B.mj, n = B.n, w = B.w;
  const bool hasI = I < P, hasJ = J < P;
  if (!(hasI && hasJ) && round != 0) return;     // a lone panel only rotates in round 0
  if (!hasI && !hasJ) return;
  // Panel versions (count of write-backs) and, per panel pair, the versions
  // at which the pair was last found orthogonal (no rotation in its task).
  // A cross round whose two panels have not changed since then would find
  // the same columns, compute the same dot products and rotate nothing, so it
  // is skipped; results are bitwise those of running it.
  const bool versioned = Pp <= PANEL_VERSION_MAX;
  int *pv = ly.pver + (size_t)kbig * PVER_STRIDE;
  int *prec = pv + PANEL_VERSION_MAX;
  const int plo = min(I, J), phi = max(I, J);
  const bool track = versioned && hasI && hasJ && round != 0;
  if (track && prec[plo * PANEL_VERSION_MAX + phi] == ((pv[plo] << 16) | pv[phi])) return;
  const int i0 = hasI ? I * w : 0, wI = hasI ? min(w, n - I * w) : 0;
  const int j0 = hasJ ? J * w : 0, wJ = hasJ ? min(w, n - J * w) : 0;
  const int nc = wI + wJ;
  extern __shared__ __attribute__((aligned(16))) double s_dyn[];
  T *sA = reinterpret_cast<T *>(s_dyn);
  cd *A = jacobi_operand(ly, ly.base[g], B);
  // the two panels are contiguous column ranges of the operand
  const double sc = jacobi_scale<T>(B.fro2);
  copy_in(sA, A + (size_t)i0 * m, wI * m, sc);
  copy_in(sA + (size_t)wI * m, A + (size_t)j0 * m, wJ * m, sc);
  __syncthreads();
  const double tol = jacobi_tol<T>(m), tiny = jacobi_floor<T>(m, B.fro2 * sc * sc);
  __shared__ double s_nrm[64];
  column_norms(sA, m, nc, s_nrm);
  int rot = 0;
  // panels of at most one pair per 64-lane slot take whole wavefronts per
  // pair: half the elements per lane (long columns stay in registers) for
  // one more, cheap, lane-swap step of every reduction
  if (w * 64 <= (int)blockDim.x && GBS_PANEL_WIDE) {
    if (round == 0)
      with_chunks<64>(m, [&]<int NC>() { round_robin_pass_l<64, T, NC>(sA, s_nrm, m, nc, tol, tiny, rot); });
    else if (m <= 64 * CE)
      with_chunks<64>(m, [&]<int NC>() {
        cross_pass_stationary<T, NC>(sA, s_nrm, m, w, wI, wJ, tol, tiny, rot);
      });
    else
      cross_pass_l<64>(sA, s_nrm, m, w, wI, wJ, tol, tiny, rot);
  } else if (round == 0) {
    round_robin_pass_l<GBS_PANEL_LANES>(sA, s_nrm, m, nc, tol, tiny, rot);
  } else {
    cross_pass_l<GBS_PANEL_LANES>(sA, s_nrm, m, w, wI, wJ, tol, tiny, rot);
  }
  __shared__ int s_any;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  if (rot) s_any = 1;
  __syncthreads();
  if (s_any && threadIdx.x == 0) rf[sweep % 3] = 1;
  if (!s_any) {                // nothing rotated: the panels in memory are unchanged
    if (track && threadIdx.x == 0)
      prec[plo * PANEL_VERSION_MAX + phi] = (pv[plo] << 16) | pv[phi];
    return;
  }
  copy_out(A + (size_t)i0 * m, sA, wI * m, 1.0 / sc);
  copy_out(A + (size_t)j0 * m, sA + (size_t)wI * m, wJ * m, 1.0 / sc);
  if (versioned && threadIdx.x == 0) {
    if (hasI) ++pv[I];
    if (hasJ) ++pv[J];
  }
}

// ----------------------------------------------------------------------------
// Panel rounds in Gram form (the FP64 path).  A task's two panels (at most 16
// columns each; padded index space of 32: panel I at 0..15, panel J at
// 16..31) are not staged in LDS.  Their Gram matrix G = X^H X is formed on
// the FP64 matrix cores straight from global memory; the task's rotations
// (the same pairs, in the same order, as the column passes above) are
// computed from G and applied to it from both sides, G <- J^H G J, while
// their product W = J_1 J_2 ... accumulates; then the columns receive all of
// them at once, X <- X W, again on the matrix cores.  The rotation of a pair
// (p, q) with g = G[p][q], al = G[p][p], be = G[q][q] follows the formulas of
// the column passes (zeta, t, c, s and e = conj(g) / |g|): column p of J is
// c on row p and -s e on row q, column q is s on row p and c e on row q.  In
// exact arithmetic the rotations are those of the column passes; G holds the
// same inner products (each rounded once per update instead of recomputed),
// and the final pass with no rotation decides convergence on a G formed
// afresh from the columns.  LDS: G double-buffered, 33 KB; W lives in the
// registers of the three updating waves during the rotations and passes
// through LDS once before the product, so four tasks share a CU.
// ----------------------------------------------------------------------------
constexpr int PG_THREADS = 256;     // wave 0 forms rotations, waves 1..3 update
constexpr int PG_N = 32;
constexpr int PG_WROWS = 6;         // rows of W per updating half-wave (6 x 6 >= 32)
typedef double pg_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ pg_d4 pg_mfma(double a, double b, pg_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Complex products in a fixed sequence of fused operations (every caller
// rounds alike).
__device__ __forceinline__ cd pg_mul(cd a, cd b) {          // a b
  return cmk(fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re));
}
__device__ __forceinline__ cd pg_mulc(cd a, cd b) {         // conj(a) b
  return cmk(fma(a.re, b.re, a.im * b.im), fma(a.re, b.im, -(a.im * b.re)));
}
__device__ __forceinline__ cd pg_fma(cd a, cd b, cd c) {    // a b + c
  return cmk(fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im)));
}

// Entry (i, j), i <= j, of J^H G J for the round's coefficients: self[k] =
// J[k][k], other[k] = J[part[k]][k], part[k] = partner of k (k itself, with
// self 1 and other 0, when k is not rotated).  Branch-free and in one fixed
// sequence of operations, so that the threads forming the next round's
// rotations get the very bits the update writes.
__device__ __forceinline__ cd pg_entry(const cd *G, int i, int j, const cd *self, const cd *other,
                                       const int *part) {
  const int pi = part[i], pj = part[j];
  const cd ai = self[i], bi = other[i], aj = self[j], bj = other[j];
  const cd t1 = pg_fma(G[i * 32 + pj], bj, pg_mul(G[i * 32 + j], aj));
  const cd t2 = pg_fma(G[pi * 32 + pj], bj, pg_mul(G[pi * 32 + j], aj));
  cd v = pg_mulc(ai, t1);
  const cd u = pg_mulc(bi, t2);
  v = cmk(v.re + u.re, v.im + u.im);
  if (i == j) v.im = 0.0;
  return v;
}

// Whether the pair with al = |x_p|^2, be = |x_q|^2, g = x_p^H x_q rotates
// (the tests of the column passes).
__device__ __forceinline__ bool pg_active(double al, double be, cd gq, double tol, double tiny) {
  const double ga2 = gq.re * gq.re + gq.im * gq.im;
  return fmin(al, be) > tiny && (ga2 > tol * tol * (al * be)) && (ga2 > 1e-300);
}

// Partner of padded index k in inner round rr of a task (round 0: the
// round-robin pairs of the compact columns, I's then J's; other rounds: the
// cross pairs (t, wI + (t + rr) mod w)); isp: k is the pair's first column.
__device__ __forceinline__ int pg_partner(int k, int rr, bool round0, int wI, int wJ, int w,
                                          bool &isp) {
  isp = false;
  const int nc = wI + wJ;
  if (round0) {
    const int ck = k < 16 ? (k < wI ? k : -1) : (k - 16 < wJ ? wI + (k - 16) : -1);
    if (ck < 0 || nc < 2) return -1;
    const int npc = nc + (nc & 1);
    int pc;
    if (ck == npc - 1) {
      pc = rr;
    } else if (ck == rr) {
      pc = npc - 1;
      isp = true;
    } else {
      // ck, rr < npc - 1: every sum below lies in [0, 2 (npc - 1))
      const int mod = npc - 1;
      int s1 = ck - rr + mod;
      if (s1 >= mod) s1 -= mod;
      if (s1 <= npc / 2 - 1) {
        isp = true;
        pc = rr - s1 + mod;
      } else {
        pc = rr + (mod - s1);
      }
      if (pc >= mod) pc -= mod;
    }
    return pc < nc ? (pc < wI ? pc : 16 + (pc - wI)) : -1;
  }
  // k - 16, rr < w here
  if (k < 16) {
    if (k >= wI) return -1;
    const int u = k + rr >= w ? k + rr - w : k + rr;
    isp = true;
    return u < wJ ? 16 + u : -1;
  }
  if (k - 16 >= wJ) return -1;
  const int t = k - 16 - rr < 0 ? k - 16 - rr + w : k - 16 - rr;
  return t < wI ? t : -1;
}

__global__ __launch_bounds__(PG_THREADS, 4) void k_panel_gram(Layer ly, int step) {
  const int task = blockIdx.x;
  int lo = 0, hi = ly.nact;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ly.task_pre[mid] <= task) lo = mid; else hi = mid;
  }
  const int kbig = ly.task_blk[lo];
  const int kpair = task - ly.task_pre[lo];
  int g, bi;
  big_block_of(ly, kbig, g, bi);
  const BlkDesc B = ly.blk[ly.gates[g].blk0 + bi];
  const int P = B.npan, Pp = P + (P & 1);
  if (kpair >= Pp / 2) return;
  const int sweep = step / (Pp - 1), round = step % (Pp - 1);
  if (sweep >= min(MAX_SWEEPS, ly.states[ly.gates[g].inst].max_sweeps)) return;
  int *rf = ly.rotf + 4 * (size_t)kbig;
  if (rf[3]) return;
  if (round == 0 && sweep > 0 && rf[(sweep - 1) % 3] == 0) {   // previous sweep: no rotation
    if (threadIdx.x == 0) rf[3] = sweep;
    return;
  }
  if (round == 0 && kpair == 0 && threadIdx.x == 0) rf[(sweep + 1) % 3] = 0;
  int I, J;
  if (kpair == 0) {
    I = round;
    J = Pp - 1;
  } else {
    I = (round + kpair) % (Pp - 1);
    J = (round - kpair + Pp - 1) % (Pp - 1);
  }
  const int m = B.mj, n = B.n, w = B.w;
  const bool hasI = I < P, hasJ = J < P;
  if (!(hasI && hasJ) && round != 0) return;     // a lone panel only rotates in round 0
  if (!hasI && !hasJ) return;
  // panel versions and verification records, as in k_panel
  const bool versioned = Pp <= PANEL_VERSION_MAX;
  int *pv = ly.pver + (size_t)kbig * PVER_STRIDE;
  int *prec = pv + PANEL_VERSION_MAX;
  const int plo = min(I, J), phi = max(I, J);
  const bool track = versioned && hasI && hasJ && round != 0;
  if (track && prec[plo * PANEL_VERSION_MAX + phi] == ((pv[plo] << 16) | pv[phi])) return;
  const int i0 = hasI ? I * w : 0, wI = hasI ? min(w, n - I * w) : 0;
  const int j0 = hasJ ? J * w : 0, wJ = hasJ ? min(w, n - J * w) : 0;
  const int nc = wI + wJ;
  cd *A = jacobi_operand(ly, ly.base[g], B);
  __shared__ cd sG[2][PG_N * PG_N];      // G[i][j] at i * PG_N + j; W before the product
  __shared__ cd s_self[2][PG_N], s_other[2][PG_N];   // J[i][i], J[partner(i)][i]
  __shared__ int s_part[2][PG_N];        // partner of i in the round (i itself: none)
  __shared__ int s_rot[2];               // the round rotates some pair
  __shared__ unsigned s_touch;           // padded indices rotated in some round
  __shared__ int s_pre;                  // some pair of the task passes the tests on the fresh Gram
  __shared__ int s_any;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  if (threadIdx.x == 0) s_pre = 0;
  // global column of padded index k, -1 when there is none
  auto col_of = [&](int k) -> int {
    if (k < 16) return k < wI ? i0 + k : -1;
    return k - 16 < wJ ? j0 + (k - 16) : -1;
  };
  // 1. the Gram tiles (I, I), (I, J), (J, J): wave v takes rows [v R, v R +
  // R) of all three from one set of loads (lane (lr, lk) feeds column lr of
  // each panel at row y + lk; tile entry [i][j] = sum_y conj(X[y][P + i])
  // X[y][Q + j] lands in lane (lr = j, lk) register r with i = 4 r + lk), 16
  // rows' loads in flight together (the registers a second batch would take
  // hold the third accumulator of the (I, J) block); the four partial Grams
  // are then summed pairwise.
  {
    const int cI = col_of(lr), cJ = col_of(16 + lr);
    const cd *xi = cI >= 0 ? A + (size_t)cI * m : nullptr;
    const cd *xj = cJ >= 0 ? A + (size_t)cJ * m : nullptr;
    const int R = ((m + 4 * nwv * 4 - 1) / (4 * nwv * 4)) * 16;     // rows per wave, multiple of 16
    const int ya = min(m, wave * R), yb = min(m, ya + R);
    pg_d4 ar = {0.0, 0.0, 0.0, 0.0}, ai = ar, br = ar, bq = ar, bi = ar, cr = ar, ci = ar;
    constexpr int GB = 4;                              // 4-row steps per batch
    cd a[GB], b[GB];
    auto load = [&](int y0, cd *ra, cd *rb) {
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        const int y = y0 + 4 * u + lk;
        ra[u] = (xi && y < yb) ? xi[y] : cmk(0.0, 0.0);
        rb[u] = (xj && y < yb) ? xj[y] : cmk(0.0, 0.0);
      }
    };
    for (int y0 = ya; y0 < yb; y0 += 4 * GB) {
      load(y0, a, b);
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        // (I, I): conj(a) a; (I, J): conj(a) b; (J, J): conj(b) b.  The
        // diagonal blocks' imaginary parts are M - M^T with M = Re^T Im, so
        // ai and ci accumulate M alone; (I, J) takes three products (Gauss:
        // P = Re Re, Q = Im Im, R = (Re a - Im a)(Re b + Im b); G = P + Q +
        // i (R - P + Q)): nine products per step, not twelve
        ar = pg_mfma(a[u].re, a[u].re, ar);
        ar = pg_mfma(a[u].im, a[u].im, ar);
        ai = pg_mfma(a[u].re, a[u].im, ai);
        br = pg_mfma(a[u].re, b[u].re, br);
        bq = pg_mfma(a[u].im, b[u].im, bq);
        bi = pg_mfma(a[u].re - a[u].im, b[u].re + b[u].im, bi);
        cr = pg_mfma(b[u].re, b[u].re, cr);
        cr = pg_mfma(b[u].im, b[u].im, cr);
        ci = pg_mfma(b[u].re, b[u].im, ci);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {          // (I, J) from P, Q, R
      const double p = br[r], q = bq[r];
      br[r] = p + q;
      bi[r] = (bi[r] - p) + q;
    }
    // the four partial Grams at the tiles' own positions (upper blocks):
    // G = (v0 + v1) + (v2 + v3), waves 1 and 3 through sG[1] and sG[0],
    // then wave 2's sum through sG[1]
    auto put = [&](cd *dst) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * r + lk, j = lr;
        dst[i * PG_N + j] = cmk(ar[r], ai[r]);
        dst[i * PG_N + 16 + j] = cmk(br[r], bi[r]);
        dst[(16 + i) * PG_N + 16 + j] = cmk(cr[r], ci[r]);
      }
    };
    auto add = [&](const cd *src) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * r + lk, j = lr;
        const cd pa = src[i * PG_N + j], pb = src[i * PG_N + 16 + j],
                 pc = src[(16 + i) * PG_N + 16 + j];
        ar[r] += pa.re;
        ai[r] += pa.im;
        br[r] += pb.re;
        bi[r] += pb.im;
        cr[r] += pc.re;
        ci[r] += pc.im;
      }
    };
    if (wave == 1) put(sG[1]);
    if (wave == 3) put(sG[0]);
    __syncthreads();
    if (wave == 0) add(sG[1]);
    if (wave == 2) add(sG[0]);
    __syncthreads();
    if (wave == 2) put(sG[1]);
    __syncthreads();
    if (wave == 0) {
      add(sG[1]);
      // M of the two diagonal blocks through sG[1] (read above by this wave
      // only): their imaginary parts are M[i][j] - M[j][i]
      double *sm = reinterpret_cast<double *>(sG[1]);      // [2][16][16]
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * r + lk, j = lr;
        sm[i * 16 + j] = ai[r];
        sm[256 + i * 16 + j] = ci[r];
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * r + lk, j = lr;
        const double vr0[3] = {ar[r], br[r], cr[r]},
                     vi0[3] = {ai[r] - sm[j * 16 + i], bi[r], ci[r] - sm[256 + j * 16 + i]};
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const double vr = vr0[t];
          double vi = vi0[t];
          const int ri = t == 2 ? 16 + i : i, cj = t == 0 ? j : 16 + j;
          if (t == 1) {
            sG[0][ri * PG_N + cj] = cmk(vr, vi);
            sG[0][cj * PG_N + ri] = cmk(vr, -vi);
          } else if (i <= j) {            // Hermitian: upper triangle, mirrored
            if (i == j) vi = 0.0;
            sG[0][ri * PG_N + cj] = cmk(vr, vi);
            sG[0][cj * PG_N + ri] = cmk(vr, -vi);
          }
        }
      }
    }
    __syncthreads();
  }
  // W = J_1 J_2 ... in registers: updating half-wave h = (thread - 64) / 32
  // holds rows h + 6 jr (jr < PG_WROWS; rows past 31 stay zero) of column
  // thread % 32
  static_assert(PG_THREADS == 256, "three updating waves hold W");
  const int ut = (int)threadIdx.x - 64;
  const int wh = ut >= 0 ? ut >> 5 : 0, wk = threadIdx.x & 31;
  cd wreg[PG_WROWS];
#pragma unroll
  for (int jr = 0; jr < PG_WROWS; ++jr) wreg[jr] = cmk(wh + 6 * jr == wk ? 1.0 : 0.0, 0.0);
  if (threadIdx.x == 0) {
    s_any = 0;
    s_touch = 0u;
  }
  const double tol = jacobi_tol(m), tiny = jacobi_floor(m, B.fro2);
  // 2. the task's rotations on G, accumulated into W.  Round rr applies the
  // coefficients in slot rr & 1; meanwhile threads 0..31 form the next
  // round's (from the entries of J^H G J they need, computed as the update
  // computes them), so that each round takes one barrier.
  const int npc = nc + (nc & 1);
  // The task's rounds pair every two real indices (round 0) or every real
  // index of I with every real index of J (the other rounds).  If no such
  // pair passes the tests on the fresh Gram, the first round rotates
  // nothing, G stays as it is, and so on: no round rotates, and the rounds
  // are skipped.
  {
    bool hit = false;
    for (int e = threadIdx.x; e < PG_N * PG_N; e += blockDim.x) {
      const int i = e >> 5, j = e & 31;
      const bool ri = i < 16 ? i < wI : i - 16 < wJ, rj = j < 16 ? j < wI : j - 16 < wJ;
      const bool inset = ri && rj && (round == 0 ? i < j : (i < 16 && j >= 16));
      if (inset && pg_active(sG[0][i * PG_N + i].re, sG[0][j * PG_N + j].re, sG[0][i * PG_N + j],
                             tol, tiny))
        hit = true;
    }
    if (hit) s_pre = 1;
    __syncthreads();
  }
  const int nrounds = !s_pre ? 0 : round == 0 ? npc - 1 : w;
  // rotation of padded index k in round rr from the current G (entries via
  // get(i, j)); writes slot sl
  auto form = [&](int rr, int sl, auto get) {
    const int k = threadIdx.x;
    bool isp;
    const int part = pg_partner(k, rr, round == 0, wI, wJ, w, isp);
    cd self = cmk(1.0, 0.0), other = cmk(0.0, 0.0);
    int pj = k;
    if (part >= 0) {
      const int p = isp ? k : part, q = isp ? part : k;
      const double al = get(p, p).re, be = get(q, q).re;
      const cd gq = get(p, q);
      if (pg_active(al, be, gq, tol, tiny)) {
        const double ga2 = gq.re * gq.re + gq.im * gq.im;
        const double rga = rsqrt(ga2);
        const double zeta = (be - al) * (0.5 * rga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = rsqrt(1.0 + t * t), sn = c * t;
        const double er = gq.re * rga, ei = -gq.im * rga;      // e = conj(g) / |g|
        if (isp) {
          self = cmk(c, 0.0);
          other = cmk(-sn * er, -sn * ei);                  // J[q][p] = -s e
        } else {
          self = cmk(c * er, c * ei);                       // J[q][q] = c e
          other = cmk(sn, 0.0);                             // J[p][q] = s
        }
        pj = part;
        s_any = 1;
      }
    }
    s_self[sl][k] = self;
    s_other[sl][k] = other;
    s_part[sl][k] = pj;
    const unsigned long long bal = __ballot(pj != k);
    if (k == 0) {
      s_rot[sl] = bal != 0ull;
      s_touch |= (unsigned)bal;
    }
  };
  if (threadIdx.x < PG_N && nrounds > 0)
    form(0, 0, [&](int i, int j) { return sG[0][i * PG_N + j]; });
  int cur = 0;
  for (int rr = 0; rr < nrounds; ++rr) {
    __syncthreads();
    const int sl = rr & 1;
    const cd *G0 = sG[cur];
    cd *G1 = sG[cur ^ 1];
    const cd *cs = s_self[sl], *co = s_other[sl];
    const int *cp = s_part[sl];
    if (threadIdx.x < PG_N && rr + 1 < nrounds)
      form(rr + 1, sl ^ 1, [&](int i, int j) {
        return i <= j ? pg_entry(G0, i, j, cs, co, cp) : cconj(pg_entry(G0, j, i, cs, co, cp));
      });
    // G' = J^H G J (upper triangle, mirrored), W' = W J: waves 1.. (wave 0
    // forms the next round's rotations meanwhile).  The upper triangle is
    // enumerated as 16 row pairs (i, 31 - i) of 33 entries each.  A round
    // without a rotation leaves G and W as they are (J = I: the update would
    // copy them exactly), and G stays in its buffer.
    const int nut = (int)blockDim.x - 64;
    const bool rot = s_rot[sl] != 0;
    if (ut >= 0 && rot) {
#pragma unroll
      for (int it = 0; it < 3; ++it) {
        const int e = ut + it * nut;
        if (e < 528) {
          const int rp = e / 33, c = e - 33 * rp;
          const int i = c < 32 - rp ? rp : 31 - rp;
          const int j = c < 32 - rp ? rp + c : i + (c - (32 - rp));
          const cd v = pg_entry(G0, i, j, cs, co, cp);
          G1[i * PG_N + j] = v;
          G1[j * PG_N + i] = cconj(v);
        }
      }
      // column wk of W: W[i][wk] self[wk] + W[i][partner] other[wk], the
      // partner's entry from the lane holding it (same half-wave, same row)
      const int pk = cp[wk];
      const cd sk = cs[wk], ok = co[wk];
      const int src = (threadIdx.x & 32) | pk;
#pragma unroll
      for (int jr = 0; jr < PG_WROWS; ++jr) {
        const cd wq = cmk(__shfl(wreg[jr].re, src), __shfl(wreg[jr].im, src));
        if (pk != wk) wreg[jr] = pg_fma(wq, ok, pg_mul(wreg[jr], sk));
      }
    }
    if (rot) cur ^= 1;
  }
  __syncthreads();
  if (s_any && threadIdx.x == 0) rf[sweep % 3] = 1;
  if (!s_any) {                // nothing rotated: the panels in memory are unchanged
    if (track && threadIdx.x == 0)
      prec[plo * PANEL_VERSION_MAX + phi] = (pv[plo] << 16) | pv[phi];
    return;
  }
  cd *sW = sG[0];              // W[i][j] at i * PG_N + j (G is no longer needed)
  if (ut >= 0) {
#pragma unroll
    for (int jr = 0; jr < PG_WROWS; ++jr)
      if (wh + 6 * jr < PG_N) sW[(wh + 6 * jr) * PG_N + wk] = wreg[jr];
  }
  __syncthreads();
  // 3. X <- X W by 16-row tiles: D[y][j] = sum_k X[y][k] W[k][j]; lane (lr,
  // lk) feeds row y0 + lr of column k0 + lk and W[k0 + lk][16 jt + lr], and
  // holds D rows 4 r + lk, column lr of each column tile jt.  A wave reads
  // every column of its rows before it writes them.  W is a product of
  // rotations of the touched indices, so an untouched column of X is left
  // as it is (not read, not multiplied, not written) and takes no part in
  // the touched ones.
  const unsigned touch = s_touch;
  cd x[PG_N / 4];
  int xoff[PG_N / 4];                    // element offset of column 4 s8 + lk, -1: none
#pragma unroll
  for (int s8 = 0; s8 < PG_N / 4; ++s8) {
    const int c = ((touch >> (4 * s8 + lk)) & 1u) ? col_of(4 * s8 + lk) : -1;
    xoff[s8] = c >= 0 ? c * m : -1;
  }
  auto load_tile = [&](int t0, cd *rx) {
    const int y = 16 * t0 + lr;
#pragma unroll
    for (int s8 = 0; s8 < PG_N / 4; ++s8)
      rx[s8] = (xoff[s8] >= 0 && y < m) ? A[(unsigned)(xoff[s8] + y)] : cmk(0.0, 0.0);
  };
  load_tile(wave, x);
  const int c0 = ((touch >> lr) & 1u) ? col_of(lr) : -1;
  const int c1 = ((touch >> (16 + lr)) & 1u) ? col_of(16 + lr) : -1;
  for (int t0 = wave; 16 * t0 < m; t0 += nwv) {
    const int y0 = 16 * t0;
    cd xn[PG_N / 4];
    load_tile(t0 + nwv, xn);             // next tile's rows, in flight meanwhile
    // one column tile at a time (its accumulators and W operands live only
    // for its own products)
#pragma unroll 1
    for (int jt = 0; jt < 2; ++jt) {
      if (((touch >> (16 * jt)) & 0xffffu) == 0u) continue;
      // three real products (Gauss): t1 = Re X Re W, t2 = Im X Im W,
      // t3 = (Re X + Im X)(Re W + Im W); D = (t1 - t2) + i (t3 - t1 - t2)
      pg_d4 t1 = {0.0, 0.0, 0.0, 0.0}, t2 = t1, t3 = t1;
#pragma unroll
      for (int s8 = 0; s8 < PG_N / 4; ++s8) {
        if (((touch >> (4 * s8)) & 0xfu) == 0u) continue;
        const cd wv = sW[(4 * s8 + lk) * PG_N + 16 * jt + lr];
        t1 = pg_mfma(x[s8].re, wv.re, t1);
        t2 = pg_mfma(x[s8].im, wv.im, t2);
        t3 = pg_mfma(x[s8].re + x[s8].im, wv.re + wv.im, t3);
      }
      const int c = jt == 0 ? c0 : c1;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int yo = y0 + 4 * r + lk;
        if (yo < m && c >= 0) A[(size_t)c * m + yo] = cmk(t1[r] - t2[r], (t3[r] - t1[r]) - t2[r]);
      }
    }
#pragma unroll
    for (int s8 = 0; s8 < PG_N / 4; ++s8) x[s8] = xn[s8];
  }
  if (versioned && threadIdx.x == 0) {
    if (hasI && (touch & 0xffffu)) ++pv[I];
    if (hasJ && (touch >> 16)) ++pv[J];
  }
}

// Big blocks by operand rows, largest first (bucketed by log2 of the rows):
// the panel launches lay their tasks out in this order, so the longest tasks
// start first and the short ones fill the launch's tail.  A block's results
// do not depend on where its tasks sit in a launch.
__global__ __launch_bounds__(1024) void k_big_order(Layer ly) {
  __shared__ int s_cnt[QR_ORDER_BUCKETS], s_off[QR_ORDER_BUCKETS];
  for (int i = threadIdx.x; i < QR_ORDER_BUCKETS; i += blockDim.x) s_cnt[i] = 0;
  __syncthreads();
  auto bucket = [&](int k) -> int {
    int g, bi;
    big_block_of(ly, k, g, bi);
    const BlkDesc &B = ly.blk[ly.gates[g].blk0 + bi];
    const int b = (int)(8.0 * log2(fmax((double)B.mj, 1.0)));
    return QR_ORDER_BUCKETS - 1 - min(b, QR_ORDER_BUCKETS - 1);
  };
  for (int k = threadIdx.x; k < ly.total_big; k += blockDim.x) atomicAdd(&s_cnt[bucket(k)], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int b = 0; b < QR_ORDER_BUCKETS; ++b) {
      s_off[b] = acc;
      acc += s_cnt[b];
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < ly.total_big; k += blockDim.x)
    ly.big_order[atomicAdd(&s_off[bucket(k)], 1)] = k;
}

// Big blocks not yet converged, compacted into the task list of the next
// panel launches: task_blk[i] = flat index of the i-th still-rotating block,
// task_pre[i] = its first task (Pp / 2 panel pairs each), task_pre[n] = all
// tasks; active[0] = blocks, active[1] = tasks.  With `last`, the simulations
// owning a block that still rotates get their error latched (sweep limit).
// A block whose simulation has a lower sweep limit and has used it up by
// launch `next_step` is retired here with its simulation's error latched.
__global__ __launch_bounds__(1024) void k_big_count(Layer ly, int last, int next_step) {
  __shared__ int s_iscan[17];
  int nb = 0, nt = 0;
  for (int b0 = 0; b0 < ly.total_big; b0 += blockDim.x) {
    const int k = b0 + threadIdx.x < ly.total_big ? ly.big_order[b0 + threadIdx.x] : -1;
    int act = 0, tasks = 0;
    if (k >= 0 && !ly.rotf[4 * (size_t)k + 3]) {
      int g, bi;
      big_block_of(ly, k, g, bi);
      const BlkDesc &B = ly.blk[ly.gates[g].blk0 + bi];
      const State &st = ly.states[ly.gates[g].inst];
      const int Pp = B.npan + (B.npan & 1);
      const int msw = min(MAX_SWEEPS, st.max_sweeps);
      if (msw < MAX_SWEEPS && next_step / (Pp > 1 ? Pp - 1 : 1) >= msw) {
        ly.rotf[4 * (size_t)k + 3] = msw;
        atomicOr(st.err, ERR_SVD_NOT_CONVERGED);
      } else {
        act = 1;
        tasks = Pp / 2;
        if (last) atomicOr(st.err, ERR_SVD_NOT_CONVERGED);
      }
    }
    int tb, tt;
    const int pb = nb + block_exclusive_scan<int>(act, s_iscan, tb);
    const int pt = nt + block_exclusive_scan<int>(tasks, s_iscan, tt);
    if (act) {
      ly.task_blk[pb] = k;
      ly.task_pre[pb] = pt;
    }
    nb += tb;
    nt += tt;
  }
  if (threadIdx.x == 0) {
    ly.task_pre[nb] = nt;
    ly.active[0] = nb;
    ly.active[1] = nt;
  }
}

__global__ __launch_bounds__(256) void k_big_finish(Layer ly, int sweeps_run) {
  int g, bi;
  big_block_of(ly, blockIdx.x, g, bi);
  const GateParam gp = ly.gates[g];
  const State st = ly.states[gp.inst];
  BlkDesc *Bp = ly.blk + gp.blk0 + bi;
  const BlkDesc B = *Bp;
  cd *A = jacobi_operand(ly, ly.base[g], B);
  extern __shared__ __attribute__((aligned(16))) double s_sig[];
  if (!B.qr && charge_n(B.q) == charge_np(B.q) && ly.tot[g].sym) self_mirror_phase(ly, gp, B, A);
  sort_values(st.err, A, B.mj, B.n, s_sig, ly.sv + gp.lst0 + B.svoff, ly.perm + gp.lst0 + B.svoff);
  if (threadIdx.x == 0) {
    const int done = ly.rotf[4 * (size_t)blockIdx.x + 3];
    Bp->sweeps = done ? done : MAX_SWEEPS;
  }
}

__global__ void k_leftvec(Layer ly, int nchunk);
__global__ void k_scatter(Layer ly);

int svd_lds_bytes() {
  // initialised once per process (thread-safe static initialisation)
  static const int bytes = [] {
    int dev = 0, v = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 65536;
    const int b = (v > 163840 ? 163840 : v) - 2048;   // room for static LDS
    hipFuncSetAttribute((const void *)k_svd_small<cd>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    hipFuncSetAttribute((const void *)k_svd_small<cf>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    hipFuncSetAttribute((const void *)k_panel<cd>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    hipFuncSetAttribute((const void *)k_panel<cf>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    hipFuncSetAttribute((const void *)k_qr, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    // k_qr_panel's sketch path has more static LDS than the 2 KB the others leave
    hipFuncSetAttribute((const void *)k_qr_panel, hipFuncAttributeMaxDynamicSharedMemorySize, b - 2048);
    hipFuncSetAttribute((const void *)k_leftvec, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    hipFuncSetAttribute((const void *)k_scatter, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    hipFuncSetAttribute((const void *)k_big_finish, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    hipFuncSetAttribute((const void *)k_contract<4>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    hipFuncSetAttribute((const void *)k_contract<8>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    hipFuncSetAttribute((const void *)k_contract<16>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    return b;
  }();
  return bytes;
}

hipError_t launch_svd_small(Layer ly, hipStream_t s) {
  if (ly.total_blocks == 0) return hipSuccess;
  const int lb = svd_lds_bytes();
  // size classes: (LDS bound, threads)
  const int cap[4] = {16384, 40960, 81920, lb};
  const int thr[4] = {256, 256, 512, 512};
  int lo = 0;
  for (int k = 0; k < 4; ++k) {
    const int hi = cap[k] < lb ? cap[k] : lb;
    if (hi <= lo) continue;
    if (ly.mixed)
      hipLaunchKernelGGL(k_svd_small<cf>, dim3(ly.total_blocks), dim3(thr[k]), (size_t)hi, s, ly,
                         lo, hi);
    else
      hipLaunchKernelGGL(k_svd_small<cd>, dim3(ly.total_blocks), dim3(thr[k]), (size_t)hi, s, ly,
                         lo, hi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    lo = hi;
  }
  return hipSuccess;
}

hipError_t launch_svd_big_prep(Layer ly, hipStream_t s) {
  if (ly.total_big == 0) return hipSuccess;
  hipLaunchKernelGGL(k_big_prep, dim3(ly.total_big), dim3(256), 0, s, ly);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_big_order, dim3(1), dim3(1024), 0, s, ly);
  return hipGetLastError();
}

// GBS_PANEL_HALF_LDS = 1: panel workgroups take half the LDS (and 512
// threads) so that two share a CU.  Over whole evolutions the narrower
// panels' extra rounds cancel what the shared CU returns, and they double
// the panels' HBM traffic, so the default keeps one panel workgroup per CU.
#ifndef GBS_PANEL_HALF_LDS
#define GBS_PANEL_HALF_LDS 0
#endif

int panel_lds_bytes(int max_chi) {
  const int lb = svd_lds_bytes();
  if (!GBS_PANEL_HALF_LDS) return lb;
  const int half = svd_panel_half(lb);
  // two columns of the longest operand must fit at panel width 1
  return 2 * (int)sizeof(cd) * max_chi <= half ? half : lb;
}

hipError_t launch_svd_panel_step(Layer ly, int step, hipStream_t s) {
  if (ly.total_big == 0) return hipSuccess;
  const int lb = svd_lds_bytes();
  // half the LDS per workgroup: two panel workgroups share a CU, one loading
  // or storing its panels while the other rotates
  const int thr = (ly.panel_lds <= lb / 2 && PANEL_THREADS > 256) ? PANEL_THREADS / 2
                                                                  : PANEL_THREADS;
  if (ly.ntask <= 0) return hipSuccess;
  if (ly.mixed)
    hipLaunchKernelGGL(k_panel<cf>, dim3(ly.ntask), dim3(thr), (size_t)ly.panel_lds, s, ly, step);
  else
    hipLaunchKernelGGL(k_panel_gram, dim3(ly.ntask), dim3(PG_THREADS), 0, s, ly, step);
  return hipGetLastError();
}

int panel_version_ints() { return PVER_STRIDE; }

int svd_max_steps(Layer ly) { return MAX_SWEEPS * (ly.maxpp > 1 ? ly.maxpp - 1 : 1) + 1; }

hipError_t launch_svd_count(Layer ly, int last, int next_step, hipStream_t s) {
  hipLaunchKernelGGL(k_big_count, dim3(1), dim3(1024), 0, s, ly, last, next_step);
  return hipGetLastError();
}

hipError_t launch_svd_big_finish(Layer ly, int sweeps_run, int max_chi, hipStream_t s) {
  if (ly.total_big == 0) return hipSuccess;
  hipLaunchKernelGGL(k_big_finish, dim3(ly.total_big), dim3(256), sizeof(double) * (size_t)max_chi,
                     s, ly, sweeps_run);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Truncation, one workgroup per gate: rank cut 1e-14 of the gate's largest
// singular value, mirror-pair units, size-weighted top-chi select, kept counts
// per block and the new bond's offsets (charge order, then decreasing value).
// ----------------------------------------------------------------------------
__device__ inline int count_above(const double *sv, int n, double cut) {
  int lo = 0, hi = n;   // sv descending: first index with sv < cut
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (sv[mid] >= cut) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(1024) void k_select(Layer ly) {
  const int g = blockIdx.x;
  const GateParam gp = ly.gates[g];
  const State st = ly.states[gp.inst];
  const int chi = st.chi;
  const int j = gp.site;
  const int nblk = ly.tot[g].nblk;
  BlkDesc *blk = ly.blk + gp.blk0;
  const double *sv = ly.sv + gp.lst0;
  unsigned long long *uv = ly.uval + gp.lst0;
  unsigned long long *uk = ly.ukey + gp.lst0;
  int *us = ly.usize + gp.lst0;
  __shared__ double s_max;
  __shared__ int s_iscan[17];
  if (threadIdx.x == 0) s_max = 0.0;
  __syncthreads();
  double mx = 0.0;
  for (int bi = threadIdx.x; bi < nblk; bi += blockDim.x)
    if (blk[bi].comp) mx = fmax(mx, sv[blk[bi].svoff]);
  atomicMax((unsigned long long *)&s_max, (unsigned long long)__double_as_longlong(mx));
  __syncthreads();
  const double cut = 1e-14 * s_max;
  for (int bi = threadIdx.x; bi < nblk; bi += blockDim.x)
    if (blk[bi].comp)
      blk[bi].len = (s_max > 0.0) ? count_above(sv + blk[bi].svoff, blk[bi].n, cut) : 0;
  __syncthreads();
  for (int bi = threadIdx.x; bi < nblk; bi += blockDim.x)   // derived blocks share the spectrum
    if (!blk[bi].comp) blk[bi].len = blk[blk[bi].mirror].len;
  __syncthreads();
  // units owned by each block
  int ub = 0;
  for (int b0 = 0; b0 < nblk; b0 += blockDim.x) {
    const int bi = b0 + threadIdx.x;
    int cnt = 0;
    if (bi < nblk) {
      const BlkDesc &B = blk[bi];
      const int q0 = charge_n(B.q), q1 = charge_np(B.q);
      if (q0 == q1) cnt = B.len;
      else if (q0 < q1) cnt = max(B.len, B.mirror >= 0 ? blk[B.mirror].len : 0);
      else cnt = (B.mirror < 0) ? B.len : 0;
    }
    int tot;
    const int pos = ub + block_exclusive_scan<int>(cnt, s_iscan, tot);
    if (bi < nblk) blk[bi].uoff = pos;
    ub += tot;
  }
  __syncthreads();
  const int U = ub;
  for (int bi = threadIdx.x; bi < nblk; bi += blockDim.x) {
    const BlkDesc B = blk[bi];
    const int q0 = charge_n(B.q), q1 = charge_np(B.q);
    const bool owner = (q0 == q1) || (q0 < q1) || (B.mirror < 0);
    if (!owner) continue;
    const bool paired = (q0 != q1) && (B.mirror >= 0);
    const int lp = paired ? blk[B.mirror].len : 0;
    const double *sp =
        paired ? sv + (blk[B.mirror].comp ? blk[B.mirror].svoff : B.svoff) : nullptr;
    const int cnt = paired ? max(B.len, lp) : B.len;
    const int canon = pack_charge(min(q0, q1), max(q0, q1));
    for (int i = 0; i < cnt; ++i) {
      double v = 0.0;
      int sz = 0;
      if (i < B.len) { v = sv[B.svoff + i]; ++sz; }
      if (i < lp) { v = fmax(v, sp[i]); ++sz; }
      uv[B.uoff + i] = (unsigned long long)__double_as_longlong(v);
      uk[B.uoff + i] = ((unsigned long long)(canon + 1) << 20) | (unsigned long long)i;
      us[B.uoff + i] = sz;
    }
  }
  __syncthreads();
  const SelectResult sr = topk_select(uv, uk, us, U, chi, st.err);
  // kept units of each owner form a prefix of its ranks
  for (int bi = threadIdx.x; bi < nblk; bi += blockDim.x) {
    const BlkDesc B = blk[bi];
    const int q0 = charge_n(B.q), q1 = charge_np(B.q);
    const bool owner = (q0 == q1) || (q0 < q1) || (B.mirror < 0);
    const int ob = owner ? bi : B.mirror;
    const BlkDesc O = blk[ob];
    const int oq0 = charge_n(O.q), oq1 = charge_np(O.q);
    const bool opaired = (oq0 != oq1) && (O.mirror >= 0);
    const int cnt = opaired ? max(O.len, blk[O.mirror].len) : O.len;
    int K = 0;
    while (K < cnt && unit_kept(sr, uv[O.uoff + K], uk[O.uoff + K])) ++K;
    blk[bi].kq = min(K, B.len);
  }
  __syncthreads();
  int nb = 0;
  for (int b0 = 0; b0 < nblk; b0 += blockDim.x) {
    const int bi = b0 + threadIdx.x;
    const int k = (bi < nblk) ? blk[bi].kq : 0;
    int tot;
    const int pos = nb + block_exclusive_scan<int>(k, s_iscan, tot);
    if (bi < nblk) blk[bi].boff = pos;
    nb += tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) st.dim[j + 1] = min(nb, chi);
}

hipError_t launch_select(Layer ly, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(ly.ngates), dim3(1024), 0, s, ly);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Singular vectors of the kept ranks of QR'd blocks.  With A P = Q R, R = X^H
// and the Jacobi result X W = Y (orthogonal columns of norms sigma), A =
// (Q W) Sigma (P Y Sigma^-1)^H: the right singular vectors are the normalised
// columns of Y put back in the original column order, v_i[piv[x]] =
// Y[x, perm[i]] / sigma_i, and u_i = A0 v_i / sigma_i
// from the pristine operand.  For a self-mirror block of a Hermitian state
// the phase of v_i is fixed first (v J-real up to a phase: bilinear sum over
// the mirrored operand columns), which makes u_i J-real too.  One wavefront
// per vector; u_i goes to the U pool (at the operand offset), conj(v_i) to
// the V pool (at the R offset), each lane owning fixed rows.
// ----------------------------------------------------------------------------
constexpr int LV_CHUNK = 8;    // kept vectors per pass over the pristine sector
constexpr int LV_XCHUNK = 256; // vector entries staged in LDS at a time

// U[:, c] = A0 v_c / sigma_c for the kept vectors of a QR'd block as a dense
// complex product on the FP64 matrix cores: v_mfma_f64_16x16x4_f64 takes a
// 16 x 4 tile of A (one double per lane: row lane % 16, k = lane / 16), a
// 4 x 16 tile of B (k = lane / 16, column lane % 16) and accumulates a 16 x 16
// tile of D (lane holds rows 4 r + lane / 16, r < 4, column lane % 16).  The
// complex product uses four real products, (Ar Br - Ai Bi) + i (Ar Bi + Ai Br),
// with two accumulator pairs (even and odd k steps) to keep the matrix pipe
// busy.  Rows of U are tiled by 16 (one tile per wavefront at a time), the kept
// vectors by 16, and the vectors are staged in LDS LVM_X entries at a time.
typedef double lv_d4 __attribute__((ext_vector_type(4)));
constexpr int LVM_X = 64;

__device__ void leftvec_mfma(const cd *A0, int m, int n, const cd *V, const double *sv, int kq,
                             cd *U, cd *sW) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ntile = (m + 15) / 16;
  for (int c0 = 0; c0 < kq; c0 += 16) {
    const int nc = min(16, kq - c0);
    for (int t0 = 0; t0 < ntile; t0 += nw) {
      const int t = t0 + wave;                  // this wave's row tile (may be past the end)
      const int yr = 16 * t + li;               // A row of this lane
      lv_d4 cr0 = {0, 0, 0, 0}, ci0 = {0, 0, 0, 0}, cr1 = {0, 0, 0, 0}, ci1 = {0, 0, 0, 0};
      for (int x0 = 0; x0 < n; x0 += LVM_X) {
        const int nx = min(LVM_X, n - x0);
        __syncthreads();
        // sW[x][c] = v_c[x0 + x] = conj of the stored (conjugated) vector
        for (int idx = threadIdx.x; idx < LVM_X * 16; idx += blockDim.x) {
          const int x = idx >> 4, c = idx & 15;
          sW[idx] = (x < nx && c < nc) ? cconj(V[(size_t)(c0 + c) * n + x0 + x]) : cmk(0.0, 0.0);
        }
        __syncthreads();
        if (t < ntile) {
          for (int k4 = 0; k4 < nx; k4 += 8) {
            // two k steps of 4 per iteration, one per accumulator pair
            const int xa = k4 + lk, xb = k4 + 4 + lk;
            const cd a = (yr < m && xa < nx) ? A0[(size_t)(x0 + xa) * m + yr] : cmk(0.0, 0.0);
            const cd b = sW[xa * 16 + li];
            const cd a2 = (yr < m && xb < nx) ? A0[(size_t)(x0 + xb) * m + yr] : cmk(0.0, 0.0);
            const cd b2 = xb < LVM_X ? sW[xb * 16 + li] : cmk(0.0, 0.0);
            cr0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.re, cr0, 0, 0, 0);
            ci0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.im, ci0, 0, 0, 0);
            cr1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.re, b2.re, cr1, 0, 0, 0);
            ci1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.re, b2.im, ci1, 0, 0, 0);
            cr0 = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.im, b.im, cr0, 0, 0, 0);
            ci0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b.re, ci0, 0, 0, 0);
            cr1 = __builtin_amdgcn_mfma_f64_16x16x4f64(-a2.im, b2.im, cr1, 0, 0, 0);
            ci1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.im, b2.re, ci1, 0, 0, 0);
          }
        }
      }
      if (t < ntile && li < nc) {
        const double s1 = 1.0 / sv[c0 + li];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int y = 16 * t + 4 * r + lk;
          if (y < m) U[(size_t)(c0 + li) * m + y] = cmk((cr0[r] + cr1[r]) * s1, (ci0[r] + ci1[r]) * s1);
        }
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_leftvec(Layer ly, int nchunk) {
  const int flat = blockIdx.x;
  const int g = find_gate_blk(ly.base, ly.ngates, flat);
  const GateBase gb = ly.base[g];
  const GateParam gp = ly.gates[g];
  const BlkDesc B = ly.blk[gp.blk0 + (flat - gb.blk)];
  if (!B.comp || !B.qr || B.kq == 0) return;
  const int m = B.m, n = B.n;
  const cd *A0 = ly.A0 + gb.e + B.eoff;
  const cd *Y = ly.R + gb.r + B.joff;
  double *sv = ly.sv + gp.lst0 + B.svoff;
  const int *perm = ly.perm + gp.lst0 + B.svoff;
  cd *U = ly.U + gb.e + B.eoff;
  cd *V = ly.V + gb.r + B.joff;
  const bool selfm = ly.tot[g].sym && charge_n(B.q) == charge_np(B.q);
  // operand columns: right-bond indices (stored Theta) or left-bond indices (Theta^T)
  const int *lst = !B.t ? ly.cols + gp.lst0 + B.coff : ly.rows + gp.lst0 + B.roff;
  const int *mx = (!B.t ? ly.mirR : ly.mirL) + gp.mir0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int *piv = ly.piv + gp.lst0 + B.svoff;
  extern __shared__ __attribute__((aligned(16))) double s_dyn[];
  cd *sV = reinterpret_cast<cd *>(s_dyn);    // LV_CHUNK right vectors, [c][x]
  __shared__ double s_red[16];
  // 1. right vectors (conjugated, original column order), one wavefront each
  for (int i0 = 0; i0 < B.kq; i0 += nw) {
    const int i = i0 + wave;
    cd f = cmk(1.0, 0.0);
    if (i < B.kq) {
      // right vector of A P is Y[:, perm[i]] / sigma; of A: v[piv[x]] = that[x]
      const cd *y = Y + (size_t)perm[i] * n;
      double s1 = 1.0 / sv[i];
      if (ly.mixed) {          // the FP32 Jacobi's norm is not exact: normalise in FP64
        double nn = 0.0;
        for (int x = lane; x < n; x += 64) nn += cabs2(y[x]);
        s1 = 1.0 / sqrt(wave_sum(nn));
      }
      cd *v = V + (size_t)i * n;
      for (int x = lane; x < n; x += 64) v[piv[x]] = cconj(cscale(y[x], s1));   // conj(v)
    }
    __syncthreads();
    if (selfm && i < B.kq) {
      // conj(v) is J-real up to a phase exactly when v is; fix it on conj(v)
      cd *v = V + (size_t)i * n;
      double sr = 0.0, si = 0.0, nr = 0.0;
      for (int x = lane; x < n; x += 64) {
        const int xm = lower_bound(lst, n, mx[lst[x]]);
        const cd p = cmul(v[x], v[xm]);
        sr += p.re;
        si += p.im;
        nr += cabs2(v[x]);
      }
      sr = wave_sum(sr);
      si = wave_sum(si);
      nr = wave_sum(nr);
      const double sa = sqrt(sr * sr + si * si);
      if (sa > 0.5 * nr && sa > 0.0) {
        const double ang = -0.5 * atan2(si, sr);
        f = cmk(cos(ang), sin(ang));
      }
    }
    __syncthreads();
    if (selfm && i < B.kq) {
      cd *v = V + (size_t)i * n;
      for (int x = lane; x < n; x += 64) v[x] = cmul(v[x], f);
    }
    __syncthreads();
  }
  if (!ly.mixed) {
    leftvec_mfma(A0, m, n, V, sv, B.kq, U, sV);
    return;
  }
  // 2. U = A0 V, LV_CHUNK vectors per pass over A0 (A0 read once per pass);
  // the vectors are staged in LDS LV_XCHUNK entries at a time, so that the
  // workgroup's LDS does not scale with the bond dimension
  for (int c0 = 0; c0 < B.kq; c0 += nchunk) {
    const int nc = min(nchunk, B.kq - c0);
    double nu[LV_CHUNK];
#pragma unroll
    for (int c = 0; c < LV_CHUNK; ++c) nu[c] = 0.0;
    for (int y0 = 0; y0 < m; y0 += blockDim.x) {
      const int y = y0 + threadIdx.x;
      const bool row = y < m;
      cd acc[LV_CHUNK];
#pragma unroll
      for (int c = 0; c < LV_CHUNK; ++c) acc[c] = cmk(0.0, 0.0);
      for (int x0 = 0; x0 < n; x0 += LV_XCHUNK) {
        const int nx = min(LV_XCHUNK, n - x0);
        __syncthreads();
        for (int idx = threadIdx.x; idx < nc * nx; idx += blockDim.x) {
          const int c = idx / nx, xl = idx % nx;
          sV[(size_t)c * LV_XCHUNK + xl] = cconj(V[(size_t)(c0 + c) * n + x0 + xl]);    // v
        }
        __syncthreads();
        if (row) {
          const cd *a0 = A0 + (size_t)x0 * m + y;
          int xl = 0;
          for (; xl + 3 < nx; xl += 4) {
            const cd a[4] = {a0[(size_t)xl * m], a0[(size_t)(xl + 1) * m],
                             a0[(size_t)(xl + 2) * m], a0[(size_t)(xl + 3) * m]};
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int c = 0; c < LV_CHUNK; ++c)
                if (c < nc) cfma(acc[c], a[u], sV[(size_t)c * LV_XCHUNK + xl + u]);
          }
          for (; xl < nx; ++xl) {
            const cd a = a0[(size_t)xl * m];
#pragma unroll
            for (int c = 0; c < LV_CHUNK; ++c)
              if (c < nc) cfma(acc[c], a, sV[(size_t)c * LV_XCHUNK + xl]);
          }
        }
      }
      if (row) {
#pragma unroll
        for (int c = 0; c < LV_CHUNK; ++c)
          if (c < nc) {
            const double s1 = ly.mixed ? 1.0 : 1.0 / sv[c0 + c];
            U[(size_t)(c0 + c) * m + y] = cscale(acc[c], s1);
            nu[c] += cabs2(acc[c]);
          }
      }
    }
    if (ly.mixed) {
      // sigma_i refined in FP64 as |A0 v_i|, u_i normalised
      __shared__ double s_lam[LV_CHUNK];
      for (int c = 0; c < nc; ++c) {
        const double t = block_sum(nu[c], s_red);
        if (threadIdx.x == 0) s_lam[c] = sqrt(t);
      }
      __syncthreads();
      for (int c = 0; c < nc; ++c) {
        const double lam = s_lam[c];
        const double r = lam > 0.0 ? 1.0 / lam : 0.0;
        for (int y = threadIdx.x; y < m; y += blockDim.x)
          U[(size_t)(c0 + c) * m + y] = cscale(U[(size_t)(c0 + c) * m + y], r);
        if (threadIdx.x == 0) sv[c0 + c] = lam;
      }
    }
    __syncthreads();
  }
}

hipError_t launch_leftvec(Layer ly, int max_chi, hipStream_t s) {
  if (ly.total_blocks == 0) return hipSuccess;
  (void)max_chi;
  hipLaunchKernelGGL(k_leftvec, dim3(ly.total_blocks), dim3(256),
                     sizeof(cd) * (size_t)LV_CHUNK * LV_XCHUNK, s, ly, LV_CHUNK);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// New tensors: zero Gamma_j, Gamma_{j+1} and the new bond, then for the kept
// ranks i of every computed block (beta = boff + i, sigma_i, operand column
// c = perm[i]):
//   u[y]   = A[y, c] / sigma_i                       (operand rows y)
//   v[x]   = sum_y A0[y, x] conj(A[y, c]) / sigma_i^2 (operand columns x)
// For a stored Theta (rows = left bond, columns = right bond):
//   Gamma_j[a, beta] = u[a] / lam_L[a],  Gamma_{j+1}[beta, b] = v[b] / lam_R[b];
// for a stored Theta^T the roles of u and v swap.  (A0 = U Sigma V^H gives
// V[:, i] = A0^H u_i / sigma_i; conj(V) is Theta's W^H row, resp. left vector.)
// With Hermiticity, the derived mirror block gets the conjugates on the mirror
// indices and a self-mirror block is made exactly J-real:
// x[y] <- (x[y] + conj(x[y~])) / 2.
// ----------------------------------------------------------------------------
__global__ void k_zero(Layer ly) {
  const int g = blockIdx.y;
  const GateParam gp = ly.gates[g];
  const State st = ly.states[gp.inst];
  const int j = gp.site;
  const size_t chi2 = (size_t)st.chi * st.chi;
  cd *G0 = st.gam + (size_t)j * chi2;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * chi2;
       i += (size_t)gridDim.x * blockDim.x)
    G0[i] = cmk(0.0, 0.0);
  if (blockIdx.x == 0) {
    const int nd = st.dim[j + 1];
    for (int i = nd + threadIdx.x; i < st.chi; i += blockDim.x) {
      st.lam[(size_t)(j + 1) * st.chi + i] = 0.0;
      st.chg[(size_t)(j + 1) * st.chi + i] = CHARGE_NONE;
    }
  }
}

__global__ __launch_bounds__(256) void k_scatter(Layer ly) {
  const int flat = blockIdx.x;
  const int g = find_gate_blk(ly.base, ly.ngates, flat);
  const GateBase gb = ly.base[g];
  const GateParam gp = ly.gates[g];
  const State st = ly.states[gp.inst];
  const BlkDesc *blk = ly.blk + gp.blk0;
  const BlkDesc B = blk[flat - gb.blk];
  if (!B.comp || B.kq == 0) return;   // derived blocks are written by their canonical block
  const int chi = st.chi;
  const int j = gp.site;
  const bool sym = ly.tot[g].sym != 0;
  const int q0 = charge_n(B.q), q1 = charge_np(B.q);
  const bool selfm = sym && q0 == q1;
  const bool mirw = sym && q0 < q1 && B.mirror >= 0;
  const int mboff = mirw ? blk[B.mirror].boff : 0;
  const int mq = pack_charge(q1, q0);
  const int m = B.m, n = B.n;
  const cd *A = ly.A + gb.e + B.eoff;
  const cd *A0 = ly.A0 + gb.e + B.eoff;
  const double *sv = ly.sv + gp.lst0 + B.svoff;
  const int *perm = ly.perm + gp.lst0 + B.svoff;
  const int *rows = ly.rows + gp.lst0 + B.roff;
  const int *cols = ly.cols + gp.lst0 + B.coff;
  const int *mL = ly.mirL + gp.mir0;
  const int *mR = ly.mirR + gp.mir0;
  // operand rows y / columns x as bond indices, their mirror maps and weights
  const int *ly_ = !B.t ? rows : cols, *lx = !B.t ? cols : rows;
  const int *my = !B.t ? mL : mR, *mx = !B.t ? mR : mL;
  const double *lamL = st.lam + (size_t)j * chi;
  const double *lamR = st.lam + (size_t)(j + 2) * chi;
  cd *G1 = st.gam + (size_t)j * chi * chi;
  cd *G2 = st.gam + (size_t)(j + 1) * chi * chi;
  extern __shared__ __attribute__((aligned(16))) double s_dyn[];
  cd *sv_x = reinterpret_cast<cd *>(s_dyn);          // v[x], n entries
  __shared__ double s_red[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = threadIdx.x; i < B.kq; i += blockDim.x) {
    st.lam[(size_t)(j + 1) * chi + B.boff + i] = sv[i];
    st.chg[(size_t)(j + 1) * chi + B.boff + i] = B.q;
    if (mirw) {
      st.lam[(size_t)(j + 1) * chi + mboff + i] = sv[i];
      st.chg[(size_t)(j + 1) * chi + mboff + i] = mq;
    }
  }
  for (int i = 0; i < B.kq; ++i) {
    // u = Ac * s1: column perm[i] of U Sigma scaled, or the QR'd block's u_i
    const double s1 = B.qr ? 1.0 : 1.0 / sv[i];
    const double s2 = s1 / sv[i];
    const cd *Ac = B.qr ? ly.U + gb.e + B.eoff + (size_t)i * m : A + (size_t)perm[i] * m;
    if (B.qr) {
      const cd *vc = ly.V + gb.r + B.joff + (size_t)i * n;
      for (int x = threadIdx.x; x < n; x += blockDim.x) sv_x[x] = vc[x];
    } else
    for (int x = wave; x < n; x += nw) {
      const cd *A0x = A0 + (size_t)x * m;
      double re = 0.0, im = 0.0;
      for (int y = lane; y < m; y += 64) {
        const cd p = cmulc(Ac[y], A0x[y]);     // A0[y, x] conj(Ac[y])
        re += p.re;
        im += p.im;
      }
      re = wave_sum(re);
      im = wave_sum(im);
      if (lane == 0) sv_x[x] = cmk(re * s2, im * s2);
    }
    __syncthreads();
    if (ly.mixed && !B.qr) {
      // the FP32 Jacobi's u is accurate to FP32 only: sigma_i refined in FP64
      // as |A0^H u_i|, v_i normalised
      double nn = 0.0;
      for (int x = threadIdx.x; x < n; x += blockDim.x) nn += cabs2(sv_x[x]);
      nn = block_sum(nn, s_red);
      const double r = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
      for (int x = threadIdx.x; x < n; x += blockDim.x) sv_x[x] = cscale(sv_x[x], r);
      if (threadIdx.x == 0) {
        const double lam = sv[i] * sqrt(nn);
        st.lam[(size_t)(j + 1) * chi + B.boff + i] = lam;
        if (mirw) st.lam[(size_t)(j + 1) * chi + mboff + i] = lam;
      }
      __syncthreads();
    }
    // operand-row side
    for (int y = threadIdx.x; y < m; y += blockDim.x) {
      cd u = cscale(Ac[y], s1);
      const int idx = ly_[y];
      if (selfm) u = cscale(cadd(u, cconj(cscale(Ac[lower_bound(ly_, m, my[idx])], s1))), 0.5);
      if (!B.t) {
        G1[(size_t)idx * chi + B.boff + i] = cscale(u, 1.0 / lamL[idx]);
        if (mirw) G1[(size_t)my[idx] * chi + mboff + i] = cscale(cconj(u), 1.0 / lamL[my[idx]]);
      } else {
        G2[(size_t)(B.boff + i) * chi + idx] = cscale(u, 1.0 / lamR[idx]);
        if (mirw) G2[(size_t)(mboff + i) * chi + my[idx]] = cscale(cconj(u), 1.0 / lamR[my[idx]]);
      }
    }
    // operand-column side
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
      cd v = sv_x[x];
      const int idx = lx[x];
      if (selfm) v = cscale(cadd(v, cconj(sv_x[lower_bound(lx, n, mx[idx])])), 0.5);
      if (!B.t) {
        G2[(size_t)(B.boff + i) * chi + idx] = cscale(v, 1.0 / lamR[idx]);
        if (mirw) G2[(size_t)(mboff + i) * chi + mx[idx]] = cscale(cconj(v), 1.0 / lamR[mx[idx]]);
      } else {
        G1[(size_t)idx * chi + B.boff + i] = cscale(v, 1.0 / lamL[idx]);
        if (mirw) G1[(size_t)mx[idx] * chi + mboff + i] = cscale(cconj(v), 1.0 / lamL[mx[idx]]);
      }
    }
    __syncthreads();
  }
}

hipError_t launch_scatter(Layer ly, int max_chi, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(64, ly.ngates), dim3(256), 0, s, ly);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ly.total_blocks == 0) return e;
  hipLaunchKernelGGL(k_scatter, dim3(ly.total_blocks), dim3(256), sizeof(cd) * (size_t)max_chi, s,
                     ly);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Operator EE of a bond: S = -sum p log2 p, p = lam^2 / sum lam^2.
// ----------------------------------------------------------------------------
__device__ inline void bond_entropy(State st, int b) {
  const int D = st.dim[b];
  const double *lam = st.lam + (size_t)b * st.chi;
  __shared__ double s_a[16], s_b[16];
  double n2 = 0.0;
  for (int i = threadIdx.x; i < D; i += blockDim.x) n2 += lam[i] * lam[i];
  n2 = wave_sum(n2);
  if ((threadIdx.x & 63) == 0) s_a[threadIdx.x >> 6] = n2;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += s_a[w];
  double h = 0.0;
  for (int i = threadIdx.x; i < D; i += blockDim.x) {
    const double p = lam[i] * lam[i] / tot;
    if (p > 0.0) h -= p * log2(p);
  }
  h = wave_sum(h);
  if ((threadIdx.x & 63) == 0) s_b[threadIdx.x >> 6] = h;
  __syncthreads();
  if (threadIdx.x == 0) {
    double S = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) S += s_b[w];
    st.ee[b] = S;
    if (!isfinite(S)) atomicOr(st.err, ERR_NONFINITE);
    else if (b >= 1 && b <= st.M - 1)
      atomicMax(st.ee_max, (unsigned long long)__double_as_longlong(fmax(S, 0.0)));
  }
}

__global__ __launch_bounds__(256) void k_entropy_layer(Layer ly) {
  const GateParam gp = ly.gates[blockIdx.x];
  bond_entropy(ly.states[gp.inst], gp.site + 1);
}

hipError_t launch_entropy_layer(Layer ly, hipStream_t s) {
  hipLaunchKernelGGL(k_entropy_layer, dim3(ly.ngates), dim3(256), 0, s, ly);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_entropy_all(State st) {
  bond_entropy(st, blockIdx.x + 1);
}

hipError_t launch_entropy_all(State st, hipStream_t s) {
  if (st.M < 2) return hipSuccess;
  hipLaunchKernelGGL(k_entropy_all, dim3(st.M - 1), dim3(256), 0, s, st);
  return hipGetLastError();
}

}  // namespace gbs
