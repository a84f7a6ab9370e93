// C ABI of the Riesz-map solver: setup (host reference build, numbering and
// patches, then device assembly and FP64 factorisation of the patch and
// coarse matrices), operator and preconditioner applies, and PCG.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/rz.h"
#include "kernels.hpp"
#include "multigrid.hpp"
#include "refelem.hpp"
#include "topology.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

struct RzError {
  int code;
  std::string msg;
};

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw RzError{e_ == hipErrorOutOfMemory ? RZ_ERR_OOM : RZ_ERR_DEVICE,              \
                    std::string(#call) + ": " + hipGetErrorString(e_)};                 \
  } while (0)

struct DevPatchSet {
  rz::PatchApply pa{};
  int64_t n_inv = 0;  // packed inverse entries
  std::vector<int64_t> sizes;  // patch sizes (for the FP32 layout)
};

}  // namespace

struct rz_problem {
  int d = 0, k = 0, p = 0;
  rz::Family fam = rz::FAM_CG;
  rz::RefElement el;
  rz::Topology top;
  std::vector<rz::PatchSet> patches;
  // the standard H(div) Hiptmair-Toselli decomposition only: per patch set
  // the coupling of its columns to the NedTwo potential functions (empty
  // sets elsewhere), their element, reference stack and weights (the
  // regularising mass 1e-8 beta of eq:local-potential-problem-added-mass)
  std::vector<rz::PatchSet> patches2;
  rz::RefElement el2;
  double *R2 = nullptr, *w2 = nullptr;
  int64_t off_I = 0;
  int max_iter = 1000;
  int precision = RZ_FP64;
  double setup_ms = 0.0;  // wall time of rz_setup
  double *scratch = nullptr;  // this device's static work array (rz_apply_A_noalloc)
  // Dirichlet boundary: input facet flags, the removed dofs (ascending), their
  // device mask (n_dofs bytes) and list; bm holds the masked right-hand sides
  // the W^k solver: exact (dense inverse) or the multigrid V-cycle
  int coarse = RZ_COARSE_EXACT;
  rz::MgDev mgdev{};
  double rho_W = 1.0;
  std::vector<uint8_t> dir_flags;
  std::vector<int32_t> dir_dofs;
  const uint8_t *dmask = nullptr;
  const int32_t *dlist = nullptr;
  double *bm = nullptr;
  // correction solves to 3e-3: an outer step cannot contract the true
  // residual by much more than ~1e-3 (the FP32 operator's error times the
  // condition number), so tighter inner solves only add iterations
  double inner_rtol = 3e-3;
  // preconditioner form; hybrid: group weights and local column ranges
  int pc = RZ_PC_ADDITIVE;
  int decomp = RZ_DECOMP_PAPER;  // rz_decomposition of the patches
  double rho_I = 1.0, rho_G = 1.0;
  int col_int = 0;            // local interior columns [col_int, n)
  int col_w0 = 0, col_w1 = 0; // local columns of the entities that carry the Whitney dofs
  // device data
  std::vector<void *> mem;
  double *R = nullptr, *Afrag = nullptr, *w = nullptr, *dinv = nullptr;
  int32_t *cell_dofs = nullptr;
  // local order of the operator apply: the Whitney dofs of the k-entities,
  // the other interface dofs, the interior dofs (apply position -> element
  // index); the apply's cell->dof map and reference fragments follow it
  std::vector<int> perm;
  int n_whitney = 0;
  int32_t *cell_dofs_apply = nullptr;
  rz::ApplyATables at{};
  std::vector<DevPatchSet> dps;
  rz::CoarseApply ca{};
  // Krylov workspace for up to ws_cols right-hand sides (grown on demand;
  // ws_gen counts reallocations, so captured graphs can tell they are stale)
  int ws_cols = 0;
  int ws_gen = 0;
  std::vector<void *> ws;
  rz::PcgState *st = nullptr;
  rz::PcgState *st_host = nullptr;
  double *r = nullptr, *z = nullptr, *pv = nullptr, *Ap = nullptr;
  double *partA = nullptr, *partR = nullptr, *partZ = nullptr, *partB = nullptr;  // block partials
  // refinement: outer state (true residual), outer residual and correction
  rz::PcgState *sto = nullptr, *sto_host = nullptr;
  double *ro = nullptr, *dx = nullptr;
  // hybrid sweep: tracked residual and group correction
  double *hs = nullptr, *hd = nullptr;
  // captured PCG iteration chunks (rz_solve), keyed by what the launches bake in
  bool graphs = true;
  hipStream_t gs = nullptr;            // stream the captured chunks run on
  hipEvent_t g_in = nullptr, g_out = nullptr;
  struct GraphEntry {
    double *x;
    int64_t ldx;
    int nc;
    unsigned lo;
    int gen;
    hipGraphExec_t exec;
    bool eager_done;  // the key's first chunk ran without capture
  };
  std::vector<GraphEntry> gcache;
  void free_graphs() {
    for (auto &g : gcache)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    gcache.clear();
  }
  rz::CoarseFold fold{};
  std::vector<rz::PatchApply> pas;  // patch sets for the launchers

  template <class T>
  T *dev(size_t count) {
    void *ptr = nullptr;
    if (count == 0) count = 1;
    HIPCHK(hipMalloc(&ptr, count * sizeof(T)));
    mem.push_back(ptr);
    return static_cast<T *>(ptr);
  }
  template <class T>
  T *upload(const std::vector<T> &v, hipStream_t s) {
    T *ptr = dev<T>(v.size());
    // blocking copy: the host vector may be a temporary of the caller
    (void)s;
    if (!v.empty()) HIPCHK(hipMemcpy(ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return ptr;
  }
  void free_ws() {
    for (void *ptr : ws) (void)hipFree(ptr);
    ws.clear();
    if (st_host) (void)hipHostFree(st_host);
    if (sto_host) (void)hipHostFree(sto_host);
    st_host = sto_host = nullptr;
    sto = nullptr;
    ro = dx = nullptr;
    hs = hd = nullptr;
    bm = nullptr;
    ws_cols = 0;
  }
  ~rz_problem() {
    free_graphs();
    if (g_in) (void)hipEventDestroy(g_in);
    if (g_out) (void)hipEventDestroy(g_out);
    if (gs) (void)hipStreamDestroy(gs);
    free_ws();
    for (void *ptr : mem) (void)hipFree(ptr);
  }
};

namespace {

int round_up(int64_t a, int b) { return int((a + b - 1) / b * b); }

void check_cells(const rz_problem &P, const double *coords) {
  const int d = P.d;
  for (int64_t c = 0; c < P.top.n_cells; ++c) {
    const int64_t *v = &P.top.cells[c * (d + 1)];
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, h = 0;
    for (int b = 0; b < d; ++b)
      for (int a = 0; a < d; ++a) J[a][b] = coords[v[b + 1] * d + a] - coords[v[0] * d + a];
    for (int i = 0; i <= d; ++i)
      for (int j = i + 1; j <= d; ++j) {
        double s = 0;
        for (int a = 0; a < d; ++a) {
          const double t = coords[v[j] * d + a] - coords[v[i] * d + a];
          s += t * t;
        }
        h = std::max(h, std::sqrt(s));
      }
    double det = d == 3 ? J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                              J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                              J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0])
                        : J[0][0] * J[1][1] - J[0][1] * J[1][0];
    if (!(std::fabs(det) > 1e-12 * std::pow(h, d)))
      throw RzError{RZ_ERR_DEGENERATE_CELL, "degenerate cell " + std::to_string(c)};
  }
}

// factor a batch of patch matrices (chunked to bound the dense workspace)
void setup_patch_set(rz_problem &P, const rz::PatchSet &ps, DevPatchSet &out, hipStream_t s,
                     const rz::PatchSet *ps2 = nullptr) {
  const int64_t B = ps.n_patches();
  const int maxsz = int(ps.max_size());
  if (maxsz > rz::kMaxPatch)
    throw RzError{RZ_ERR_UNSUPPORTED, "interface patch of " + std::to_string(maxsz) + " dofs exceeds " +
                                          std::to_string(rz::kMaxPatch)};
  const int E = 2;  // FP64 segment length
  const bool fold = maxsz > rz::kFoldMin;
  const int N = std::max(32, round_up(maxsz, 32));
  std::vector<int32_t> sizes(B);
  std::vector<int64_t> off(B);
  int64_t tot = 0;
  for (int64_t b = 0; b < B; ++b) {
    sizes[b] = int32_t(ps.patch_col[b + 1] - ps.patch_col[b]);
    off[b] = tot;
    tot += fold ? rz::fold_size(sizes[b], 8) : rz::seg_size(sizes[b], E);
  }
  double *inv = P.dev<double>(tot);
  const int64_t budget = int64_t(6) << 30;  // bytes for A + L^{-1} per chunk
  const int64_t chunk = std::max<int64_t>(1, budget / (int64_t(N) * N * 16));
  const int64_t nch = std::min(chunk, B);
  double *Abuf = nullptr, *Lbuf = nullptr;
  int32_t *dsizes = nullptr;
  int64_t *doff = nullptr;
  int *dstatus = nullptr;
  double *work = nullptr;  // split sums of the triangular inverse (chunks of nch and of the remainder)
  const int64_t nwork = std::max(rz::chol_inverse_work(nch, N), B % nch ? rz::chol_inverse_work(B % nch, N) : 0);
  HIPCHK(hipMalloc(&Abuf, size_t(nch) * N * N * 8));
  HIPCHK(hipMalloc(&Lbuf, size_t(nch) * N * N * 8));
  HIPCHK(hipMalloc(&dsizes, size_t(B) * 4));
  HIPCHK(hipMalloc(&doff, size_t(B) * 8));
  HIPCHK(hipMalloc(&dstatus, 4));
  if (nwork) HIPCHK(hipMalloc(&work, size_t(nwork) * 8));
  struct Freer {
    std::vector<void *> v;
    ~Freer() {
      for (void *p : v) (void)hipFree(p);
    }
  } fr{{Abuf, Lbuf, dsizes, doff, dstatus, work}};
  HIPCHK(hipMemcpyAsync(dsizes, sizes.data(), size_t(B) * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(doff, off.data(), size_t(B) * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(dstatus, 0, 4, s));
  // coupling triples (patch column, local dof, coefficient), needed only here
  int32_t *t_col = nullptr, *t_loc = nullptr;
  double *t_coef = nullptr;
  const size_t ntr = std::max<size_t>(1, ps.tr_col.size());
  HIPCHK(hipMalloc(&t_col, ntr * 4));
  HIPCHK(hipMalloc(&t_loc, ntr * 4));
  HIPCHK(hipMalloc(&t_coef, ntr * 8));
  fr.v.push_back(t_col);
  fr.v.push_back(t_loc);
  fr.v.push_back(t_coef);
  HIPCHK(hipMemcpyAsync(t_col, ps.tr_col.data(), ps.tr_col.size() * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(t_loc, ps.tr_loc.data(), ps.tr_loc.size() * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(t_coef, ps.tr_coef.data(), ps.tr_coef.size() * 8, hipMemcpyHostToDevice, s));
  // the second family's coupling triples (NedTwo potentials), if any
  const bool two = ps2 && ps2->n_patches() == B && B > 0;
  int32_t *t2_col = nullptr, *t2_loc = nullptr;
  double *t2_coef = nullptr;
  if (two) {
    const size_t n2 = std::max<size_t>(1, ps2->tr_col.size());
    HIPCHK(hipMalloc(&t2_col, n2 * 4));
    HIPCHK(hipMalloc(&t2_loc, n2 * 4));
    HIPCHK(hipMalloc(&t2_coef, n2 * 8));
    fr.v.push_back(t2_col);
    fr.v.push_back(t2_loc);
    fr.v.push_back(t2_coef);
    HIPCHK(hipMemcpyAsync(t2_col, ps2->tr_col.data(), ps2->tr_col.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(t2_loc, ps2->tr_loc.data(), ps2->tr_loc.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(t2_coef, ps2->tr_coef.data(), ps2->tr_coef.size() * 8, hipMemcpyHostToDevice, s));
  }
  // adds the (patch, cell) items of patches [p0, p1) of q to the chunk's matrices
  auto assemble = [&](const rz::PatchSet &q, int64_t p0, int64_t p1, const int32_t *tc, const int32_t *tl,
                      const double *tf, int n, int Q, const double *R, const double *w) {
    const int64_t i0 = q.pc_ptr[p0], i1 = q.pc_ptr[p1];
    if (i1 == i0) return;
    std::vector<int32_t> item_patch(i1 - i0), item_cell(q.pc_cell.begin() + i0, q.pc_cell.begin() + i1);
    std::vector<int64_t> item_trip(q.pc_trip.begin() + i0, q.pc_trip.begin() + i1 + 1);
    for (int64_t p = p0; p < p1; ++p)
      for (int64_t it = q.pc_ptr[p]; it < q.pc_ptr[p + 1]; ++it) item_patch[it - i0] = int32_t(p - p0);
    int32_t *d_ip = nullptr, *d_ic = nullptr;
    int64_t *d_it = nullptr;
    HIPCHK(hipMalloc(&d_ip, item_patch.size() * 4));
    HIPCHK(hipMalloc(&d_ic, item_cell.size() * 4));
    HIPCHK(hipMalloc(&d_it, item_trip.size() * 8));
    fr.v.push_back(d_ip);
    fr.v.push_back(d_ic);
    fr.v.push_back(d_it);
    HIPCHK(hipMemcpy(d_ip, item_patch.data(), item_patch.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d_ic, item_cell.data(), item_cell.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d_it, item_trip.data(), item_trip.size() * 8, hipMemcpyHostToDevice));
    rz::launch_patch_assemble(i1 - i0, d_ip, d_ic, d_it, tc, tl, tf, n, Q, R, w, N, Abuf, s);
  };
  for (int64_t p0 = 0; p0 < B; p0 += nch) {
    const int64_t p1 = std::min(B, p0 + nch), nb = p1 - p0;
    HIPCHK(hipMemsetAsync(Abuf, 0, size_t(nb) * N * N * 8, s));
    HIPCHK(hipMemsetAsync(Lbuf, 0, size_t(nb) * N * N * 8, s));
    rz::launch_pad_identity(nb, N, dsizes + p0, Abuf, s);
    assemble(ps, p0, p1, t_col, t_loc, t_coef, P.el.n, P.el.Q, P.R, P.w);
    if (two) assemble(*ps2, p0, p1, t2_col, t2_loc, t2_coef, P.el2.n, P.el2.Q, P.R2, P.w2);
    rz::launch_chol_inverse(nb, N, Abuf, Lbuf, dstatus, work, s);
    if (fold) rz::launch_pack_fold(nb, N, dsizes + p0, doff + p0, Abuf, inv, s);
    else rz::launch_pack_seg(nb, N, E, dsizes + p0, doff + p0, Abuf, inv, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
  }
  int status = 0;
  HIPCHK(hipMemcpy(&status, dstatus, 4, hipMemcpyDeviceToHost));
  if (status) throw RzError{RZ_ERR_NOT_SPD, "non-positive pivot in a patch Cholesky factorisation"};
  // work chunks: row ranges of ~equal packed-element counts
  std::vector<int64_t> chunk_patch;
  std::vector<int32_t> chunk_rows;
#ifndef RZ_CHUNK
#define RZ_CHUNK 32768
#endif
  for (int64_t b = 0; b < B && fold; ++b) {
    // folded: chunks of equal pair-row counts (2 hP entries each)
    const int m = sizes[b];
    const int h = (m + 1) / 2;
    const int rows = int(std::max<int64_t>(1, RZ_CHUNK / (2 * int64_t(rz::fold_hp(m, 8)))));
    for (int r0 = 0; r0 <= h; r0 += rows) {
      chunk_patch.push_back(b);
      chunk_rows.push_back(r0);
      chunk_rows.push_back(std::min(h + 1, r0 + rows));
    }
  }
  for (int64_t b = 0; b < B && !fold; ++b) {
    const int m = sizes[b];
    const int64_t target = RZ_CHUNK;
    int r0 = 0;
    int64_t acc = 0;
    for (int i = 0; i < m; ++i) {
      acc += (m + E - 1) / E * E - i / E * E;  // stored entries of row i
      if (acc >= target || i == m - 1) {
        chunk_patch.push_back(b);
        chunk_rows.push_back(r0);
        chunk_rows.push_back(i + 1);
        r0 = i + 1;
        acc = 0;
      }
    }
  }
  // folded sets in XCD-aware order: workgroups go to the 8 XCDs round robin
  // (block j to XCD j % 8), so block j = 8 i + x takes chunk start[x] + i of
  // XCD x's contiguous eighth of the list; the chunks of one patch then share
  // one XCD's L2 for the patch's gather and scatter maps and right-hand side
  // (measured 3-5% faster on the 625-855-dof star sets; slower on sets of
  // one or two chunks per patch, which keep the patch order)
  const int64_t nck = int64_t(chunk_patch.size());
  if (fold && nck > 8) {
    const int64_t q = nck / 8, rem = nck % 8;
    std::vector<int64_t> cp(nck);
    std::vector<int32_t> cr(2 * nck);
    for (int64_t j = 0; j < nck; ++j) {
      const int64_t x = j % 8, i = j / 8;
      const int64_t src = x * q + std::min<int64_t>(x, rem) + i;  // i < q + (x < rem)
      cp[j] = chunk_patch[src];
      cr[2 * j] = chunk_rows[2 * src];
      cr[2 * j + 1] = chunk_rows[2 * src + 1];
    }
    chunk_patch.swap(cp);
    chunk_rows.swap(cr);
  }
  if (!fold) {
    // the set's dofs with their (patch column, coefficient) entries, patch
    // columns ascending: the fixed-order scatter of the multi-column solves
    const int64_t SM = ps.patch_col[B], nE = ps.col_ent[SM], nd = P.top.n_dofs;
    std::vector<int64_t> start(nd + 1, 0);
    for (int64_t e = 0; e < nE; ++e) ++start[ps.ent_dof[e] + 1];
    for (int64_t d = 0; d < nd; ++d) start[d + 1] += start[d];
    std::vector<int64_t> pos(start.begin(), start.end() - 1);
    std::vector<int32_t> apr(nE);
    std::vector<double> acoef(nE);
    for (int64_t pr = 0; pr < SM; ++pr)
      for (int64_t e = ps.col_ent[pr]; e < ps.col_ent[pr + 1]; ++e) {
        const int64_t k = pos[ps.ent_dof[e]]++;
        apr[k] = int32_t(pr);
        acoef[k] = ps.ent_coef[e];
      }
    std::vector<int32_t> adof;
    std::vector<int64_t> aptr{0};
    for (int64_t d = 0; d < nd; ++d)
      if (start[d + 1] > start[d]) {
        adof.push_back(int32_t(d));
        aptr.push_back(start[d + 1]);
      }
    std::vector<int32_t> where(nd, -1), ent_a(nE);
    for (size_t a = 0; a < adof.size(); ++a) where[adof[a]] = int32_t(a);
    for (int64_t e = 0; e < nE; ++e) ent_a[e] = where[ps.ent_dof[e]];
    out.pa.ent_a = P.upload(ent_a, s);
    out.pa.sum_size = SM;
    out.pa.n_adof = int64_t(adof.size());
    out.pa.adof = P.upload(adof, s);
    out.pa.aptr = P.upload(aptr, s);
    out.pa.apr = P.upload(apr, s);
    out.pa.acoef = P.upload(acoef, s);
  }
  out.pa.n_patches = B;
  out.pa.n_chunks = nck;
  out.pa.chunk_patch = P.upload(chunk_patch, s);
  out.pa.chunk_rows = P.upload(chunk_rows, s);
  out.pa.max_size = maxsz;
  out.pa.fold = fold ? 1 : 0;
  out.pa.n_entries = tot;
  out.pa.patch_col = P.upload(ps.patch_col, s);
  out.pa.col_ent = P.upload(ps.col_ent, s);
  out.pa.inv_off = P.upload(off, s);
  out.pa.ent_dof = P.upload(ps.ent_dof, s);
  out.pa.ent_coef = P.upload(ps.ent_coef, s);
  out.pa.inv = inv;
  out.n_inv = tot;
  out.sizes.assign(sizes.begin(), sizes.end());
}

void setup_coarse(rz_problem &P, hipStream_t s) {
  std::vector<int32_t> wdofs, wloc, widx;
  int nwl = 0;
  rz::whitney_dofs(P.top, P.el, wdofs, wloc, widx, nwl);
  const int nW = int(wdofs.size());
  const int N = std::max(64, round_up(nW, 64));
  const int NT = N / 64;
  // one "patch" whose items are the cells, coupling their local Whitney dofs
  const int64_t nc = P.top.n_cells;
  std::vector<int32_t> item_patch(nc, 0), item_cell(nc), tr_col, tr_loc;
  std::vector<int64_t> item_trip(nc + 1, 0);
  std::vector<double> tr_coef;
  // removed (Dirichlet) Whitney dofs keep their coarse index but are
  // decoupled: no cell couples them and their diagonal is one
  std::vector<uint8_t> wrem(nW, 0);
  std::vector<int32_t> wrem_idx;
  if (!P.dir_dofs.empty())
    for (int i = 0; i < nW; ++i)
      if (std::binary_search(P.dir_dofs.begin(), P.dir_dofs.end(), wdofs[i])) wrem[i] = 1, wrem_idx.push_back(i);
  for (int64_t c = 0; c < nc; ++c) {
    item_cell[c] = int32_t(c);
    for (int a = 0; a < nwl; ++a) {
      if (wrem[widx[c * nwl + a]]) continue;
      tr_col.push_back(widx[c * nwl + a]);
      tr_loc.push_back(wloc[a]);
      tr_coef.push_back(1.0);
    }
    item_trip[c + 1] = int64_t(tr_col.size());
  }
  double *Abuf = nullptr, *Lbuf = nullptr;
  int *dstatus = nullptr;
  int32_t *dsz = nullptr;
  HIPCHK(hipMalloc(&Abuf, size_t(N) * N * 8));
  HIPCHK(hipMalloc(&Lbuf, size_t(N) * N * 8));
  HIPCHK(hipMalloc(&dstatus, 4));
  HIPCHK(hipMalloc(&dsz, 4));
  double *work = nullptr;  // split sums of the triangular inverse
  if (const int64_t nwork = rz::chol_inverse_work(1, N)) HIPCHK(hipMalloc(&work, size_t(nwork) * 8));
  std::vector<void *> tmp{Abuf, Lbuf, dstatus, dsz, work};
  struct Freer {
    std::vector<void *> &v;
    ~Freer() {
      for (void *p : v) (void)hipFree(p);
    }
  } fr{tmp};
  auto up = [&](auto &v) {
    using T = typename std::decay_t<decltype(v)>::value_type;
    T *ptr = nullptr;
    HIPCHK(hipMalloc(&ptr, std::max<size_t>(1, v.size()) * sizeof(T)));
    tmp.push_back(ptr);
    HIPCHK(hipMemcpy(ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return ptr;
  };
  int32_t *d_ip = up(item_patch), *d_ic = up(item_cell), *d_col = up(tr_col), *d_loc = up(tr_loc);
  int64_t *d_it = up(item_trip);
  double *d_coef = up(tr_coef);
  HIPCHK(hipMemsetAsync(Abuf, 0, size_t(N) * N * 8, s));
  HIPCHK(hipMemsetAsync(Lbuf, 0, size_t(N) * N * 8, s));
  HIPCHK(hipMemsetAsync(dstatus, 0, 4, s));
  HIPCHK(hipMemcpy(dsz, &nW, 4, hipMemcpyHostToDevice));
  rz::launch_pad_identity(1, N, dsz, Abuf, s);
  rz::launch_patch_assemble(nc, d_ip, d_ic, d_it, d_col, d_loc, d_coef, P.el.n, P.el.Q, P.R, P.w, N, Abuf, s);
  if (!wrem_idx.empty()) rz::launch_set_diag(N, up(wrem_idx), int(wrem_idx.size()), Abuf, s);
  rz::launch_chol_inverse(1, N, Abuf, Lbuf, dstatus, work, s);
  double *tiles = P.dev<double>(size_t(NT) * (NT + 1) / 2 * 4096);
  rz::launch_pack_tiles(N, nW, Abuf, tiles, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  int status = 0;
  HIPCHK(hipMemcpy(&status, dstatus, 4, hipMemcpyDeviceToHost));
  if (status) throw RzError{RZ_ERR_NOT_SPD, "non-positive pivot in the coarse Cholesky factorisation"};
  P.ca.nW = nW;
  P.ca.NT = NT;
  P.ca.wdofs = P.upload(wdofs, s);
  P.ca.tiles = tiles;
  P.ca.mg = nullptr;
  P.ca.wscale = 1.0;
}

// The geometric multigrid V-cycle on W^k over the caller's mesh hierarchy
// (in place of the dense coarse inverse): host set-up of the levels, then
// upload.  The Whitney block A[W, W] is assembled on the host from the
// element's Whitney sub-blocks and the geometric weights.
void setup_multigrid(rz_problem &P, const rz_mesh *m, const rz_options *o, hipStream_t s) {
  if (P.fam == rz::FAM_NEDTWO || P.fam == rz::FAM_BDM)
    throw RzError{RZ_ERR_UNSUPPORTED, "the multigrid coarse solver is built for the first-kind spaces"};
  if (!P.dir_dofs.empty())
    throw RzError{RZ_ERR_UNSUPPORTED, "the multigrid coarse solver is built for pure Neumann problems"};
  if (o->mg_levels < 2 || !o->mg_meshes) throw RzError{RZ_ERR_ARG, "multigrid needs mg_levels >= 2 meshes"};
  const int d = P.d;
  const rz_mesh *H = o->mg_meshes;
  for (int l = 0; l < o->mg_levels; ++l)
    if (H[l].dim != d || !H[l].coords || !H[l].cells || H[l].n_vertices <= 0 || H[l].n_cells <= 0)
      throw RzError{RZ_ERR_ARG, "bad mesh in the multigrid hierarchy"};
  if (H[0].n_vertices != m->n_vertices || H[0].n_cells != m->n_cells ||
      std::memcmp(H[0].cells, m->cells, sizeof(int64_t) * (d + 1) * m->n_cells) != 0)
    throw RzError{RZ_ERR_MESH, "the finest hierarchy mesh must have the problem's vertices and cells"};
  // the form degree of the Whitney space: 2D RT_p is k = 1 (the quarter
  // turn of Ned_p: the H(curl) prolongation and smoother serve it unchanged)
  const int k = P.k;
  // level topologies (entity lists of the lowest-order element)
  rz::RefElement el1 = rz::build_reference(d, P.fam, 1);
  std::vector<rz::Topology> coarse_tops;
  coarse_tops.reserve(o->mg_levels);
  std::vector<const rz::Topology *> tops{&P.top};
  std::vector<const double *> X{H[0].coords};
  for (int l = 1; l < o->mg_levels; ++l) {
    coarse_tops.push_back(rz::build_topology(d, H[l].n_vertices, H[l].n_cells, H[l].cells, el1));
    tops.push_back(&coarse_tops.back());
    X.push_back(H[l].coords);
  }
  // A[W, W] from the Whitney sub-blocks of the cell matrices
  std::vector<int32_t> wdofs, wloc, widx;
  int nwl = 0;
  rz::whitney_dofs(P.top, P.el, wdofs, wloc, widx, nwl);
  const int nW = int(wdofs.size());
  const int64_t nc = P.top.n_cells;
  const int Q = P.el.Q, n = P.el.n;
  std::vector<double> w(size_t(nc) * Q);
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(w.data(), P.w, w.size() * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<int64_t> tr;
  std::vector<int32_t> tc;
  std::vector<double> tv;
  for (int64_t c = 0; c < nc; ++c)
    for (int a = 0; a < nwl; ++a)
      for (int b = 0; b < nwl; ++b) {
        double v = 0.0;
        for (int q = 0; q < Q; ++q) v += w[c * Q + q] * P.el.R[(size_t(q) * n + wloc[a]) * n + wloc[b]];
        tr.push_back(widx[c * nwl + a]);
        tc.push_back(widx[c * nwl + b]);
        tv.push_back(v);
      }
  const rz::Csr AW = rz::csr_from_triplets(nW, nW, tr, tc, tv);
  rz::MgHierarchy Hm;
  try {
    Hm = rz::build_multigrid(k, AW, tops, X, 2);
  } catch (const std::invalid_argument &e) {
    throw RzError{RZ_ERR_MESH, e.what()};
  }
  if (int(Hm.lev.size()) > 12) throw RzError{RZ_ERR_UNSUPPORTED, "at most 12 multigrid levels"};
  rz::MgDev &D = P.mgdev;
  D.k = k;
  D.nu = Hm.nu;
  D.L = int(Hm.lev.size());
  for (int l = 0; l < D.L; ++l) {
    const rz::MgLevel &lv = Hm.lev[l];
    rz::MgDevLevel &dl = D.lev[l];
    dl.n = lv.A.n_rows;
    dl.Ap = P.upload(lv.A.ptr, s), dl.Ac = P.upload(lv.A.col, s), dl.Av = P.upload(lv.A.val, s);
    if (l + 1 == D.L) break;
    dl.Pp = P.upload(lv.P.ptr, s), dl.Pc = P.upload(lv.P.col, s), dl.Pv = P.upload(lv.P.val, s);
    dl.Rp = P.upload(lv.R.ptr, s), dl.Rc = P.upload(lv.R.col, s), dl.Rv = P.upload(lv.R.val, s);
    dl.omega = lv.omega;
    if (!lv.dinv.empty()) dl.dinv = P.upload(lv.dinv, s);
    if (k == 1) {
      dl.nv = lv.Gt.n_rows;
      dl.Gp = P.upload(lv.G.ptr, s), dl.Gc = P.upload(lv.G.col, s), dl.Gv = P.upload(lv.G.val, s);
      dl.Gtp = P.upload(lv.Gt.ptr, s), dl.Gtc = P.upload(lv.Gt.col, s), dl.Gtv = P.upload(lv.Gt.val, s);
      dl.gdiag = P.upload(lv.gdiag, s);
    }
    if (k == 2) {
      for (size_t e = 0; e + 1 < lv.star_ptr.size(); ++e)
        if (lv.star_ptr[e + 1] - lv.star_ptr[e] > 8)
          throw RzError{RZ_ERR_UNSUPPORTED, "multigrid: an edge with more than 8 faces"};
      dl.nstar = int64_t(lv.star_ptr.size()) - 1;
      dl.sp = P.upload(lv.star_ptr, s), dl.sf = P.upload(lv.star_face, s), dl.so = P.upload(lv.inv_off, s);
      dl.sinv = P.upload(lv.inv, s);
    }
  }
  D.cinv = P.upload(Hm.coarse_inv, s);
  P.ca.nW = nW;
  P.ca.NT = std::max(1, (nW + 63) / 64);
  P.ca.wdofs = P.upload(wdofs, s);
  P.ca.tiles = nullptr;
  P.ca.mg = &P.mgdev;
  P.ca.wscale = 1.0;
  P.coarse = RZ_COARSE_MG;
  if (P.pc == RZ_PC_HYBRID) {
    // the V-cycle is an inexact solver: its own weight, as for the other groups
    P.rho_W = rz::lanczos_weight(
        nW, [&](const double *x, double *y) { rz::csr_apply(AW, x, y); },
        [&](const double *r, double *z) { rz::mg_cycle_host(Hm, r, z); }, 0x5EED4000ull);
    P.ca.wscale = 1.0 / P.rho_W;
  }
}

void do_setup(rz_problem &P, const rz_mesh *m, hipStream_t s) {
  // numbering, patches
  P.top = rz::build_topology(P.d, m->n_vertices, m->n_cells, m->cells, P.el);
  check_cells(P, m->coords);
  const bool hdiv_ht = P.d == 3 && (P.fam == rz::FAM_RT || P.fam == rz::FAM_BDM) &&
                       (P.decomp == RZ_DECOMP_HIPTMAIR || P.decomp == RZ_DECOMP_HIPTMAIR_FULL);
  if (hdiv_ht) {
    // the potentials are NedTwo functions: NedTwo_p for RT_p, NedTwo_{p+1} for BDM_p
    P.el2 = rz::build_reference(3, rz::FAM_NEDTWO, P.p + (P.fam == rz::FAM_BDM ? 1 : 0));
    const rz::Topology t2 = rz::build_topology(3, m->n_vertices, m->n_cells, m->cells, P.el2);
    P.patches = rz::build_hdiv_hiptmair(P.top, P.el, t2, P.el2, P.decomp == RZ_DECOMP_HIPTMAIR_FULL, P.patches2);
  } else {
    P.patches = rz::build_patches(P.top, P.el, rz::Decomposition(P.decomp));
  }
  if (!P.dir_flags.empty()) {
    // X^k_{p,D} (Sec. 5): remove the functions tied to subsimplices of Gamma_D
    P.dir_dofs = rz::dirichlet_dofs(P.top, P.el, m->cells, P.dir_flags.data());
    std::vector<uint8_t> removed(P.top.n_dofs, 0);
    for (int32_t g : P.dir_dofs) removed[g] = 1;
    for (auto &ps : P.patches) rz::restrict_patches(ps, removed);
    P.dmask = P.upload(removed, s);
    P.dlist = P.upload(P.dir_dofs, s);
  }
  // first dof of the Jacobi group: the interior dofs, or none when the full
  // vertex stars (eq:pafw) hold them
  P.off_I = rz::decomposition_full(P.decomp) ? P.top.n_dofs : P.top.offset[P.d];
  const int n = P.el.n, Q = P.el.Q, d = P.d;
  // the apply's local order: Whitney dofs of the k-entities first, so the
  // hybrid's coarse correction (nonzero only there) is applied with a
  // column range of one or two k-blocks; interior dofs stay last
  P.perm.clear();
  for (int i = 0; i < n; ++i)
    if (P.el.dofs[i].entity_dim == P.el.k && P.el.dofs[i].kind == rz::KIND_W) P.perm.push_back(i);
  P.n_whitney = int(P.perm.size());
  for (int i = 0; i < n; ++i)
    if (P.el.dofs[i].entity_dim != d && !(P.el.dofs[i].entity_dim == P.el.k && P.el.dofs[i].kind == rz::KIND_W))
      P.perm.push_back(i);
  for (int i = 0; i < n; ++i)
    if (P.el.dofs[i].entity_dim == d) P.perm.push_back(i);
  // reference tables: plain (element order) and in MFMA fragment order (apply order)
  P.R = P.upload(P.el.R, s);
  const int NP = round_up(n, 16), KP = round_up(n, 4), KB = KP / 4, NMB = NP / 16;
  std::vector<double> frag(size_t(NMB) * Q * KB * 64, 0.0);
  for (int mb = 0; mb < NMB; ++mb)
    for (int q = 0; q < Q; ++q)
      for (int kb = 0; kb < KB; ++kb)
        for (int lane = 0; lane < 64; ++lane) {
          const int row = mb * 16 + (lane & 15), col = kb * 4 + (lane >> 4);
          if (row < n && col < n)
            frag[((size_t(mb) * KB + kb) * Q + q) * 64 + lane] =
                P.el.R[(size_t(q) * n + P.perm[row]) * n + P.perm[col]];
        }
  P.Afrag = P.upload(frag, s);
  P.cell_dofs = P.upload(P.top.cell_dofs, s);
  std::vector<int32_t> cda(P.top.cell_dofs.size());
  for (int64_t c = 0; c < int64_t(P.top.n_cells); ++c)
    for (int j = 0; j < n; ++j) cda[c * n + j] = P.top.cell_dofs[c * n + P.perm[j]];
  P.cell_dofs_apply = P.upload(cda, s);
  P.w = P.dev<double>(size_t(P.top.n_cells) * Q);
}

}  // namespace

static void ensure_ws(rz_problem *P, int ncol);
static void estimate_weights(rz_problem *P, hipStream_t s);

// Work space of rz_apply_A_noalloc: the operator's cell-local vectors (Xc,
// Yc) in a static device array instead of the handle's workspace, so that
// call allocates nothing.  Each GPU the library runs on holds its own copy
// for the life of the process.  In host code the array's name is not a
// device address: kernels receive the address hipGetSymbolAddress returns,
// looked up once per device during rz_setup with that device current.
namespace {
constexpr size_t kScratchBytes = size_t(128) << 20;
__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;  // device -> address of its scratch

double *scratch_address() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  double *ptr = nullptr;
  HIPCHK(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
  g_scratch_ptr[dev] = ptr;
  return ptr;
}
}  // namespace

// rz_decomposition values and the spaces they are built for
// the family of a space constant (second kind: NedTwo_p, BDM_p)
static rz::Family family_of(int space) {
  switch (space) {
    case RZ_HGRAD: return rz::FAM_CG;
    case RZ_HCURL: return rz::FAM_NED;
    case RZ_HDIV: return rz::FAM_RT;
    case RZ_HCURL2: return rz::FAM_NEDTWO;
    default: return rz::FAM_BDM;
  }
}

static int check_decomposition(int32_t dec, int space, int dim) {
  if (dec < RZ_DECOMP_PAPER || dec > RZ_DECOMP_TYPEI_FULL) return fail(RZ_ERR_ARG, "unknown decomposition");
  // 2D H(div) is the quarter turn of 2D H(curl) and shares its decompositions
  if ((dec == RZ_DECOMP_HIPTMAIR || dec == RZ_DECOMP_HIPTMAIR_FULL) && space == RZ_HGRAD)
    return fail(RZ_ERR_UNSUPPORTED, "the Hiptmair-Toselli decompositions need H(curl) or H(div)");
  if ((dec == RZ_DECOMP_TYPEI || dec == RZ_DECOMP_TYPEI_FULL) && space == RZ_HGRAD)
    return fail(RZ_ERR_UNSUPPORTED, "the type-I Hiptmair-Toselli decompositions need H(curl) or H(div)");
  return RZ_OK;
}

extern "C" {

const char *rz_last_error(void) { return g_err.c_str(); }

int rz_setup(const rz_mesh *m, int32_t degree, rz_space space, const rz_options *opts, void *hip_stream,
             rz_problem **out) {
  if (!m || !out || !m->coords || !m->cells) return fail(RZ_ERR_ARG, "null argument");
  *out = nullptr;
  if (m->dim != 2 && m->dim != 3) return fail(RZ_ERR_ARG, "dim must be 2 or 3");
  if (m->n_vertices <= 0 || m->n_cells <= 0) return fail(RZ_ERR_ARG, "empty mesh");
  const double alpha = opts ? opts->alpha : 1.0, beta = opts ? opts->beta : 1.0;
  if (!(alpha >= 0.0) || !(beta > 0.0)) return fail(RZ_ERR_ARG, "need alpha >= 0 and beta > 0");
  if (degree < 1 || degree > 10) return fail(RZ_ERR_UNSUPPORTED, "degree must be in 1..10");
  if (space < RZ_HGRAD || space > RZ_HDIV2) return fail(RZ_ERR_ARG, "unknown space");
  if (m->dim == 2 && space > RZ_HDIV)
    return fail(RZ_ERR_UNSUPPORTED, "the second-kind spaces are built for tetrahedral meshes");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const auto t_setup = std::chrono::steady_clock::now();
  auto P = std::make_unique<rz_problem>();
  P->d = m->dim;
  P->p = degree;
  if (opts && opts->max_iter > 0) P->max_iter = std::min<int>(opts->max_iter, rz::kMaxIter);
  if (opts) {
    if (opts->precision < RZ_FP64 || opts->precision > RZ_BF16_PC) return fail(RZ_ERR_ARG, "unknown precision");
    if (!(opts->inner_rtol < 1.0)) return fail(RZ_ERR_ARG, "inner_rtol must be below 1");
    P->precision = opts->precision;
    if (opts->inner_rtol > 0.0) P->inner_rtol = opts->inner_rtol;
    if (opts->pc != RZ_PC_ADDITIVE && opts->pc != RZ_PC_HYBRID) return fail(RZ_ERR_ARG, "unknown preconditioner");
    P->pc = opts->pc;
    P->graphs = opts->eager == 0;
    if (int e = check_decomposition(opts->decomposition, space, m->dim)) return e;
    P->decomp = opts->decomposition;
    if (opts->dirichlet_facet) {
      if ((opts->decomposition == RZ_DECOMP_HIPTMAIR || opts->decomposition == RZ_DECOMP_HIPTMAIR_FULL) &&
          m->dim == 3 && (space == RZ_HDIV || space == RZ_HDIV2))
        return fail(RZ_ERR_UNSUPPORTED, "the H(div) Hiptmair-Toselli potentials are built for pure Neumann problems");
      P->dir_flags.assign(opts->dirichlet_facet, opts->dirichlet_facet + m->n_cells * (m->dim + 1));
    }
    if (opts->coarse != RZ_COARSE_EXACT && opts->coarse != RZ_COARSE_MG)
      return fail(RZ_ERR_ARG, "unknown coarse solver");
  }
  P->fam = family_of(space);
  try {
    P->el = rz::build_reference(P->d, P->fam, degree);
    P->k = P->el.k;
    do_setup(*P, m, s);
    const int d = P->d, n = P->el.n, Q = P->el.Q;
    const int64_t nc = P->top.n_cells;
    // weights (recomputed here so the coordinates buffer is at hand)
    {
      std::vector<double> X(size_t(nc) * (d + 1) * d);
      for (int64_t c = 0; c < nc; ++c)
        for (int a = 0; a <= d; ++a)
          for (int b = 0; b < d; ++b)
            X[(c * (d + 1) + a) * d + b] = m->coords[P->top.cells[c * (d + 1) + a] * d + b];
      std::vector<double> V(size_t(d + 1) * d);
      rz::eq_vertices(d, V.data());
      rz::Dense E(d, d);
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) E(a, b) = V[(b + 1) * d + a] - V[a];
      rz::Dense Ei = rz::inverse(E);
      double *dX = P->upload(X, s);
      double *dEi = P->upload(Ei.a, s);
      const int pullback = P->k == 0 ? 0 : ((P->el.fam == rz::FAM_RT || P->el.fam == rz::FAM_BDM) ? 2 : 1);
      rz::launch_weights(d, pullback, nc, dX, dEi, alpha, beta, P->w, Q, s);
      if (!P->patches2.empty()) {
        // the NedTwo mass 1e-8 beta (covariant pullback, no curl term)
        P->w2 = P->dev<double>(size_t(nc) * P->el2.Q);
        rz::launch_weights(d, 1, nc, dX, dEi, 0.0, 1e-8 * beta, P->w2, P->el2.Q, s);
        P->R2 = P->upload(P->el2.R, s);
      }
    }
    // interior diagonal (Jacobi on X^k_I; an empty group under the full
    // vertex stars)
    const bool full_stars = rz::decomposition_full(P->decomp);
    std::vector<int32_t> loc_int;
    for (int i = 0; i < n; ++i)
      if (P->el.dofs[i].entity_dim == d) loc_int.push_back(i);
    P->dinv = P->dev<double>(std::max<int64_t>(1, P->top.n_interior));
    if (!full_stars) {
      int32_t *dloc = P->upload(loc_int, s);
      rz::launch_interior_diag(nc, n, Q, P->R, P->w, P->cell_dofs, dloc, int(loc_int.size()), P->off_I, P->dinv,
                               s);
    }
    HIPCHK(hipGetLastError());
    // apply_A tables
    P->at.n = n;
    P->at.Q = Q;
    P->at.NP = round_up(n, 16);
    P->at.KP = round_up(n, 4);
    P->at.Afrag = P->Afrag;
    P->at.w = P->w;
    P->at.cell_dofs = P->cell_dofs_apply;
    P->at.n_cells = nc;
    P->at.dmask = P->dmask;
    P->ca.dmask = P->dmask;
    // assembly lists of the three-stage apply: for every dof, the positions
    // of its (cell, local row) results in Yc, cells ascending
    {
      const int64_t ncp = (nc + 255) / 256 * 256;  // whole blocks of 4 waves x 64 cells
      const int64_t nd = P->top.n_dofs;
      if (int64_t(P->at.NP) * ncp >= (int64_t(1) << 31))
        throw RzError{RZ_ERR_UNSUPPORTED, "mesh too large for 32-bit cell-local indices"};
      // (cell, row r of the apply order) holds dof cell_dofs[cell][perm[r]]
      const std::vector<int> &pm = P->perm;
      std::vector<int64_t> ptr(nd + 1, 0);
      for (int64_t e = 0; e < nc * n; ++e) ++ptr[P->top.cell_dofs[e] + 1];
      for (int64_t i = 0; i < nd; ++i) ptr[i + 1] += ptr[i];
      std::vector<int32_t> ent(size_t(nc) * n);
      std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
      for (int64_t c = 0; c < nc; ++c)
        for (int r = 0; r < n; ++r) ent[fill[P->top.cell_dofs[c * n + pm[r]]]++] = int32_t(rz::yc_index(ncp, c, r));
      P->at.ncp = ncp;
      P->at.n_dofs = nd;
      P->at.asm_ptr = P->upload(ptr, s);
      P->at.asm_ent = P->upload(ent, s);
    }
    // interface patches and coarse space
    P->dps.resize(P->patches.size());
    for (size_t i = 0; i < P->patches.size(); ++i)
      setup_patch_set(*P, P->patches[i], P->dps[i], s, P->patches2.empty() ? nullptr : &P->patches2[i]);
    if (opts && opts->coarse == RZ_COARSE_MG)
      setup_multigrid(*P, m, opts, s);
    else
      setup_coarse(*P, s);
    if (P->precision != RZ_FP64) {
      // FP32 copies: the inverses (both modes) and the operator tables (refinement)
      auto lo = [&](const double *a, int64_t count) {
        float *b = P->dev<float>(size_t(count));
        rz::launch_to_float(count, a, b, s);
        return static_cast<const float *>(b);
      };
      if (P->precision == RZ_FP32_IR || P->precision == RZ_BF16_PC) {
        P->at.Afrag32 = lo(P->Afrag, int64_t(P->at.NP) * P->at.KP * Q);
        P->at.w32 = lo(P->w, nc * Q);
      }
      const bool bf16 = P->precision == RZ_BF16_PC;
      const int VL = bf16 ? 8 : 4;
      for (auto &d : P->dps) {
        std::vector<int64_t> offl(d.sizes.size());
        int64_t totl = 0;
        for (size_t b = 0; b < d.sizes.size(); ++b) {
          offl[b] = totl;
          totl += d.pa.fold ? rz::fold_size(int(d.sizes[b]), bf16 ? 2 : 4) : rz::seg_size(int(d.sizes[b]), VL);
        }
        const int64_t *doff = P->upload(offl, s);
        if (bf16) {
          uint16_t *inv16 = P->dev<uint16_t>(size_t(totl));
          rz::launch_seg_to_bf16(d.pa.n_patches, d.pa.patch_col, d.pa.inv_off, doff, d.pa.inv, inv16, d.pa.fold, s);
          d.pa.inv16 = inv16;
          d.pa.inv_off16 = doff;
        } else {
          float *inv32 = P->dev<float>(size_t(totl));
          rz::launch_seg_to_float(d.pa.n_patches, d.pa.patch_col, d.pa.inv_off, doff, d.pa.inv, inv32, d.pa.fold, s);
          d.pa.inv32 = inv32;
          d.pa.inv_off32 = doff;
        }
      }
      // the coarse inverse stays FP32 under RZ_BF16_PC: its condition grows
      // like h^-2, and a bfloat16 copy loses definiteness on modest meshes
      // (the patch matrices are local and stay well conditioned)
      if (P->ca.tiles) P->ca.tiles32 = lo(P->ca.tiles, int64_t(P->ca.NT) * (P->ca.NT + 1) / 2 * 4096);
      HIPCHK(hipGetLastError());
    }
    for (auto &d : P->dps) P->pas.push_back(d.pa);
    P->fold.off = P->top.offset[P->k];
    P->fold.N = P->el.per_entity[P->k];
    P->fold.span = P->top.n_ent[P->k] * P->fold.N;
    // local column ranges (apply order) of the hybrid sweep's restricted
    // applies: the Whitney dofs [0, n_whitney), the interface [0, col_int),
    // the interior [col_int, n)
    {
      P->col_int = n - int(loc_int.size());
      P->col_w0 = 0;
      P->col_w1 = P->n_whitney;
      for (int i = 0; i < n; ++i) {
        const rz::LocalDof &ld = P->el.dofs[P->perm[i]];
        const bool in_int = ld.entity_dim == d, in_w = i < P->col_w1;
        if (in_int != (i >= P->col_int) || in_w != (ld.entity_dim == P->k && ld.kind == rz::KIND_W))
          throw RzError{RZ_ERR_UNSUPPORTED, "unexpected local dof order"};
      }
      // the full vertex stars cover the interior too: the patch group's
      // corrections live on every local column, and no rows are interior
      if (full_stars) P->col_int = n;
    }
    HIPCHK(hipStreamSynchronize(s));
    if (P->pc == RZ_PC_HYBRID) estimate_weights(P.get(), s);
    P->scratch = scratch_address();
  } catch (const RzError &e) {
    return fail(e.code, e.msg);
  } catch (const std::invalid_argument &e) {
    return fail(RZ_ERR_MESH, e.what());
  } catch (const std::bad_alloc &) {
    return fail(RZ_ERR_OOM, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(RZ_ERR_UNSUPPORTED, e.what());
  }
  P->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_setup).count();
  *out = P.release();
  return RZ_OK;
}

int rz_sizes(const rz_problem *P, int64_t *n_dofs, int64_t *n_interior, int32_t *n_loc, int32_t *Q) {
  if (!P) return fail(RZ_ERR_ARG, "null handle");
  if (n_dofs) *n_dofs = P->top.n_dofs;
  if (n_interior) *n_interior = P->top.n_interior;
  if (n_loc) *n_loc = P->el.n;
  if (Q) *Q = P->el.Q;
  return RZ_OK;
}

int rz_pc_weights(const rz_problem *P, double *rho) {
  if (!P || !rho) return fail(RZ_ERR_ARG, "null argument");
  rho[0] = P->rho_I;
  rho[1] = P->rho_G;
  rho[2] = P->rho_W;
  return RZ_OK;
}

int rz_patch_set_info(const rz_problem *P, int32_t set, int32_t *n_sets, int64_t *n_patches, int32_t *max_size,
                      int64_t *stored_entries, int64_t *packed_entries, int64_t *sum_size) {
  if (!P) return fail(RZ_ERR_ARG, "null argument");
  if (n_sets) *n_sets = int32_t(P->dps.size());
  if (set < 0 || set >= int32_t(P->dps.size())) {
    if (n_patches || max_size || stored_entries || packed_entries || sum_size)
      return fail(RZ_ERR_ARG, "no such patch family");
    return RZ_OK;
  }
  const DevPatchSet &d = P->dps[set];
  int64_t packed = 0, msum = 0, mmax = 0;
  for (int64_t m : d.sizes) packed += m * (m + 1) / 2, msum += m, mmax = std::max(mmax, m);
  if (n_patches) *n_patches = int64_t(d.sizes.size());
  if (max_size) *max_size = int32_t(mmax);
  if (stored_entries) *stored_entries = d.n_inv;
  if (packed_entries) *packed_entries = packed;
  if (sum_size) *sum_size = msum;
  return RZ_OK;
}

int rz_patch_set_apply(rz_problem *P, int32_t set, const double *r, double *z, int32_t n_rhs, int64_t ld,
                       void *hip_stream) {
  if (!P || !r || !z) return fail(RZ_ERR_ARG, "null argument");
  if (set < 0 || set >= int32_t(P->pas.size())) return fail(RZ_ERR_ARG, "no such patch family");
  if (n_rhs < 1 || ld < P->top.n_dofs) return fail(RZ_ERR_ARG, "bad n_rhs or ld");
  rz::launch_patch_apply(P->pas[set], r, ld, z, ld, n_rhs, nullptr, static_cast<hipStream_t>(hip_stream), false, 1.0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RZ_ERR_DEVICE, hipGetErrorString(e));
  return RZ_OK;
}

int rz_dirichlet_dofs(const rz_problem *P, int64_t *n, int32_t *dofs) {
  if (!P) return fail(RZ_ERR_ARG, "null argument");
  if (n) *n = int64_t(P->dir_dofs.size());
  if (dofs) std::copy(P->dir_dofs.begin(), P->dir_dofs.end(), dofs);
  return RZ_OK;
}

static int reduction_blocks(int ncol) { return std::max(4, 512 / std::max(1, ncol)); }

// grows the Krylov workspace to hold ncol columns
static void ensure_ws(rz_problem *P, int ncol) {
  if (ncol <= P->ws_cols) return;
  P->free_ws();
  ++P->ws_gen;
  for (auto &d : P->dps) d.pa.zb = d.pa.rt = nullptr, d.pa.zb_cols = 0;
  for (auto &pa : P->pas) pa.zb = pa.rt = nullptr, pa.zb_cols = 0;
  const int64_t nd = P->top.n_dofs;
  const int RB = reduction_blocks(ncol);
  auto alloc = [&](size_t bytes) {
    void *ptr = nullptr;
    HIPCHK(hipMalloc(&ptr, std::max<size_t>(bytes, 8)));
    P->ws.push_back(ptr);
    return ptr;
  };
  P->st = static_cast<rz::PcgState *>(alloc(sizeof(rz::PcgState) * ncol));
  HIPCHK(hipHostMalloc((void **)&P->st_host, sizeof(rz::PcgState) * ncol, hipHostMallocDefault));
  P->r = static_cast<double *>(alloc(sizeof(double) * nd * ncol));
  P->z = static_cast<double *>(alloc(sizeof(double) * nd * ncol));
  P->pv = static_cast<double *>(alloc(sizeof(double) * nd * ncol));
  P->Ap = static_cast<double *>(alloc(sizeof(double) * nd * ncol));
  // any later solve with fewer columns uses more blocks per column; RB * nc <= 512 + 4 nc always
  const size_t npart = size_t(std::max<int64_t>(int64_t(RB) * ncol, 512 + 4 * int64_t(ncol)));
  P->partA = static_cast<double *>(alloc(sizeof(double) * npart));
  P->partR = static_cast<double *>(alloc(sizeof(double) * npart));
  P->partZ = static_cast<double *>(alloc(sizeof(double) * npart));
  P->partB = static_cast<double *>(alloc(sizeof(double) * npart));
  const size_t npad = size_t(P->ca.NT) * 64;
  P->ca.rW = static_cast<double *>(alloc(sizeof(double) * npad * ncol));
  P->ca.zW = static_cast<double *>(alloc(sizeof(double) * npad * ncol));
  P->fold.zW = P->ca.zW;
  // cell-local work vectors of the three-stage operator apply
  P->at.Xc = static_cast<double *>(alloc(sizeof(double) * size_t(P->at.KP) * P->at.ncp * ncol));
  P->at.Yc = static_cast<double *>(alloc(sizeof(double) * size_t(P->at.NP) * P->at.ncp * ncol));
  P->at.ws_cols = ncol;
  if (P->pc == RZ_PC_HYBRID) {
    P->hs = static_cast<double *>(alloc(sizeof(double) * nd * ncol));
    P->hd = static_cast<double *>(alloc(sizeof(double) * nd * ncol));
  }
  if (P->precision == RZ_FP32_IR) {
    P->sto = static_cast<rz::PcgState *>(alloc(sizeof(rz::PcgState) * ncol));
    HIPCHK(hipHostMalloc((void **)&P->sto_host, sizeof(rz::PcgState) * ncol, hipHostMallocDefault));
    P->ro = static_cast<double *>(alloc(sizeof(double) * nd * ncol));
    P->dx = static_cast<double *>(alloc(sizeof(double) * nd * ncol));
  }
  if (P->dlist) P->bm = static_cast<double *>(alloc(sizeof(double) * nd * ncol));
  for (int l = 0; l < P->mgdev.L; ++l) {
    rz::MgDevLevel &dl = P->mgdev.lev[l];
    if (l > 0) {
      dl.b = static_cast<double *>(alloc(sizeof(double) * dl.n * ncol));
      dl.x = static_cast<double *>(alloc(sizeof(double) * dl.n * ncol));
    }
    dl.t = static_cast<double *>(alloc(sizeof(double) * dl.n * ncol));
    dl.z = static_cast<double *>(alloc(sizeof(double) * dl.n * ncol));
    if (dl.nv) dl.u = static_cast<double *>(alloc(sizeof(double) * dl.nv * ncol));
  }
  P->ws_cols = ncol;
  if (ncol >= 8) {
    // many columns: the patch solves of the segmented sets become MFMA
    // products over fragment-ordered copies of the inverses (FP64; bfloat16
    // under RZ_BF16_PC; FP32 under RZ_FP32_PC and RZ_FP32_IR, whose inner
    // solves use the FP32 copies), with one shared result buffer
    const int kind = P->precision == RZ_BF16_PC ? 1 : (P->precision == RZ_FP64 ? 0 : 2);
    size_t zbytes = 0, rbytes = 0;
    for (auto &d : P->dps) {
      if (d.pa.fold || d.pa.n_patches == 0) continue;
      const void *have = kind == 1 ? (const void *)d.pa.frag16
                         : kind == 2 ? (const void *)d.pa.frag32 : (const void *)d.pa.frag64;
      if (!have) {
        std::vector<int64_t> off(d.sizes.size());
        int64_t tot = 0;
        for (size_t b = 0; b < d.sizes.size(); ++b) {
          off[b] = tot;
          tot += rz::frag_size(int(d.sizes[b]), kind);
        }
        const int64_t *doff = P->upload(off, nullptr);
        if (kind == 1) {
          uint16_t *f = P->dev<uint16_t>(size_t(tot));
          rz::launch_seg_to_frag(d.pa, kind, f, doff, nullptr);
          d.pa.frag16 = f;
          d.pa.frag_off16 = doff;
        } else if (kind == 2) {
          float *f = P->dev<float>(size_t(tot));
          rz::launch_seg_to_frag(d.pa, kind, f, doff, nullptr);
          d.pa.frag32 = f;
          d.pa.frag_off32 = doff;
        } else {
          double *f = P->dev<double>(size_t(tot));
          rz::launch_seg_to_frag(d.pa, kind, f, doff, nullptr);
          d.pa.frag64 = f;
          d.pa.frag_off64 = doff;
        }
      }
      zbytes = std::max(zbytes, size_t(d.pa.sum_size) * ncol * (kind == 0 ? 8 : 4));
      rbytes = std::max(rbytes, size_t(d.pa.n_adof) * ncol * 8);
    }
    if (zbytes) {
      void *zb = alloc(zbytes), *rt = alloc(rbytes);
      for (auto &d : P->dps)
        if (!d.pa.fold) d.pa.zb = zb, d.pa.rt = rt, d.pa.zb_cols = ncol;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    for (size_t i = 0; i < P->dps.size() && i < P->pas.size(); ++i) P->pas[i] = P->dps[i].pa;
  }
  if (ncol >= 8 && !P->ca.full && P->ca.tiles) {
    // many columns: the coarse solve becomes a GEMM over a full copy of the inverse
    const int NT = P->ca.NT;
    double *full = P->dev<double>(size_t(NT) * NT * 4096);
    rz::launch_coarse_expand(NT, P->ca.tiles, full, nullptr);
    HIPCHK(hipDeviceSynchronize());
    P->ca.full = full;
  }
}

// which pieces read the FP32 copies: the operator, the patch/coarse inverses
// reduced-precision pieces: kLoA the operator (everywhere: refinement's
// inner solves), kLoP the patch/coarse inverses, kLoH the operator inside
// the hybrid sweep only (the PCG operator stays FP64)
constexpr unsigned kLoA = 1, kLoP = 2, kLoH = 4;
// the pieces of plain (not refined) PCG that read reduced-precision copies
static unsigned pc_lo(const rz_problem *P) {
  if (P->precision == RZ_FP64) return 0u;
  return kLoP | (P->precision == RZ_BF16_PC ? kLoH : 0u);
}

// Symmetric multiplicative hybrid (Sec. 7.1): groups X_I (point-Jacobi),
// X_Gamma (additive interface patches) and W (exact coarse solve), swept
// I, Gamma, W, Gamma, I with z += rho_m^{-1} B_m (b - A z).  The residual
// s = r - A z is tracked: each correction d is applied to A restricted to
// the local columns it lives on (interior, interface, or the entities that
// carry the Whitney dofs) and subtracted from s.  With st the first kernel
// also takes the PCG convergence test (partR: block partials of ||r||^2).
static void hybrid_apply(rz_problem *P, const double *r, int64_t ldr, double *z, int64_t ldz, int nc,
                         rz::PcgState *st, const double *partR, int RB, unsigned lo, hipStream_t s) {
  const bool loA = lo & (kLoA | kLoH), loP = lo & kLoP;
  const int64_t nd = P->top.n_dofs;
  const int n = P->el.n;
  const double w1 = 1.0 / P->rho_I, w2 = 1.0 / P->rho_G;
  double *sres = P->hs, *d = P->hd;
  // d = 0 from here on before each correction: hyb_init clears it, and each
  // restricted apply of a correction clears it once it has read it
  rz::launch_hyb_init(nd, P->off_I, P->dinv, w1, r, ldr, z, ldz, sres, d, partR, RB, nc, st, s);
  if (P->col_int < n) rz::launch_apply_A(P->at, z, ldz, sres, nd, nc, st, s, loA, P->col_int, n, -1.0);
  // last: only the interior rows of the tracked residual are read afterwards
  // (by the final Jacobi step), so the second interface correction is
  // applied with A[I, Gamma] alone
  auto interface = [&](bool last) {
    for (auto &pa : P->pas) rz::launch_patch_apply(pa, sres, nd, d, nd, nc, st, s, loP, w2);
    rz::launch_add(nd, d, z, ldz, nc, st, s);
    if (last) {
      if (P->col_int < n)  // no interior rows: nothing reads the residual again
        rz::launch_apply_A(P->at, d, nd, sres, nd, nc, st, s, loA, 0, P->col_int, -1.0, P->col_int, P->off_I);
    } else
      rz::launch_apply_A(P->at, d, nd, sres, nd, nc, st, s, loA, 0, P->col_int, -1.0, 0, 0, false, true);
  };
  interface(false);
  rz::launch_coarse_gather(P->ca, sres, nd, nc, s);
  rz::launch_coarse_tiles(P->ca, nc, st, s, loP);
  rz::launch_coarse_scatter2(P->ca, nd, d, z, ldz, nc, st, s);
  rz::launch_apply_A(P->at, d, nd, sres, nd, nc, st, s, loA, P->col_w0, P->col_w1, -1.0, 0, 0, false, true);
  interface(true);
  rz::launch_jacobi_add(nd, P->off_I, P->dinv, w1, sres, z, ldz, nc, st, s);
}

static double host_dot(rz_problem *P, const double *a, const double *b, hipStream_t s) {
  const int RB = 64;
  const rz::CoarseFold nofold{nullptr, 0, 0, 1};
  rz::launch_dot(P->top.n_dofs, a, P->top.n_dofs, b, P->top.n_dofs, nofold, P->ca.NT * 64, P->partA, RB, 1, nullptr, s);
  double part[RB];
  HIPCHK(hipMemcpyAsync(part, P->partA, sizeof(part), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double v = 0.0;
  for (int i = 0; i < RB; ++i) v += part[i];
  return v;
}

// Weights rho = (lambda_min + 3 lambda_max) / 4 of the interior and
// interface groups (Sec. 7.1): extreme Ritz values of up to 10 CG steps on A
// restricted to the group's dofs [lo, hi), preconditioned by the group's
// solver, from b = 2u - 1 with u from SplitMix64 (seed 0x5EED1000 interior,
// 0x5EED2000 interface) per dof in ascending order; the steps stop early
// once ||r|| <= 1e-12 ||b||.  An empty group has rho = 1.
static double group_weight(rz_problem *P, int64_t lo, int64_t hi, uint64_t seed, bool interior, hipStream_t s) {
  const int64_t nd = P->top.n_dofs;
  if (hi <= lo) return 1.0;
  std::vector<double> hb(nd, 0.0);
  uint64_t state = seed;
  std::vector<uint8_t> removed(nd, 0);
  for (int32_t g : P->dir_dofs) removed[g] = 1;
  for (int64_t i = lo; i < hi; ++i) {
    if (removed[i]) continue;  // not in X^k_{p,D}: no draw
    state += 0x9E3779B97F4A7C15ull;
    uint64_t zz = state;
    zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ull;
    zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBull;
    zz ^= zz >> 31;
    hb[i] = 2.0 * (double(zz >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  }
  double *r = P->r, *z = P->z, *p = P->pv, *q = P->Ap;
  HIPCHK(hipMemcpy(r, hb.data(), nd * 8, hipMemcpyHostToDevice));
  auto apply_M = [&]() {
    rz::launch_fill(z, nd, nd, 1, nullptr, s);
    if (interior) {
      rz::launch_jacobi_add(nd, P->off_I, P->dinv, 1.0, r, z, nd, 1, nullptr, s);
    } else {
      for (auto &pa : P->pas) rz::launch_patch_apply(pa, r, nd, z, nd, 1, nullptr, s, false, 1.0);
      rz::launch_mask(nd, lo, hi, z, s);
    }
  };
  const double bb = host_dot(P, r, r, s);
  apply_M();
  HIPCHK(hipMemcpyAsync(p, z, nd * 8, hipMemcpyDeviceToDevice, s));
  double rz = host_dot(P, r, z, s);
  std::vector<double> al, be;
  for (int it = 0; it < 10 && rz > 0.0; ++it) {
    rz::launch_apply_A(P->at, p, nd, q, nd, 1, nullptr, s, false, 0, -1, 1.0, 0, 0, true);
    rz::launch_mask(nd, lo, hi, q, s);
    const double pq = host_dot(P, p, q, s);
    if (!(pq > 0.0)) throw RzError{RZ_ERR_NOT_SPD, "weight estimate: p^T A p <= 0"};
    const double a = rz / pq;
    al.push_back(a);
    rz::launch_axpby(nd, -a, q, 1.0, r, s);
    if (host_dot(P, r, r, s) <= 1e-24 * bb) break;
    apply_M();
    const double rz_new = host_dot(P, r, z, s);
    be.push_back(rz_new / rz);
    rz = rz_new;
    rz::launch_axpby(nd, 1.0, z, be.back(), p, s);
  }
  const int k = int(al.size());
  if (k == 0) return 1.0;
  rz::Dense T(k, k);
  for (int j = 0; j < k; ++j) {
    T(j, j) = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j > 0) T(j, j - 1) = T(j - 1, j) = std::sqrt(be[j - 1]) / al[j - 1];
  }
  std::vector<double> ev;
  rz::Dense V;
  rz::sym_eig(T, ev, V);
  return (ev.front() + 3.0 * ev.back()) / 4.0;
}

static void estimate_weights(rz_problem *P, hipStream_t s) {
  ensure_ws(P, 1);
  P->rho_I = group_weight(P, P->off_I, P->top.n_dofs, 0x5EED1000ull, true, s);
  P->rho_G = group_weight(P, 0, P->off_I, 0x5EED2000ull, false, s);
}

static int apply_A(rz_problem *P, const double *x, double *y, int32_t n_rhs, int64_t ld, void *hip_stream,
                   bool lo) {
  if (!P || !x || !y) return fail(RZ_ERR_ARG, "null argument");
  if (n_rhs < 1 || ld < P->top.n_dofs) return fail(RZ_ERR_ARG, "bad n_rhs or ld");
  if (lo && !P->at.Afrag32)
    return fail(RZ_ERR_ARG, "FP32 operator copies exist only for RZ_FP32_IR and RZ_BF16_PC handles");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  try {
    ensure_ws(P, n_rhs);
  } catch (const RzError &e) {
    return fail(e.code, e.msg);
  }
  rz::launch_apply_A(P->at, x, ld, y, ld, n_rhs, nullptr, s, lo, 0, -1, 1.0, 0, 0, true);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RZ_ERR_DEVICE, hipGetErrorString(e));
  return RZ_OK;
}

static int apply_P(rz_problem *P, const double *r, double *z, int32_t n_rhs, int64_t ld, void *hip_stream,
                   bool lo) {
  if (!P || !r || !z) return fail(RZ_ERR_ARG, "null argument");
  if (n_rhs < 1 || ld < P->top.n_dofs) return fail(RZ_ERR_ARG, "bad n_rhs or ld");
  if (lo && !P->ca.tiles32)
    return fail(RZ_ERR_ARG, "reduced-precision inverse copies exist only for RZ_FP32_IR, RZ_FP32_PC and RZ_BF16_PC "
                            "handles");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  try {
    ensure_ws(P, n_rhs);
  } catch (const RzError &e) {
    return fail(e.code, e.msg);
  }
  // the FP32 preconditioner of the handle's precision: inverses, plus the
  // operator inside the hybrid sweep under refinement
  const unsigned m = lo ? (kLoP | (P->at.Afrag32 ? kLoH : 0u)) : 0u;
  if (P->pc == RZ_PC_HYBRID)
    hybrid_apply(P, r, ld, z, ld, n_rhs, nullptr, nullptr, 0, m, s);
  else
    rz::launch_apply_P(P->pas.data(), int(P->pas.size()), P->ca, P->top.n_dofs, P->off_I, P->dinv, r, ld, z, ld,
                       n_rhs, s, lo);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RZ_ERR_DEVICE, hipGetErrorString(e));
  return RZ_OK;
}

int rz_apply_A(rz_problem *P, const double *x, double *y, int32_t n_rhs, int64_t ld, void *hip_stream) {
  return apply_A(P, x, y, n_rhs, ld, hip_stream, false);
}
int rz_apply_P(rz_problem *P, const double *r, double *z, int32_t n_rhs, int64_t ld, void *hip_stream) {
  return apply_P(P, r, z, n_rhs, ld, hip_stream, false);
}
int rz_apply_A_fp32(rz_problem *P, const double *x, double *y, int32_t n_rhs, int64_t ld, void *hip_stream) {
  return apply_A(P, x, y, n_rhs, ld, hip_stream, true);
}
int rz_apply_P_fp32(rz_problem *P, const double *r, double *z, int32_t n_rhs, int64_t ld, void *hip_stream) {
  return apply_P(P, r, z, n_rhs, ld, hip_stream, true);
}

int rz_apply_A_noalloc(rz_problem *P, const double *x, double *y, int32_t n_rhs, int64_t ld, void *hip_stream) {
  if (!P || !x || !y) return fail(RZ_ERR_ARG, "null argument");
  if (n_rhs < 1 || ld < P->top.n_dofs) return fail(RZ_ERR_ARG, "bad n_rhs or ld");
  if (!P->scratch) return fail(RZ_ERR_DEVICE, "static work array not looked up");
  const size_t per_col = (size_t(P->at.KP) + size_t(P->at.NP)) * size_t(P->at.ncp) * sizeof(double);
  if (per_col * size_t(n_rhs) > kScratchBytes)
    return fail(RZ_ERR_ARG, "rz_apply_A_noalloc: " + std::to_string(n_rhs) + " columns need " +
                                std::to_string(per_col * size_t(n_rhs)) + " bytes of cell-local work space, above the " +
                                std::to_string(kScratchBytes) + "-byte static array");
  rz::ApplyATables t = P->at;
  t.Xc = P->scratch;
  t.Yc = P->scratch + size_t(t.KP) * size_t(t.ncp) * size_t(n_rhs);
  t.ws_cols = n_rhs;
  rz::launch_apply_A(t, x, ld, y, ld, n_rhs, nullptr, static_cast<hipStream_t>(hip_stream), false, 0, -1, 1.0, 0, 0,
                     true);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RZ_ERR_DEVICE, hipGetErrorString(e));
  return RZ_OK;
}

// Lanczos estimate of kappa(P^{-1} A) from the CG coefficients (Sec. 7.1 reports these)
static double lanczos_cond(const rz::PcgState &h) {
  const int kk = std::min(h.iter, rz::kMaxIter);
  if (kk <= 0) return 1.0;
  rz::Dense T(kk, kk);
  for (int j = 0; j < kk; ++j) {
    T(j, j) = 1.0 / h.alphas[j] + (j > 0 ? h.betas[j - 1] / h.alphas[j - 1] : 0.0);
    if (j > 0) T(j, j - 1) = T(j - 1, j) = std::sqrt(std::max(0.0, h.betas[j - 1])) / h.alphas[j - 1];
  }
  std::vector<double> ev;
  rz::Dense V;
  rz::sym_eig(T, ev, V);
  return ev.front() > 0 ? ev.back() / ev.front() : 1.0;
}

// PCG (Sec. 7.1) on A x = b over nc columns to ||r_j|| <= tol ||b_j||, from x
// (or from zero when x_zero).  lo: kLoA / kLoP, which pieces read FP32 copies.
// outer (or null): columns whose outer state is done are skipped.  On return
// st_host holds every column's final state.
// PCG set-up part: r, ||b||, the per-column state, z = P^{-1} r, p = z.
static void pcg_begin(rz_problem *P, const double *b, int64_t ldb, double *x, int64_t ldx, int nc, double tol,
                      unsigned lo, bool x_zero, const rz::PcgState *outer, hipStream_t s) {
  const int64_t nd = P->top.n_dofs;
  const int maxit = P->max_iter;
  const int RB = reduction_blocks(nc);
  const int npad = P->ca.NT * 64;
  const rz::CoarseFold nofold{nullptr, 0, 0, 1};
  if (x_zero) {
    // r = b, ||r|| = ||b||
    rz::launch_fill(x, nd, ldx, nc, nullptr, s);
    rz::launch_copy(nd, b, ldb, P->r, nd, nc, s);
    rz::launch_dot(nd, b, ldb, b, ldb, nofold, npad, P->partB, RB, nc, nullptr, s);
    rz::launch_pcg_start(P->partB, P->partB, RB, tol * tol, maxit, P->st, nc, s, outer);
  } else {
    // r = b - A x, convergence reference ||b||
    rz::launch_apply_A(P->at, x, ldx, P->Ap, nd, nc, nullptr, s, lo & kLoA, 0, -1, 1.0, 0, 0, true);
    rz::launch_residual(nd, b, ldb, P->Ap, P->r, nc, s);
    rz::launch_dot(nd, b, ldb, b, ldb, nofold, npad, P->partB, RB, nc, nullptr, s);
    rz::launch_dot(nd, P->r, nd, P->r, nd, nofold, npad, P->partR, RB, nc, nullptr, s);
    rz::launch_pcg_start(P->partB, P->partR, RB, tol * tol, maxit, P->st, nc, s, outer);
  }
  // z = P^{-1} r, (r, z), p = z, Ap = 0
  if (P->pc == RZ_PC_HYBRID)
    hybrid_apply(P, P->r, nd, P->z, nd, nc, nullptr, nullptr, RB, lo, s);
  else
    rz::launch_apply_P(P->pas.data(), int(P->pas.size()), P->ca, nd, P->off_I, P->dinv, P->r, nd, P->z, nd, nc, s,
                       lo & kLoP);
  rz::launch_dot(nd, P->r, nd, P->z, nd, nofold, npad, P->partZ, RB, nc, P->st, s);
  rz::launch_copy(nd, P->z, nd, P->pv, nd, nc, s);
  rz::launch_fill(P->Ap, nd, nd, nc, nullptr, s);
}

// kPcgChunk PCG iterations: kernel launches only (no copies or host
// work), so the sequence can be captured into a HIP graph.
constexpr int kPcgChunk = 8;
static void pcg_chunk(rz_problem *P, double *x, int64_t ldx, int nc, unsigned lo, hipStream_t s) {
  const int64_t nd = P->top.n_dofs;
  const int RB = reduction_blocks(nc);
  const int npad = P->ca.NT * 64;
  const rz::CoarseFold nofold{nullptr, 0, 0, 1};
  const bool hyb = P->pc == RZ_PC_HYBRID;
  for (int it = 0; it < kPcgChunk; ++it) {
    // Ap was cleared by the previous p update; partZ holds the partials of (r, z)
    rz::launch_apply_A(P->at, P->pv, nd, P->Ap, nd, nc, P->st, s, lo & kLoA);
    rz::launch_dot(nd, P->pv, nd, P->Ap, nd, nofold, npad, P->partA, RB, nc, P->st, s);
    rz::launch_update_xr(nd, x, ldx, P->r, P->pv, P->Ap, P->partZ, P->partA, P->partR, RB, nc, P->st, s);
    if (hyb) {
      // convergence test and the hybrid sweep z = B r
      hybrid_apply(P, P->r, nd, P->z, nd, nc, P->st, P->partR, RB, lo, s);
      rz::launch_dot(nd, P->r, nd, P->z, nd, nofold, npad, P->partZ, RB, nc, P->st, s);
      rz::launch_update_p(nd, P->pv, P->z, nofold, npad, P->Ap, P->partZ, RB, nc, P->st, s);
      continue;
    }
    // convergence test, then z = P^{-1} r with the coarse part left in zW
    rz::launch_check_jacobi(nd, P->off_I, P->dinv, P->r, P->z, P->ca, P->partR, RB, nc, P->st, s);
    for (auto &pa : P->pas) rz::launch_patch_apply(pa, P->r, nd, P->z, nd, nc, P->st, s, lo & kLoP);
    rz::launch_coarse_tiles(P->ca, nc, P->st, s, lo & kLoP);
    rz::launch_dot(nd, P->r, nd, P->z, nd, P->fold, npad, P->partZ, RB, nc, P->st, s);
    rz::launch_update_p(nd, P->pv, P->z, P->fold, npad, P->Ap, P->partZ, RB, nc, P->st, s);
  }
}

static void pcg_read_head(rz_problem *P, int nc, hipStream_t s) {
  const size_t head = offsetof(rz::PcgState, alphas);
  HIPCHK(hipMemcpy2DAsync(P->st_host, sizeof(rz::PcgState), P->st, sizeof(rz::PcgState), head, nc,
                          hipMemcpyDeviceToHost, s));
}

// One chunk of PCG iterations: replayed from a HIP graph captured for the
// same (x, ldx, columns, precision, workspace) once that key has run one
// chunk directly (which also completes one-time kernel attribute set-up).
static void run_chunk(rz_problem *P, double *x, int64_t ldx, int nc, unsigned lo, hipStream_t s) {
  if (!P->graphs) {
    pcg_chunk(P, x, ldx, nc, lo, s);
    return;
  }
  rz_problem::GraphEntry *g = nullptr;
  for (auto &e : P->gcache)
    if (e.x == x && e.ldx == ldx && e.nc == nc && e.lo == lo && e.gen == P->ws_gen) g = &e;
  if (!g) {
    if (P->gcache.size() >= 4) {  // a few keys at most (solve vectors, refinement corrections)
      if (P->gcache.front().exec) HIPCHK(hipGraphExecDestroy(P->gcache.front().exec));
      P->gcache.erase(P->gcache.begin());
    }
    P->gcache.push_back({x, ldx, nc, lo, P->ws_gen, nullptr, false});
    g = &P->gcache.back();
  }
  if (!g->eager_done) {
    pcg_chunk(P, x, ldx, nc, lo, s);
    g->eager_done = true;
    return;
  }
  if (!g->exec) {
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    pcg_chunk(P, x, ldx, nc, lo, s);
    HIPCHK(hipStreamEndCapture(s, &graph));
    const hipError_t e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) throw RzError{RZ_ERR_DEVICE, hipGetErrorString(e)};
  }
  HIPCHK(hipGraphLaunch(g->exec, s));
}

static void pcg_run(rz_problem *P, const double *b, int64_t ldb, double *x, int64_t ldx, int nc, double tol, unsigned lo,
                    bool x_zero, const rz::PcgState *outer, hipStream_t user) {
  // with graphs the solve runs on the handle's own stream (capture needs a
  // stream other than the legacy default one), ordered after and before the
  // caller's stream by events
  hipStream_t s = user;
  if (P->graphs) {
    if (!P->gs) {
      HIPCHK(hipStreamCreateWithFlags(&P->gs, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&P->g_in, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&P->g_out, hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(P->g_in, user));
    HIPCHK(hipStreamWaitEvent(P->gs, P->g_in, 0));
    s = P->gs;
  }
  pcg_begin(P, b, ldb, x, ldx, nc, tol, lo, x_zero, outer, s);
  HIPCHK(hipGetLastError());
  for (int it0 = 0; it0 < P->max_iter; it0 += kPcgChunk) {
    run_chunk(P, x, ldx, nc, lo, s);
    HIPCHK(hipGetLastError());
    pcg_read_head(P, nc, s);
    HIPCHK(hipStreamSynchronize(s));
    bool all = true;
    for (int c = 0; c < nc; ++c) all = all && P->st_host[c].done;
    if (all) break;
  }
  HIPCHK(hipMemcpyAsync(P->st_host, P->st, sizeof(rz::PcgState) * nc, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (P->graphs) {
    HIPCHK(hipEventRecord(P->g_out, s));
    HIPCHK(hipStreamWaitEvent(user, P->g_out, 0));
  }
}

// Dirichlet boundary: bm = b with zeros on the removed dofs, and x = 0 there
static void mask_rhs(rz_problem *P, const double *b, int64_t ldb, double *x, int64_t ldx, int nc, hipStream_t s) {
  const int64_t nd = P->top.n_dofs;
  const int64_t nr = int64_t(P->dir_dofs.size());
  rz::launch_copy(nd, b, ldb, P->bm, nd, nc, s);
  rz::launch_zero_rows(P->dlist, nr, P->bm, nd, nc, s);
  rz::launch_zero_rows(P->dlist, nr, x, ldx, nc, s);
}

// Iterative refinement: r = b - A x in FP64, d from PCG on A d = r with the
// FP32 applies to inner_rtol, x += d, until ||b - A x|| <= rtol ||b|| per
// column.  A step that fails to halve the largest outer residual switches
// the remaining corrections to the FP64 applies.
static void refine(rz_problem *P, const double *b, int64_t ldb, double *x, int64_t ld, int nc, double rtol,
                   std::vector<int> &its, std::vector<int> &outer, std::vector<double> &cond, std::vector<double> &rel,
                   std::vector<int> &code, hipStream_t s) {
  const int64_t nd = P->top.n_dofs;
  const int RB = reduction_blocks(nc);
  const int npad = P->ca.NT * 64;
  const rz::CoarseFold nofold{nullptr, 0, 0, 1};
  const size_t head = offsetof(rz::PcgState, alphas);
  const int max_outer = 40;
  unsigned lo = kLoA | kLoP;
  std::vector<double> prev(nc, 0.0);
  for (int k = 0;; ++k) {
    // true residual and the outer convergence test
    rz::launch_apply_A(P->at, x, ld, P->Ap, nd, nc, nullptr, s, false, 0, -1, 1.0, 0, 0, true);
    rz::launch_residual(nd, b, ldb, P->Ap, P->ro, nc, s);
    rz::launch_dot(nd, b, ldb, b, ldb, nofold, npad, P->partB, RB, nc, nullptr, s);
    rz::launch_dot(nd, P->ro, nd, P->ro, nd, nofold, npad, P->partR, RB, nc, nullptr, s);
    rz::launch_pcg_start(P->partB, P->partR, RB, rtol * rtol, P->max_iter, P->sto, nc, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy2DAsync(P->sto_host, sizeof(rz::PcgState), P->sto, sizeof(rz::PcgState), head, nc,
                            hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    bool all = true;
    double worst_ratio = 0.0;
    for (int c = 0; c < nc; ++c) {
      const rz::PcgState &h = P->sto_host[c];
      rel[c] = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
      all = all && h.done;
      if (k > 0 && !h.done && prev[c] > 0) worst_ratio = std::max(worst_ratio, rel[c] / prev[c]);
      prev[c] = rel[c];
    }
    if (all || k == max_outer) break;
    if (worst_ratio > 0.5) lo = 0;
    // correction solve from zero on the columns that are not yet converged
    pcg_run(P, P->ro, nd, P->dx, nd, nc, P->inner_rtol, lo, true, P->sto, s);
    bool broke = false;
    for (int c = 0; c < nc; ++c) {
      if (P->sto_host[c].done) continue;
      const rz::PcgState &h = P->st_host[c];
      its[c] += h.iter;
      outer[c] += 1;
      if (outer[c] == 1) cond[c] = lanczos_cond(h);
      if (h.status == rz::PCG_BREAKDOWN) {
        if (!lo) code[c] = RZ_ERR_BREAKDOWN;
        broke = true;
      }
    }
    if (broke && !lo) break;
    if (broke) lo = 0;
    rz::launch_axpy(nd, P->dx, x, ld, nc, s);
  }
  for (int c = 0; c < nc; ++c)
    if (code[c] == RZ_OK && !P->sto_host[c].done) code[c] = RZ_ERR_NO_CONVERGENCE;
}

// outcome of one PCG column from its final state
static void column_info(const rz::PcgState &h, int &its, double &cond, double &rel, int &code) {
  its = h.iter;
  cond = lanczos_cond(h);
  rel = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
  code = RZ_OK;
  if (h.status == rz::PCG_MAXIT || !h.done) code = RZ_ERR_NO_CONVERGENCE;
  if (h.status == rz::PCG_BREAKDOWN) code = RZ_ERR_BREAKDOWN;
}

int rz_solve(rz_problem *P, const double *b, double *x, int32_t n_rhs, int64_t ld, double rtol, rz_info *info,
             void *hip_stream) {
  if (!P || !b || !x) return fail(RZ_ERR_ARG, "null argument");
  if (!(rtol > 0.0)) return fail(RZ_ERR_ARG, "rtol must be positive");
  if (n_rhs < 1 || ld < P->top.n_dofs) return fail(RZ_ERR_ARG, "bad n_rhs or ld");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int nc = n_rhs;
  try {
    ensure_ws(P, nc);
    std::vector<int> its(nc, 0), outer(nc, 0);
    std::vector<double> cond(nc, 1.0), rel(nc, 0.0);
    std::vector<int> code(nc, RZ_OK);
    auto t0 = std::chrono::steady_clock::now();
    // Dirichlet boundary: the removed dofs of b are ignored (a masked copy)
    // and x starts (and stays) zero on them
    const double *bb = b;
    int64_t ldb = ld;
    if (P->dlist) {
      mask_rhs(P, b, ld, x, ld, nc, s);
      bb = P->bm;
      ldb = P->top.n_dofs;
    }
    if (P->precision != RZ_FP32_IR) {
      // FP64 operator; FP32 inverses in the preconditioner for RZ_FP32_PC
      pcg_run(P, bb, ldb, x, ld, nc, rtol, pc_lo(P), false, nullptr, s);
      for (int c = 0; c < nc; ++c) column_info(P->st_host[c], its[c], cond[c], rel[c], code[c]);
    } else {
      refine(P, bb, ldb, x, ld, nc, rtol, its, outer, cond, rel, code, s);
    }
    auto t1 = std::chrono::steady_clock::now();
    int worst = RZ_OK;
    for (int c = 0; c < nc; ++c) {
      if (code[c] != RZ_OK && worst == RZ_OK) worst = code[c];
      if (info) {
        info[c].status = code[c];
        info[c].iterations = its[c];
        info[c].rel_residual = rel[c];
        info[c].cond_estimate = cond[c];
        info[c].solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        info[c].outer_iterations = outer[c];
        info[c].setup_ms = P->setup_ms;
      }
    }
    if (worst != RZ_OK) return fail(worst, worst == RZ_ERR_BREAKDOWN ? "CG breakdown" : "no convergence");
  } catch (const RzError &e) {
    return fail(e.code, e.msg);
  }
  return RZ_OK;
}

int rz_export_topology(const rz_problem *P, int32_t *cell_dofs, int64_t *n_patches, int64_t *n_patch_entries,
                       int64_t *patch_ptr, int32_t *patch_dofs) {
  if (!P) return fail(RZ_ERR_ARG, "null handle");
  if (cell_dofs) std::memcpy(cell_dofs, P->top.cell_dofs.data(), P->top.cell_dofs.size() * 4);
  const rz::PatchSet &ps = P->patches.at(0);  // plain patch set (first)
  const int64_t np = ps.n_patches();
  if (n_patches) *n_patches = np;
  if (n_patch_entries) *n_patch_entries = int64_t(ps.ent_dof.size());
  if (patch_ptr && patch_dofs) {
    for (int64_t p = 0; p <= np; ++p) patch_ptr[p] = ps.col_ent[ps.patch_col[p]];
    std::memcpy(patch_dofs, ps.ent_dof.data(), ps.ent_dof.size() * 4);
  }
  return RZ_OK;
}

int rz_export_reference(const rz_problem *P, double *Rq) {
  if (!P || !Rq) return fail(RZ_ERR_ARG, "null argument");
  std::memcpy(Rq, P->el.R.data(), P->el.R.size() * 8);
  return RZ_OK;
}

static int check_space(int32_t dim, int32_t degree, rz_space space, rz::Family &fam) {
  if (dim != 2 && dim != 3) return fail(RZ_ERR_ARG, "dim must be 2 or 3");
  if (space < RZ_HGRAD || space > RZ_HDIV2) return fail(RZ_ERR_ARG, "unknown space");
  if (degree < 1 || degree > 10) return fail(RZ_ERR_UNSUPPORTED, "degree must be in 1..10");
  if (dim == 2 && space > RZ_HDIV)
    return fail(RZ_ERR_UNSUPPORTED, "the second-kind spaces are built for tetrahedral meshes");
  fam = family_of(space);
  return RZ_OK;
}

int rz_reference(int32_t dim, int32_t degree, rz_space space, int32_t *n_loc, int32_t *Q, double *Rq) {
  rz::Family fam;
  if (int e = check_space(dim, degree, space, fam)) return e;
  try {
    rz::RefElement el = rz::build_reference(dim, fam, degree);
    if (n_loc) *n_loc = el.n;
    if (Q) *Q = el.Q;
    if (Rq) std::memcpy(Rq, el.R.data(), el.R.size() * 8);
  } catch (const std::exception &e) {
    return fail(RZ_ERR_UNSUPPORTED, e.what());
  }
  return RZ_OK;
}

static int numbering_impl(const rz_mesh *m, int32_t degree, rz_space space, int32_t dec, int64_t *n_dofs,
                          int32_t *cell_dofs, int64_t *n_patches, int64_t *n_patch_entries, int64_t *patch_ptr,
                          int32_t *patch_dofs) {
  if (!m || !m->cells) return fail(RZ_ERR_ARG, "null argument");
  if (int e = check_decomposition(dec, space, m->dim)) return e;
  rz::Family fam;
  if (int e = check_space(m->dim, degree, space, fam)) return e;
  if (m->n_vertices <= 0 || m->n_cells <= 0) return fail(RZ_ERR_ARG, "empty mesh");
  try {
    rz::RefElement el = rz::build_reference(m->dim, fam, degree);
    rz::Topology top = rz::build_topology(m->dim, m->n_vertices, m->n_cells, m->cells, el);
    if (n_dofs) *n_dofs = top.n_dofs;
    if (cell_dofs) std::memcpy(cell_dofs, top.cell_dofs.data(), top.cell_dofs.size() * 4);
    if (n_patches || n_patch_entries || (patch_ptr && patch_dofs)) {
      auto sets = rz::build_patches(top, el, rz::Decomposition(dec));
      const rz::PatchSet &ps = sets.at(0);
      const int64_t np = ps.n_patches();
      if (n_patches) *n_patches = np;
      if (n_patch_entries) *n_patch_entries = int64_t(ps.ent_dof.size());
      if (patch_ptr && patch_dofs) {
        for (int64_t p = 0; p <= np; ++p) patch_ptr[p] = ps.col_ent[ps.patch_col[p]];
        std::memcpy(patch_dofs, ps.ent_dof.data(), ps.ent_dof.size() * 4);
      }
    }
  } catch (const std::invalid_argument &e) {
    return fail(RZ_ERR_MESH, e.what());
  } catch (const std::exception &e) {
    return fail(RZ_ERR_UNSUPPORTED, e.what());
  }
  return RZ_OK;
}

int rz_numbering(const rz_mesh *m, int32_t degree, rz_space space, int64_t *n_dofs, int32_t *cell_dofs,
                 int64_t *n_patches, int64_t *n_patch_entries, int64_t *patch_ptr, int32_t *patch_dofs) {
  return numbering_impl(m, degree, space, RZ_DECOMP_PAPER, n_dofs, cell_dofs, n_patches, n_patch_entries, patch_ptr,
                        patch_dofs);
}

int rz_patch_lists(const rz_mesh *m, int32_t degree, rz_space space, int32_t decomposition, int64_t *n_patches,
                   int64_t *n_patch_entries, int64_t *patch_ptr, int32_t *patch_dofs) {
  return numbering_impl(m, degree, space, decomposition, nullptr, nullptr, n_patches, n_patch_entries, patch_ptr,
                        patch_dofs);
}

void rz_destroy(rz_problem *P) { delete P; }

}  // extern "C"

// A batch of independent problems solved together: one HIP stream per
// problem.  Each problem advances chunk by chunk on its own stream (PCG
// iterations in chunks of kPcgChunk replayed from the problem's captured
// graphs; under RZ_FP32_IR also the outer residual checks between the
// correction solves); the host launches a problem's next step as soon as its
// previous one has completed, without waiting for the others.
struct rz_batch {
  std::vector<rz_problem *> P;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done_ev;
  hipEvent_t start_ev = nullptr;
  ~rz_batch() {
    for (auto e : done_ev)
      if (e) (void)hipEventDestroy(e);
    if (start_ev) (void)hipEventDestroy(start_ev);
    for (auto st : streams)
      if (st) (void)hipStreamDestroy(st);
  }
};

// Autotuned cells per wave of the single-column operator apply, kept per
// (dim, space, degree, cells, dofs, precision) for the life of the process
// and, when the environment names a file in RZ_TUNING_FILE, in that file
// (one "dim space degree cells dofs precision cells_per_wave" line per
// key), so later batches and processes reuse the choice instead of timing
// again.
namespace {
struct TuneKey {
  int d, k, p, prec;
  int64_t n_cells, n_dofs;
  bool operator<(const TuneKey &o) const {
    return std::tie(d, k, p, prec, n_cells, n_dofs) < std::tie(o.d, o.k, o.p, o.prec, o.n_cells, o.n_dofs);
  }
};
std::map<TuneKey, int> g_tune;
std::mutex g_tune_mu;
bool g_tune_loaded = false;

void tune_file_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *path = std::getenv("RZ_TUNING_FILE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  TuneKey k{};
  long long nc = 0, nd = 0;
  int cpw = 0;
  while (std::fscanf(f, "%d %d %d %lld %lld %d %d", &k.d, &k.k, &k.p, &nc, &nd, &k.prec, &cpw) == 7) {
    k.n_cells = nc;
    k.n_dofs = nd;
    if (cpw == 16 || cpw == 32 || cpw == 64) g_tune[k] = cpw / 16;
  }
  std::fclose(f);
}

void tune_file_append(const TuneKey &k, int nb) {
  const char *path = std::getenv("RZ_TUNING_FILE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %lld %lld %d %d\n", k.d, k.k, k.p, (long long)k.n_cells, (long long)k.n_dofs, k.prec,
               16 * nb);
  std::fclose(f);
}
}  // namespace

// cells per wave of the single-column operator apply: a value set with
// rz_set_apply_tiles is kept; else the process's choice for the same key;
// else 16, 32 and 64 cells per wave are timed (best of three rounds of five
// applies each) and the fastest is kept only if it beats the occupancy
// default by more than 3% (timing noise does not flip the choice).
static void autotune_apply(rz_problem *P, hipStream_t s) {
  if (P->at.nb1 != 0) return;
  const TuneKey key{P->d, P->k, P->p, P->precision, P->top.n_cells, P->top.n_dofs};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_file_load();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      P->at.nb1 = it->second;
      return;
    }
  }
  const int64_t nd = P->top.n_dofs;
  ensure_ws(P, 1);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  rz::launch_fill(P->r, nd, nd, 1, nullptr, s);
  float t[5] = {1e30f, 1e30f, 1e30f, 1e30f, 1e30f};
  for (int round = 0; round < 3; ++round)
    for (int nb : {0, 1, 2, 4}) {
      P->at.nb1 = nb;
      rz::launch_apply_A(P->at, P->r, nd, P->Ap, nd, 1, nullptr, s);  // warm-up
      HIPCHK(hipEventRecord(e0, s));
      for (int rep = 0; rep < 5; ++rep) rz::launch_apply_A(P->at, P->r, nd, P->Ap, nd, 1, nullptr, s);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      t[nb] = std::min(t[nb], ms);
    }
  int best = 0;
  for (int nb : {1, 2, 4})
    if (t[nb] < 0.97f * t[0] && t[nb] < t[best] * (best == 0 ? 1.0f / 0.97f : 1.0f)) best = nb;
  P->at.nb1 = best;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune.emplace(key, best).second && best != 0) tune_file_append(key, best);
}

extern "C" {

int rz_set_apply_tiles(rz_problem *P, int32_t cells_per_wave, int32_t every_apply) {
  if (!P) return fail(RZ_ERR_ARG, "null argument");
  if (cells_per_wave != 0 && cells_per_wave != 16 && cells_per_wave != 32 && cells_per_wave != 64)
    return fail(RZ_ERR_ARG, "cells_per_wave must be 0, 16, 32 or 64");
  if (every_apply) {
    P->at.nb_all = cells_per_wave / 16;
    P->free_graphs();  // captured chunks baked in the old launch shapes
  } else {
    P->at.nb1 = cells_per_wave / 16;
  }
  return RZ_OK;
}

int rz_get_apply_tiles(const rz_problem *P, int32_t *cells_per_wave) {
  if (!P || !cells_per_wave) return fail(RZ_ERR_ARG, "null argument");
  *cells_per_wave = 16 * P->at.nb1;
  return RZ_OK;
}

int rz_batch_create(rz_problem *const *problems, int32_t n, rz_batch **out) {
  if (!problems || !out || n < 1) return fail(RZ_ERR_ARG, "null argument or empty batch");
  *out = nullptr;
  for (int i = 0; i < n; ++i)
    if (!problems[i]) return fail(RZ_ERR_ARG, "null problem in batch");
  auto B = std::make_unique<rz_batch>();
  try {
    B->P.assign(problems, problems + n);
    B->streams.assign(n, nullptr);
    B->done_ev.assign(n, nullptr);
    HIPCHK(hipEventCreateWithFlags(&B->start_ev, hipEventDisableTiming));
    for (int i = 0; i < n; ++i) {
      HIPCHK(hipStreamCreateWithFlags(&B->streams[i], hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&B->done_ev[i], hipEventDisableTiming));
      autotune_apply(B->P[i], B->streams[i]);
      B->P[i]->free_graphs();  // the tuned shape changes what a chunk launches
    }
  } catch (const RzError &e) {
    return fail(e.code, e.msg);
  }
  *out = B.release();
  return RZ_OK;
}

namespace {
// one batch member's progress: plain PCG chunks, or refinement alternating
// an outer residual check with the chunks of a correction solve
struct Member {
  enum Phase { PCG, OUTER, INNER, DONE } phase = PCG;
  unsigned lo = 0;          // reduced-precision pieces of the current solve
  int rounds = 0;           // chunks of the current (correction) solve
  int k = 0;                // refinement: outer checks so far
  double prev = 0.0;        // refinement: previous outer relative residual
  bool cond_pending = false;
  rz_info info{};
};
}  // namespace

int rz_batch_solve(rz_batch *B, const double *const *b, double *const *x, double rtol, rz_info *info,
                   void *hip_stream) {
  if (!B || !b || !x) return fail(RZ_ERR_ARG, "null argument");
  if (!(rtol > 0.0)) return fail(RZ_ERR_ARG, "rtol must be positive");
  const int n = int(B->P.size());
  for (int i = 0; i < n; ++i)
    if (!b[i] || !x[i]) return fail(RZ_ERR_ARG, "null vector in batch");
  hipStream_t user = static_cast<hipStream_t>(hip_stream);
  int worst = RZ_OK;
  const size_t head = offsetof(rz::PcgState, alphas);
  const int max_outer = 40;
  try {
    auto t0 = std::chrono::steady_clock::now();
    HIPCHK(hipEventRecord(B->start_ev, user));
    std::vector<Member> M(n);
    std::vector<const double *> bv(b, b + n);  // right-hand sides as solved (masked under Gamma_D)
    // refinement: FP64 true residual of x and its convergence state in sto
    auto outer_check = [&](int i) {
      rz_problem *P = B->P[i];
      hipStream_t s = B->streams[i];
      const int64_t nd = P->top.n_dofs;
      const int RB = reduction_blocks(1);
      const int npad = P->ca.NT * 64;
      const rz::CoarseFold nofold{nullptr, 0, 0, 1};
      rz::launch_apply_A(P->at, x[i], nd, P->Ap, nd, 1, nullptr, s, false, 0, -1, 1.0, 0, 0, true);
      rz::launch_residual(nd, bv[i], nd, P->Ap, P->ro, 1, s);
      rz::launch_dot(nd, bv[i], nd, bv[i], nd, nofold, npad, P->partB, RB, 1, nullptr, s);
      rz::launch_dot(nd, P->ro, nd, P->ro, nd, nofold, npad, P->partR, RB, 1, nullptr, s);
      rz::launch_pcg_start(P->partB, P->partR, RB, rtol * rtol, P->max_iter, P->sto, 1, s);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(P->sto_host, P->sto, head, hipMemcpyDeviceToHost, s));
      M[i].phase = Member::OUTER;
    };
    auto chunk = [&](int i, double *xv) {
      rz_problem *P = B->P[i];
      run_chunk(P, xv, P->top.n_dofs, 1, M[i].lo, B->streams[i]);
      HIPCHK(hipGetLastError());
      pcg_read_head(P, 1, B->streams[i]);
      ++M[i].rounds;
    };
    std::vector<int> active;
    for (int i = 0; i < n; ++i) {
      rz_problem *P = B->P[i];
      hipStream_t s = B->streams[i];
      HIPCHK(hipStreamWaitEvent(s, B->start_ev, 0));
      ensure_ws(P, 1);
      if (P->dlist) {  // Dirichlet boundary: solve with the masked right-hand side
        mask_rhs(P, bv[i], P->top.n_dofs, x[i], P->top.n_dofs, 1, s);
        bv[i] = P->bm;
      }
      if (P->precision == RZ_FP32_IR) {
        M[i].lo = kLoA | kLoP;
        outer_check(i);
      } else {
        M[i].lo = pc_lo(P);
        pcg_begin(P, bv[i], P->top.n_dofs, x[i], P->top.n_dofs, 1, rtol, M[i].lo, false, nullptr, s);
        HIPCHK(hipGetLastError());
        chunk(i, x[i]);
      }
      active.push_back(i);
    }
    // the next step of a member whose stream has drained; false when it is done
    auto advance = [&](int i) -> bool {
      rz_problem *P = B->P[i];
      hipStream_t s = B->streams[i];
      Member &m = M[i];
      const int64_t nd = P->top.n_dofs;
      if (m.phase == Member::PCG) {
        if (!P->st_host[0].done && m.rounds * kPcgChunk < P->max_iter) {
          chunk(i, x[i]);
          return true;
        }
        HIPCHK(hipMemcpyAsync(P->st_host, P->st, sizeof(rz::PcgState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int its, code;
        double cond, rel;
        column_info(P->st_host[0], its, cond, rel, code);
        m.info.status = code;
        m.info.iterations = its;
        m.info.rel_residual = rel;
        m.info.cond_estimate = cond;
        m.phase = Member::DONE;
        return false;
      }
      if (m.phase == Member::OUTER) {
        if (m.cond_pending) {  // the first correction solve's full state has arrived
          m.info.cond_estimate = lanczos_cond(P->st_host[0]);
          m.cond_pending = false;
        }
        const rz::PcgState &h = P->sto_host[0];
        const double rel = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
        m.info.rel_residual = rel;
        if (h.done || m.k == max_outer || m.info.status == RZ_ERR_BREAKDOWN) {
          if (m.info.status == RZ_OK && !h.done) m.info.status = RZ_ERR_NO_CONVERGENCE;
          m.phase = Member::DONE;
          return false;
        }
        if (m.k > 0 && m.prev > 0 && rel / m.prev > 0.5) m.lo = 0;
        m.prev = rel;
        ++m.k;
        pcg_begin(P, P->ro, nd, P->dx, nd, 1, P->inner_rtol, m.lo, true, P->sto, s);
        HIPCHK(hipGetLastError());
        m.rounds = 0;
        m.phase = Member::INNER;
        chunk(i, P->dx);
        return true;
      }
      // INNER: next chunk of the correction solve, or its end
      const rz::PcgState &h = P->st_host[0];
      if (!h.done && m.rounds * kPcgChunk < P->max_iter) {
        chunk(i, P->dx);
        return true;
      }
      m.info.iterations += h.iter;
      m.info.outer_iterations += 1;
      if (m.info.outer_iterations == 1) {
        HIPCHK(hipMemcpyAsync(P->st_host, P->st, sizeof(rz::PcgState), hipMemcpyDeviceToHost, s));
        m.cond_pending = true;
      }
      if (h.status == rz::PCG_BREAKDOWN) {
        if (!m.lo) {
          m.info.status = RZ_ERR_BREAKDOWN;
          HIPCHK(hipStreamSynchronize(s));
          if (m.cond_pending) m.info.cond_estimate = lanczos_cond(P->st_host[0]);
          m.phase = Member::DONE;
          return false;
        }
        m.lo = 0;
      }
      rz::launch_axpy(nd, P->dx, x[i], nd, 1, s);
      outer_check(i);
      return true;
    };
    std::vector<double> t_done(n, 0.0);
    while (!active.empty()) {
      std::vector<int> next;
      bool progress = false;
      for (int i : active) {
        const hipError_t q = hipStreamQuery(B->streams[i]);
        if (q == hipErrorNotReady) {
          next.push_back(i);
          continue;
        }
        if (q != hipSuccess) throw RzError{RZ_ERR_DEVICE, hipGetErrorString(q)};
        progress = true;
        if (advance(i)) {
          next.push_back(i);
        } else {
          t_done[i] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
      }
      active.swap(next);
      if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(10));
    }
    for (int i = 0; i < n; ++i) {
      if (M[i].info.status != RZ_OK && worst == RZ_OK) worst = M[i].info.status;
      if (info) {
        info[i] = M[i].info;
        info[i].solve_ms = t_done[i];
        info[i].setup_ms = B->P[i]->setup_ms;
      }
      HIPCHK(hipEventRecord(B->done_ev[i], B->streams[i]));
      HIPCHK(hipStreamWaitEvent(user, B->done_ev[i], 0));
    }
  } catch (const RzError &e) {
    return fail(e.code, e.msg);
  }
  if (worst != RZ_OK) return fail(worst, worst == RZ_ERR_BREAKDOWN ? "CG breakdown" : "no convergence");
  return RZ_OK;
}

void rz_batch_destroy(rz_batch *B) { delete B; }

}  // extern "C"

// ---------------------------------------------------------------- Hodge Laplacians
// eq:hodge-laplace on X^{k-1} x X^k (k = 1: CG_p x Ned_p, k = 2: Ned_p x RT_p,
// k = 3: RT_p x DG_{p-1}), natural boundary conditions, in the two bases:
//   [ -M_{k-1}   D^T M_k ] [sigma]
//   [  M_k D     K_k     ] [  u  ]
// with D the exterior derivative in the X^k basis (d X^{k-1}_p lies in X^k_p),
// preconditioned by the weighted Riesz maps of eq:augmented-lagrangian, each
// one application of the Schwarz preconditioner of its handle:
// (sigma, tau) + gamma (d sigma, d tau) on X^{k-1} (alpha = gamma, beta = 1)
// and gamma^{-1} (u, v) + (d u, d v) on X^k (alpha = 1, beta = 1 / gamma).
// For k = 3, K_3 = 0 and DG_{p-1} carries the L2-orthonormal basis of
// P_{p-1} on the reference cell pulled back as a 3-form (psi_hat / det J), so
// M_3 is diagonal, 1 / |det J_T| per cell: it is folded into the rows of D
// (the stored matrix is M_3 D), and gamma^{-1} M_3 is inverted exactly.
namespace {
// Entries of a reference derivative matrix at or below 1e-12 of its largest
// are taken as round-off of exact zeros and left out of the stored CSR
// (lem:d-preserves-basis-functions makes the gradient matrix the signed
// vertex-edge incidence plus an identity, yet its computed zeros fill the
// rest of the matrix at 1e-16..1e-13; the curl and divergence matrices
// carry round-off up to 1e-12 from p = 6 on, below the tables' own
// accuracy).  Dropping them changes a row of D x by at most 1e-12 max|D_hat|
// times the sum of |x| over the dropped columns.
double drop_tol(const std::vector<double> &Dh) {
  double mx = 0.0;
  for (double v : Dh) mx = std::max(mx, std::fabs(v));
  return 1e-12 * mx;
}
}  // namespace

struct rz_hodge {
  rz_problem *P0 = nullptr, *P1 = nullptr;
  int k = 1, p = 1, max_iter = 1000;
  double gamma = 1.0;
  int64_t n0 = 0, n1 = 0;
  rz::ApplyATables tM0{}, tM1{}, tK1{};  // mass of X^{k-1}, mass and stiffness of X^k
  const int64_t *dp = nullptr, *dtp = nullptr;
  const int32_t *dc = nullptr, *dtc = nullptr;
  const double *dv = nullptr, *dtv = nullptr;
  int d_lanes = 1, dt_lanes = 1;  // lanes per row of the two SpMVs
  std::vector<void *> mem;
  double *t2 = nullptr, *m2 = nullptr;  // 2 n1 each: [D sigma, u] and their X^k masses
  double *dg_inv = nullptr;            // k = 3: gamma |det J_T| per DG dof
  double *vec = nullptr;               // MINRES: 7 vectors of n0 + n1
  double *part = nullptr, *part_host = nullptr;
  static constexpr int kParts = 256;
  template <class T>
  T *dev(size_t count) {
    void *ptr = nullptr;
    HIPCHK(hipMalloc(&ptr, std::max<size_t>(count, 1) * sizeof(T)));
    mem.push_back(ptr);
    return static_cast<T *>(ptr);
  }
  template <class T>
  T *upload(const std::vector<T> &v) {
    T *ptr = dev<T>(v.size());
    if (!v.empty()) HIPCHK(hipMemcpy(ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return ptr;
  }
  ~rz_hodge() {
    for (void *ptr : mem) (void)hipFree(ptr);
    if (part_host) (void)hipHostFree(part_host);
    rz_destroy(P1);
    rz_destroy(P0);
  }
};

namespace {
// y = A x for the mixed matrix (x, y: [sigma; u])
int hodge_apply(rz_hodge *H, const double *x, double *y, hipStream_t s) {
  const int64_t n0 = H->n0, n1 = H->n1;
  const double *sg = x, *u = x + n0;
  double *y0 = y, *y1 = y + n0;
  if (H->k == 3) {
    rz::launch_csr_spmv(n1, H->dp, H->dc, H->dv, sg, y1, 1.0, false, H->d_lanes, s);  // M_3 D sigma
    rz::launch_apply_A(H->tM0, sg, n0, y0, n0, 1, nullptr, s, false, 0, -1, -1.0, 0, 0, true);  // -M sigma
    rz::launch_csr_spmv(n0, H->dtp, H->dtc, H->dtv, u, y0, 1.0, true, H->dt_lanes, s);  // + (M_3 D)^T u
    return RZ_OK;
  }
  rz::launch_csr_spmv(n1, H->dp, H->dc, H->dv, sg, H->t2, 1.0, false, H->d_lanes, s);  // D sigma
  HIPCHK(hipMemcpyAsync(H->t2 + n1, u, size_t(n1) * 8, hipMemcpyDeviceToDevice, s));   // u
  rz::launch_apply_A(H->tM1, H->t2, n1, H->m2, n1, 2, nullptr, s, false, 0, -1, 1.0, 0, 0, true);
  rz::launch_apply_A(H->tK1, u, n1, y1, n1, 1, nullptr, s, false, 0, -1, 1.0, 0, 0, true);  // K u
  rz::launch_lincomb3(n1, 1.0, y1, 1.0, H->m2, 0.0, nullptr, y1, s);                    // + M D sigma
  rz::launch_apply_A(H->tM0, sg, n0, y0, n0, 1, nullptr, s, false, 0, -1, -1.0, 0, 0, true);  // -M sigma
  rz::launch_csr_spmv(n0, H->dtp, H->dtc, H->dtv, H->m2 + n1, y0, 1.0, true, H->dt_lanes, s);  // + D^T M u
  return RZ_OK;
}

int hodge_apply_P(rz_hodge *H, const double *r, double *z, hipStream_t s) {
  int rc = apply_P(H->P0, r, z, 1, H->n0, s, false);
  if (rc != RZ_OK) return rc;
  if (H->k == 3) {
    rz::launch_diag_mul(H->n1, H->dg_inv, r + H->n0, z + H->n0, s);
    return RZ_OK;
  }
  return apply_P(H->P1, r + H->n0, z + H->n0, 1, H->n1, s, false);
}

double hodge_dot(rz_hodge *H, const double *a, const double *b, hipStream_t s) {
  rz::launch_dot_part(H->n0 + H->n1, a, b, H->part, rz_hodge::kParts, s);
  HIPCHK(hipMemcpyAsync(H->part_host, H->part, sizeof(double) * rz_hodge::kParts, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double v = 0.0;
  for (int i = 0; i < rz_hodge::kParts; ++i) v += H->part_host[i];  // fixed order
  return v;
}
}  // namespace

extern "C" {

int rz_derivative_reference(int32_t k, int32_t degree, int32_t *n_to, int32_t *n_from, double *D) {
  if (k < 1 || k > 3) return fail(RZ_ERR_UNSUPPORTED, "k must be 1 (grad), 2 (curl) or 3 (div)");
  if (degree < 1 || degree > 10) return fail(RZ_ERR_UNSUPPORTED, "degree must be in 1..10");
  try {
    if (k == 3) {
      const int na = rz::build_reference(3, rz::FAM_RT, degree).n;
      const int nb = degree * (degree + 1) * (degree + 2) / 6;
      if (n_to) *n_to = nb;
      if (n_from) *n_from = na;
      if (D) {
        std::vector<double> Dh = rz::divergence_reference_dg(3, degree);
        std::copy(Dh.begin(), Dh.end(), D);
      }
      return RZ_OK;
    }
    const rz::Family from = k == 1 ? rz::FAM_CG : rz::FAM_NED, to = k == 1 ? rz::FAM_NED : rz::FAM_RT;
    const int na = rz::build_reference(3, from, degree).n, nb = rz::build_reference(3, to, degree).n;
    if (n_to) *n_to = nb;
    if (n_from) *n_from = na;
    if (D) {
      std::vector<double> Dh = rz::derivative_reference(3, from, to, degree);
      std::copy(Dh.begin(), Dh.end(), D);
    }
  } catch (const std::exception &e) {
    return fail(RZ_ERR_UNSUPPORTED, e.what());
  }
  return RZ_OK;
}

int rz_hodge_setup(const rz_mesh *m, int32_t degree, int32_t k, double gamma, const rz_options *opts,
                   void *hip_stream, rz_hodge **out) {
  if (!m || !out) return fail(RZ_ERR_ARG, "null argument");
  *out = nullptr;
  if (k < 1 || k > 3) return fail(RZ_ERR_UNSUPPORTED, "k must be 1 (CG x Ned), 2 (Ned x RT) or 3 (RT x DG)");
  if (m->dim != 3) return fail(RZ_ERR_UNSUPPORTED, "the Hodge Laplacians are built for tetrahedral meshes");
  if (!(gamma > 0.0)) return fail(RZ_ERR_ARG, "need gamma > 0");
  if (opts && opts->precision != RZ_FP64) return fail(RZ_ERR_UNSUPPORTED, "the Hodge Laplacians run in RZ_FP64");
  if (opts && opts->dirichlet_facet) return fail(RZ_ERR_UNSUPPORTED, "the Hodge Laplacians take natural boundary conditions");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  auto H = std::make_unique<rz_hodge>();
  H->k = k;
  H->p = degree;
  H->gamma = gamma;
  if (opts && opts->max_iter > 0) H->max_iter = opts->max_iter;
  rz_options o0{};
  if (opts) o0 = *opts;
  else {
    o0.max_iter = 1000;
    o0.pc = RZ_PC_HYBRID;
  }
  rz_options o1 = o0;
  o0.alpha = gamma;  // (sigma, tau) + gamma (d sigma, d tau)
  o0.beta = 1.0;
  o1.alpha = 1.0;    // gamma^{-1} (u, v) + (d u, d v)
  o1.beta = 1.0 / gamma;
  const rz_space s0 = k == 1 ? RZ_HGRAD : k == 2 ? RZ_HCURL : RZ_HDIV, s1 = k == 1 ? RZ_HCURL : RZ_HDIV;
  int rc = rz_setup(m, degree, s0, &o0, hip_stream, &H->P0);
  if (rc != RZ_OK) return rc;
  if (k < 3) {
    rc = rz_setup(m, degree, s1, &o1, hip_stream, &H->P1);
    if (rc != RZ_OK) return rc;
  }
  rz_problem *P0 = H->P0, *P1 = H->P1;
  const int64_t nc = P0->top.n_cells;
  H->n0 = P0->top.n_dofs;
  try {
    ensure_ws(P0, 1);
    // mass-only and stiffness-only weights (linear in (alpha, beta); the
    // stacked mass family comes first: one matrix for a scalar field, six
    // component pairs for a vector field)
    const int qm0 = P0->k == 0 ? 1 : 6;
    double *wM0 = H->dev<double>(size_t(nc) * P0->el.Q);
    rz::launch_scale_weights(nc, P0->el.Q, qm0, P0->w, 1.0, 0.0, wM0, s);
    H->tM0 = P0->at;
    H->tM0.w = wM0;
    // the entries of D (n1 x n0), keyed row * n0 + col
    std::vector<std::pair<int64_t, double>> ent;
    const int na = P0->el.n;
    if (k < 3) {
      H->n1 = P1->top.n_dofs;
      ensure_ws(P1, 2);
      const int qm1 = P1->k == 0 ? 1 : 6;
      double *wM1 = H->dev<double>(size_t(nc) * P1->el.Q), *wK1 = H->dev<double>(size_t(nc) * P1->el.Q);
      rz::launch_scale_weights(nc, P1->el.Q, qm1, P1->w, gamma, 0.0, wM1, s);
      rz::launch_scale_weights(nc, P1->el.Q, qm1, P1->w, 0.0, 1.0, wK1, s);
      H->tM1 = P1->at;
      H->tM1.w = wM1;
      H->tK1 = P1->at;
      H->tK1.w = wK1;
      // D from the reference D_hat placed per cell (every cell's basis is the
      // pullback of the sorted-vertex reference basis, and the pullbacks
      // commute with d); entries shared by cells coincide
      const rz::Family f0 = k == 1 ? rz::FAM_CG : rz::FAM_NED, f1 = k == 1 ? rz::FAM_NED : rz::FAM_RT;
      const std::vector<double> Dh = rz::derivative_reference(3, f0, f1, degree);
      const double tol = drop_tol(Dh);
      const int nb = P1->el.n;
      ent.reserve(size_t(nc) * nb * 4);
      for (int64_t c = 0; c < nc; ++c)
        for (int i = 0; i < nb; ++i)
          for (int j = 0; j < na; ++j) {
            const double v = Dh[size_t(i) * na + j];
            if (std::fabs(v) <= tol) continue;
            ent.push_back({int64_t(P1->top.cell_dofs[c * nb + i]) * H->n0 + P0->top.cell_dofs[c * na + j], v});
          }
    } else {
      // DG_{p-1}: cell c owns dofs c * nb .. c * nb + nb - 1; the stored
      // matrix is M_3 D, row (c, i) = D_hat row i / |det J_c|
      const std::vector<double> Dh = rz::divergence_reference_dg(3, degree);
      const double tol = drop_tol(Dh);
      const int nb = int(Dh.size() / size_t(na));
      H->n1 = nc * nb;
      std::vector<double> Ve(12);
      rz::eq_vertices(3, Ve.data());
      auto det3 = [](const double J[3][3]) {
        return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      };
      double E[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) E[a][b] = Ve[(b + 1) * 3 + a] - Ve[a];
      const double detE = std::fabs(det3(E));
      std::vector<double> inv(size_t(H->n1));
      ent.reserve(size_t(nc) * nb * na);
      for (int64_t c = 0; c < nc; ++c) {
        const int64_t *v = &P0->top.cells[c * 4];
        double J[3][3];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) J[a][b] = m->coords[v[b + 1] * 3 + a] - m->coords[v[0] * 3 + a];
        const double dj = std::fabs(det3(J)) / detE;  // |det| of the map from the reference cell
        for (int i = 0; i < nb; ++i) {
          inv[size_t(c) * nb + i] = gamma * dj;
          for (int j = 0; j < na; ++j) {
            const double val = Dh[size_t(i) * na + j];
            if (std::fabs(val) <= tol) continue;
            ent.push_back({(c * nb + i) * H->n0 + P0->top.cell_dofs[c * na + j], val / dj});
          }
        }
      }
      H->dg_inv = H->upload(inv);
    }
    std::sort(ent.begin(), ent.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    std::vector<int64_t> keys;
    std::vector<double> vals;
    for (size_t e = 0; e < ent.size(); ++e)
      if (keys.empty() || keys.back() != ent[e].first) {
        keys.push_back(ent[e].first);
        vals.push_back(ent[e].second);
      }
    auto csr = [&](bool transpose, std::vector<int64_t> &ptr, std::vector<int32_t> &col, std::vector<double> &val) {
      const int64_t nr = transpose ? H->n0 : H->n1;
      ptr.assign(nr + 1, 0);
      for (int64_t key : keys) ++ptr[(transpose ? key % H->n0 : key / H->n0) + 1];
      for (int64_t r = 0; r < nr; ++r) ptr[r + 1] += ptr[r];
      std::vector<int64_t> pos(ptr.begin(), ptr.end() - 1);
      col.assign(keys.size(), 0);
      val.assign(keys.size(), 0.0);
      for (size_t e = 0; e < keys.size(); ++e) {
        const int64_t r = transpose ? keys[e] % H->n0 : keys[e] / H->n0;
        const int64_t cc = transpose ? keys[e] / H->n0 : keys[e] % H->n0;
        col[pos[r]] = int32_t(cc);
        val[pos[r]++] = vals[e];
      }
    };
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    // lanes per row from the mean row length (the SpMV sums a row's entries
    // lane-strided and reduces them across the lanes)
    auto lanes = [](int64_t nnz, int64_t rows) {
      const double avg = rows > 0 ? double(nnz) / double(rows) : 0.0;
      return avg < 3.0 ? 1 : avg < 12.0 ? 4 : avg < 48.0 ? 16 : 64;
    };
    H->d_lanes = lanes(int64_t(keys.size()), H->n1);
    H->dt_lanes = lanes(int64_t(keys.size()), H->n0);
    csr(false, ptr, col, val);
    H->dp = H->upload(ptr);
    H->dc = H->upload(col);
    H->dv = H->upload(val);
    csr(true, ptr, col, val);
    H->dtp = H->upload(ptr);
    H->dtc = H->upload(col);
    H->dtv = H->upload(val);
    if (k < 3) {
      H->t2 = H->dev<double>(size_t(2) * H->n1);
      H->m2 = H->dev<double>(size_t(2) * H->n1);
    }
    H->vec = H->dev<double>(size_t(7) * (H->n0 + H->n1));
    H->part = H->dev<double>(rz_hodge::kParts);
    HIPCHK(hipHostMalloc((void **)&H->part_host, sizeof(double) * rz_hodge::kParts, hipHostMallocDefault));
    HIPCHK(hipStreamSynchronize(s));
  } catch (const RzError &e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc &) {
    return fail(RZ_ERR_OOM, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(RZ_ERR_UNSUPPORTED, e.what());
  }
  *out = H.release();
  return RZ_OK;
}

int rz_hodge_sizes(const rz_hodge *H, int64_t *n0, int64_t *n1) {
  if (!H) return fail(RZ_ERR_ARG, "null handle");
  if (n0) *n0 = H->n0;
  if (n1) *n1 = H->n1;
  return RZ_OK;
}

int rz_hodge_apply(rz_hodge *H, const double *x, double *y, void *hip_stream) {
  if (!H || !x || !y) return fail(RZ_ERR_ARG, "null argument");
  try {
    hodge_apply(H, x, y, static_cast<hipStream_t>(hip_stream));
  } catch (const RzError &e) {
    return fail(e.code, e.msg);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RZ_ERR_DEVICE, hipGetErrorString(e));
  return RZ_OK;
}

int rz_hodge_apply_P(rz_hodge *H, const double *r, double *z, void *hip_stream) {
  if (!H || !r || !z) return fail(RZ_ERR_ARG, "null argument");
  return hodge_apply_P(H, r, z, static_cast<hipStream_t>(hip_stream));
}

// Preconditioned MINRES (Paige & Saunders 1975): the Lanczos process in the
// P^{-1} inner product and the Givens QR of its tridiagonal matrix, x_0 = 0,
// stopping when the preconditioned residual norm |phibar| <= rtol ||b||_P.
// The scalars live on the host (two inner products per iteration); the
// vectors, the operator and the preconditioner on the device.
int rz_hodge_solve(rz_hodge *H, const double *b, double *x, double rtol, rz_info *info, void *hip_stream) {
  if (!H || !b || !x) return fail(RZ_ERR_ARG, "null argument");
  if (!(rtol > 0.0)) return fail(RZ_ERR_ARG, "need rtol > 0");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int64_t n = H->n0 + H->n1;
  double *r1 = H->vec, *r2 = H->vec + n, *y = H->vec + 2 * n, *v = H->vec + 3 * n, *w = H->vec + 4 * n,
         *w1 = H->vec + 5 * n, *w2 = H->vec + 6 * n;
  const auto t0 = std::chrono::steady_clock::now();
  int it = 0, status = RZ_ERR_NO_CONVERGENCE;
  double rel = 1.0;
  try {
    rz::launch_lincomb3(n, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, x, s);   // x = 0
    rz::launch_lincomb3(n, 1.0, b, 0.0, nullptr, 0.0, nullptr, r1, s);        // r1 = b
    rz::launch_lincomb3(n, 1.0, b, 0.0, nullptr, 0.0, nullptr, r2, s);        // r2 = b
    rz::launch_lincomb3(n, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, w, s);
    rz::launch_lincomb3(n, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, w2, s);
    int rc = hodge_apply_P(H, r1, y, s);
    if (rc != RZ_OK) return rc;
    const double beta1 = std::sqrt(std::max(0.0, hodge_dot(H, r1, y, s)));
    if (beta1 == 0.0) {
      status = RZ_OK;
      rel = 0.0;
    } else {
      double oldb = 0.0, beta = beta1, dbar = 0.0, epsln = 0.0, phibar = beta1, cs = -1.0, sn = 0.0;
      for (it = 1; it <= H->max_iter; ++it) {
        rz::launch_lincomb3(n, 1.0 / beta, y, 0.0, nullptr, 0.0, nullptr, v, s);   // v = y / beta
        hodge_apply(H, v, y, s);                                                    // y = A v
        if (it >= 2) rz::launch_lincomb3(n, 1.0, y, -beta / oldb, r1, 0.0, nullptr, y, s);
        const double alfa = hodge_dot(H, v, y, s);
        rz::launch_lincomb3(n, 1.0, y, -alfa / beta, r2, 0.0, nullptr, y, s);
        std::swap(r1, r2);  // r1 = old r2; r2 <- y (copied below)
        rz::launch_lincomb3(n, 1.0, y, 0.0, nullptr, 0.0, nullptr, r2, s);
        rc = hodge_apply_P(H, r2, y, s);
        if (rc != RZ_OK) return rc;
        oldb = beta;
        beta = std::sqrt(std::max(0.0, hodge_dot(H, r2, y, s)));
        const double oldeps = epsln;
        const double delta = cs * dbar + sn * alfa;
        const double gbar = sn * dbar - cs * alfa;
        epsln = sn * beta;
        dbar = -cs * beta;
        const double gmm = std::max(std::hypot(gbar, beta), 1e-300);
        cs = gbar / gmm;
        sn = beta / gmm;
        const double phi = cs * phibar;
        phibar = sn * phibar;
        std::swap(w1, w2);  // w1 <- old w2, w2 <- old w (rotate)
        std::swap(w2, w);
        // w = (v - oldeps w1 - delta w2) / gamma; x += phi w
        rz::launch_lincomb3(n, 1.0 / gmm, v, -oldeps / gmm, w1, -delta / gmm, w2, w, s);
        rz::launch_lincomb3(n, 1.0, x, phi, w, 0.0, nullptr, x, s);
        rel = std::fabs(phibar) / beta1;
        if (!std::isfinite(rel)) {
          status = RZ_ERR_BREAKDOWN;
          break;
        }
        if (rel <= rtol) {
          status = RZ_OK;
          break;
        }
      }
      if (it > H->max_iter) it = H->max_iter;
    }
    HIPCHK(hipStreamSynchronize(s));
  } catch (const RzError &e) {
    return fail(e.code, e.msg);
  }
  if (info) {
    *info = rz_info{};
    info->status = status;
    info->iterations = it;
    info->rel_residual = rel;
    info->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (status == RZ_ERR_NO_CONVERGENCE) return fail(status, "MINRES reached max_iter");
  if (status == RZ_ERR_BREAKDOWN) return fail(status, "non-finite MINRES scalar");
  return RZ_OK;
}

void rz_hodge_destroy(rz_hodge *H) { delete H; }

}  // extern "C"
