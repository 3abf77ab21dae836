// Host side of the solver library: validation, device layouts, setup,
// V-cycle orchestration, FGMRES, and the C ABI declared in include/fsi_mg.h.
#include "fsi_internal.h"

#include <type_traits>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

namespace fsi {

thread_local std::string g_last_error;

// Static Krylov workspace of fsi_fgmres_solve_noalloc, one per device (each
// device that loads the library holds it until the process ends).  Host code
// never uses the symbol itself as an address: scratch_address() takes the
// device address once per device, with that device current, and keeps it.
constexpr int64_t kStaticScratchBytes = 64ll << 20;
static __device__ __align__(256) double scratch[kStaticScratchBytes / 8];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];
static double *scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Error(FSI_E_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "static workspace address");
    if (!ptr) throw Error(FSI_E_DEVICE, "static workspace address is null");
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
  }
  return g_scratch_ptr[dev];
}

void set_error(const std::string &m) { g_last_error = m; }

void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      throw Error(FSI_E_OOM, std::string(what) + ": " + hipGetErrorString(e));
    throw Error(FSI_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}

int pick_lpr(int64_t nnz, int64_t nrows) {
  if (nrows <= 0) return 2;
  const double avg = (double)nnz / (double)nrows;
  int l = 2;
  while (l < 64 && l * 4 < avg) l *= 2;
  return l;
}

// ------------------------------------------------------------------ validation
static void validate_csr(const fsi_csr &A, int64_t nrows, int64_t ncols, const char *name, int lev) {
  char buf[256];
  auto fail = [&](const char *why) {
    snprintf(buf, sizeof buf, "level %d %s: %s", lev, name, why);
    throw Error(FSI_E_INVALID, buf);
  };
  if (A.nrows != nrows || A.ncols != ncols) fail("dimension mismatch");
  if (A.nnz < 0 || A.nnz >= (int64_t)1 << 31) fail("nnz out of range");
  if (!A.rowptr || (A.nnz > 0 && (!A.colind || !A.val))) fail("null array");
  if (A.rowptr[0] != 0 || A.rowptr[A.nrows] != A.nnz) fail("row offsets do not span nnz");
  for (int64_t r = 0; r < A.nrows; ++r) {
    if (A.rowptr[r + 1] < A.rowptr[r]) fail("row offsets not monotone");
    for (int64_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) {
      const int32_t c = A.colind[p];
      if (c < 0 || c >= ncols) fail("column index out of range");
      if (p > A.rowptr[r] && c <= A.colind[p - 1]) fail("columns not strictly increasing");
    }
  }
}

static void validate_patches(const fsi_patches &P, int64_t n, int lev) {
  char buf[256];
  auto fail = [&](const char *why, int64_t k) {
    snprintf(buf, sizeof buf, "level %d patches: %s (patch %lld)", lev, why, (long long)k);
    throw Error(FSI_E_INVALID, buf);
  };
  if (P.npatch <= 0 || !P.ptr || !P.dof || !P.owned) fail("no patches", -1);
  if (P.ptr[0] != 0) fail("ptr[0] != 0", 0);
  std::vector<int> owner_count(n, 0), present(n, 0);
  for (int k = 0; k < P.npatch; ++k) {
    const int64_t a = P.ptr[k], b = P.ptr[k + 1];
    if (b <= a) fail("empty patch", k);
    if (b - a > kMaxLargePatch) fail("patch larger than the supported block size (6144 dofs)", k);
    for (int64_t p = a; p < b; ++p) {
      const int32_t d = P.dof[p];
      if (d < 0 || d >= n) fail("dof out of range", k);
      if (p > a && d <= P.dof[p - 1]) fail("dofs not strictly increasing", k);
      present[d] = 1;
      if (P.owned[p]) owner_count[d]++;
    }
  }
  for (int64_t d = 0; d < n; ++d) {
    if (owner_count[d] > 1) fail("dof owned by more than one patch", d);
    if (present[d] && owner_count[d] == 0) fail("dof covered but owned by no patch", d);
  }
}

// Dirichlet flags (optional): a flagged dof's row is the identity row (the
// Newton correction is zero there) and no patch holds it (section
// "Richardson-Schwarz smoother": the blocks are built on the unknowns)
static void validate_dirichlet(const fsi_level &L, int64_t n, int lev) {
  char buf[256];
  const fsi_csr &J = L.J;
  for (int64_t d = 0; d < n; ++d) {
    if (!L.dirichlet[d]) continue;
    const int64_t a = J.rowptr[d], b = J.rowptr[d + 1];
    if (b - a != 1 || J.colind[a] != d || J.val[a] != 1.0) {
      snprintf(buf, sizeof buf, "level %d: Dirichlet dof %lld does not hold an identity row", lev, (long long)d);
      throw Error(FSI_E_INVALID, buf);
    }
  }
  if (lev == 0) return;
  const fsi_patches &P = L.patches;
  for (int k = 0; k < P.npatch; ++k)
    for (int64_t p = P.ptr[k]; p < P.ptr[k + 1]; ++p)
      if (L.dirichlet[P.dof[p]]) {
        snprintf(buf, sizeof buf, "level %d patch %d: holds Dirichlet dof %d", lev, k, P.dof[p]);
        throw Error(FSI_E_INVALID, buf);
      }
}

// ------------------------------------------------------------------ device helpers
void *DevicePool::get(size_t bytes, size_t *got) {
  {
    std::lock_guard<std::mutex> lk(mu);
    // best fit among the cached blocks, wasting at most a quarter
    auto it = free_blocks.lower_bound(bytes);
    if (it != free_blocks.end() && it->first <= bytes + bytes / 4 + 4096) {
      void *p = it->second;
      *got = it->first;
      free_blocks.erase(it);
      in_use += (int64_t)*got;
      peak_in_use = std::max(peak_in_use, in_use);
      return p;
    }
  }
  void *p = nullptr;
  hip_check(hipMalloc(&p, bytes), "hipMalloc");
  std::lock_guard<std::mutex> lk(mu);
  all.push_back(p);
  *got = bytes;
  allocated += (int64_t)bytes;
  in_use += (int64_t)bytes;
  peak_in_use = std::max(peak_in_use, in_use);
  return p;
}
void DevicePool::put(void *p, size_t bytes) {
  std::lock_guard<std::mutex> lk(mu);
  free_blocks.emplace(bytes, p);
  in_use -= (int64_t)bytes;
}
DevicePool::~DevicePool() {
  for (void *p : all) (void)hipFree(p);
}

template <typename T>
T *dalloc(int64_t n, DevList &owned) {
  if (n <= 0) return nullptr;
  const size_t bytes = (sizeof(T) * (size_t)n + 255) / 256 * 256;
  void *p = nullptr;
  size_t got = bytes;
  if (owned.pool)
    p = owned.pool->get(bytes, &got);
  else
    hip_check(hipMalloc(&p, bytes), "hipMalloc");
  owned.v.push_back({p, got});
  return static_cast<T *>(p);
}
static void free_one(DevList &owned, size_t i) {
  auto &e = owned.v[i];
  if (owned.pool)
    owned.pool->put(e.first, e.second);
  else
    (void)hipFree(e.first);
  owned.v.erase(owned.v.begin() + i);
}
// 64-byte slots of host-coherent pinned memory that kernels write small
// results into and the host polls.  Chunks are allocated once and kept for the
// life of the process; slots are recycled.
static std::mutex g_slot_mu;
static std::vector<double *> g_free_slots;
double *pinned_slot_acquire() {
  std::lock_guard<std::mutex> lk(g_slot_mu);
  if (g_free_slots.empty()) {
    constexpr int kSlots = 256;
    double *p = nullptr;
    hip_check(hipHostMalloc((void **)&p, kSlots * 8 * sizeof(double),
                            hipHostMallocCoherent | hipHostMallocMapped | hipHostMallocPortable),
              "pinned");
    for (int i = kSlots - 1; i >= 0; --i) g_free_slots.push_back(p + 8 * i);
  }
  double *s = g_free_slots.back();
  g_free_slots.pop_back();
  for (int i = 0; i < 8; ++i) s[i] = 0.0;
  return s;
}
void pinned_slot_release(double *s) {
  std::lock_guard<std::mutex> lk(g_slot_mu);
  g_free_slots.push_back(s);
}

// Host-to-device uploads go through a pinned staging buffer of the calling
// thread: the copies are asynchronous (no per-copy staging by the runtime)
// and the host source may be released at once.  The buffer is reused after
// the stream has drained; a setup ends with such a drain.
struct Staging {
  char *buf = nullptr;
  size_t cap = 0, off = 0;
  hipStream_t st = nullptr;
  ~Staging() {
    if (buf) (void)hipHostFree(buf);
  }
};
static thread_local Staging g_stage;
static void stage_drain() {
  if (g_stage.st) hip_check(hipStreamSynchronize(g_stage.st), "upload");
  g_stage.off = 0;
  g_stage.st = nullptr;
}
static void stage_copy(void *dst, const void *src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  Staging &S = g_stage;
  if (S.st && S.st != st) stage_drain();
  if (S.off + bytes > S.cap) {
    stage_drain();
    if (bytes > S.cap) {
      if (S.buf) (void)hipHostFree(S.buf);
      S.buf = nullptr;
      S.cap = std::max<size_t>(bytes, 64u << 20);
      hip_check(hipHostMalloc((void **)&S.buf, S.cap, 0), "pinned staging");
    }
  }
  std::memcpy(S.buf + S.off, src, bytes);
  hip_check(hipMemcpyAsync(dst, S.buf + S.off, bytes, hipMemcpyHostToDevice, st), "H2D");
  S.off += (bytes + 255) / 256 * 256;
  S.st = st;
}

template <typename T>
T *dupload(const T *h, int64_t n, DevList &owned, hipStream_t st) {
  T *d = dalloc<T>(n, owned);
  if (n > 0) stage_copy(d, h, sizeof(T) * (size_t)n, st);
  return d;
}

static void upload_csr(const fsi_csr &A, DevCsr &D, bool want32, DevList &own, hipStream_t st) {
  D.n = A.nrows;
  D.m = A.ncols;
  D.nnz = (int)A.nnz;
  std::vector<int32_t> rp(A.nrows + 1);
  for (int64_t i = 0; i <= A.nrows; ++i) rp[i] = (int32_t)A.rowptr[i];
  D.rowptr = dupload(rp.data(), A.nrows + 1, own, st);
  D.col = dupload(A.colind, A.nnz, own, st);
  D.val = dupload(A.val, A.nnz, own, st);
  if (want32) {
    std::vector<float> v32(A.nnz);
    for (int64_t i = 0; i < A.nnz; ++i) v32[i] = (float)A.val[i];
    D.val32 = dupload(v32.data(), A.nnz, own, st);
  }
  D.lpr = pick_lpr(A.nnz, A.nrows);
}

// ------------------------------------------------------------------ patch layout
// the solid blocks get their own storage (FP32 owned rows, or full FP32
// inverses with refinement sweeps) in a mixed hierarchy whose options ask for it
static bool solid_split(const fsi_mg_opts &o) {
  return o.precision != FSI_PREC_FP64 &&
         ((o.solid_precision != -1 && o.solid_precision != o.precision) || o.refine_sweeps > 0);
}
static void build_patch_layout(Level &L, const fsi_patches &P, const fsi_csr &J, MG &mg,
                               hipStream_t st) {
  L.npatch = P.npatch;
  const int np = P.npatch;
  L.h_ptr.assign(P.ptr, P.ptr + np + 1);
  L.h_dof.assign(P.dof, P.dof + P.ptr[np]);
  L.h_owned.assign(P.owned, P.owned + P.ptr[np]);
  L.h_kind.assign(np, 0);
  if (P.kind) L.h_kind.assign(P.kind, P.kind + np);
  std::vector<int> pm(np), po(np), out_off(np + 1, 0), own_local, out_idx, task_patch, task_row0;
  std::vector<int64_t> pdof_off(np), woff(np + 1, 0), woff16(np + 1, 0), boff(np + 1, 0);
  std::vector<int> row_patch, row_local;
  // solid blocks (kind 1) apart when the options give them their own
  // storage: their owned rows in FP32 (task list _s, offsets into Ws), or,
  // with refinement sweeps, their whole FP32 inverses (task list over all
  // rows, offsets into Wfull) and their sparse block B_k
  const bool split = solid_split(mg.opts);
  const bool refine = split && mg.opts.refine_sweeps > 0;
  std::vector<int> task_patch_s, task_row0_s, po_full(np, 0), full_off(np + 1, 0), full_local, ftask_patch,
      ftask_row0, ref_patch;
  std::vector<int64_t> woff_full(np, 0);
  int64_t wmain = 0, wsolid = 0, wfull = 0, wmain16 = 0;
  L.mmax = 0;
  L.sum_m = L.sum_m2 = L.sum_om = 0;
  // fluid blocks with ILU(0) factors (fluid_ilu): no explicit inverse
  const bool ilu = mg.opts.fluid_ilu != 0;
  std::vector<int> ilu_patch;
  for (int k = 0; k < np; ++k) {
    const int64_t a = P.ptr[k], b = P.ptr[k + 1];
    const bool solid = split && L.h_kind[k] == 1;
    const bool is_ilu = ilu && L.h_kind[k] == 0;
    if (is_ilu) ilu_patch.push_back(k);
    pm[k] = (int)(b - a);
    pdof_off[k] = a;
    int o = 0;
    for (int64_t p = a; p < b; ++p)
      if (P.owned[p]) {
        own_local.push_back((int)(p - a));
        out_idx.push_back(P.dof[p]);
        ++o;
      }
    po[k] = o;
    out_off[k + 1] = out_off[k] + o;
    // woff[k]: offset of the patch's owned rows in its class's storage
    int64_t &wcls = solid ? wsolid : wmain;
    woff[k] = wcls;
    woff16[k] = wmain16;
    if (!is_ilu) wcls += (int64_t)o * pm[k];
    if (!is_ilu && !solid) wmain16 += (int64_t)o * ((pm[k] + 3) & ~3);
    boff[k + 1] = boff[k] + (int64_t)pm[k] * pm[k];
    for (int i = 0; i < pm[k]; ++i) {
      row_patch.push_back(k);
      row_local.push_back(i);
    }
    if (refine && solid) {
      ref_patch.push_back(k);
      po_full[k] = pm[k];
      woff_full[k] = wfull;
      wfull += (int64_t)pm[k] * pm[k];
      for (int i = 0; i < pm[k]; ++i) full_local.push_back(i);
      full_off[k + 1] = full_off[k] + pm[k];
      for (int r0 = 0; r0 < pm[k]; r0 += 64) {
        ftask_patch.push_back(k);
        ftask_row0.push_back(r0);
      }
    } else {
      full_off[k + 1] = full_off[k];
      for (int r0 = 0; r0 < o && !is_ilu; r0 += 64) {
        (solid ? task_patch_s : task_patch).push_back(k);
        (solid ? task_row0_s : task_row0).push_back(r0);
      }
    }
    L.mmax = std::max(L.mmax, pm[k]);
    L.sum_m += pm[k];
    L.sum_m2 += (int64_t)pm[k] * pm[k];
    if (!is_ilu) L.sum_om += (int64_t)o * pm[k];
  }
  woff[np] = wmain;
  woff16[np] = wmain16;
  L.total_owned = out_off[np];
  std::vector<char> is_owned(L.n, 0);
  for (int d : out_idx) is_owned[d] = 1;
  std::vector<int> unowned;
  for (int d = 0; d < L.n; ++d)
    if (!is_owned[d]) unowned.push_back(d);
  L.n_unowned = (int)unowned.size();
  L.ntask = (int)task_patch.size();
  auto &own = mg.owned;
  L.d_pm = dupload(pm.data(), np, own, st);
  L.d_po = dupload(po.data(), np, own, st);
  L.d_pdof_off = dupload(pdof_off.data(), np, own, st);
  L.d_woff = dupload(woff.data(), np + 1, own, st);
  L.d_woff16 = dupload(woff16.data(), np + 1, own, st);
  L.d_boff = dupload(boff.data(), np + 1, own, st);
  L.d_dof = dupload(P.dof, P.ptr[np], own, st);
  L.d_out_off = dupload(out_off.data(), np + 1, own, st);
  L.d_own_local = dupload(own_local.data(), (int64_t)own_local.size(), own, st);
  L.d_out_idx = dupload(out_idx.data(), (int64_t)out_idx.size(), own, st);
  L.d_task_patch = dupload(task_patch.data(), (int64_t)task_patch.size(), own, st);
  L.d_task_row0 = dupload(task_row0.data(), (int64_t)task_row0.size(), own, st);
  L.d_row_patch = dupload(row_patch.data(), (int64_t)row_patch.size(), own, st);
  L.d_row_local = dupload(row_local.data(), (int64_t)row_local.size(), own, st);
  L.d_unowned = dupload(unowned.data(), (int64_t)unowned.size(), own, st);
  L.boff_total = boff[np];
  L.woff_total = wmain;
  L.woff16_total = wmain16;
  L.woff_solid = wsolid;
  L.h_boff = boff;
  L.ntask_s = (int)task_patch_s.size();
  L.d_task_patch_s = dupload(task_patch_s.data(), (int64_t)task_patch_s.size(), own, st);
  L.d_task_row0_s = dupload(task_row0_s.data(), (int64_t)task_row0_s.size(), own, st);
  if (refine && !ref_patch.empty()) {
    // full inverses (all rows, the packing's task layout) and each refined
    // block's rows of B_k = J[I_k, I_k] as local CSR with the J entry index of
    // every value (the values follow the operator through refactors)
    L.nref = (int)ref_patch.size();
    L.wfull_total = wfull;
    L.full_rows = full_off[np];
    L.nftask = (int)ftask_patch.size();
    L.d_po_full = dupload(po_full.data(), np, own, st);
    L.d_woff_full = dupload(woff_full.data(), np, own, st);
    L.d_full_off = dupload(full_off.data(), np + 1, own, st);
    L.d_full_local = dupload(full_local.data(), (int64_t)full_local.size(), own, st);
    L.d_ftask_patch = dupload(ftask_patch.data(), (int64_t)ftask_patch.size(), own, st);
    L.d_ftask_row0 = dupload(ftask_row0.data(), (int64_t)ftask_row0.size(), own, st);
    L.d_ref_patch = dupload(ref_patch.data(), (int64_t)ref_patch.size(), own, st);
    std::vector<int> rptr_off(np, 0), rptr, rcol, rsrc;
    for (int k : ref_patch) {
      rptr_off[k] = (int)rptr.size();
      const int32_t *I = P.dof + P.ptr[k];
      const int m = pm[k];
      rptr.push_back((int)rcol.size());
      for (int i = 0; i < m; ++i) {
        const int g = I[i];
        for (int64_t q = J.rowptr[g]; q < J.rowptr[g + 1]; ++q) {
          const int32_t c = J.colind[q];
          const int32_t *f = std::lower_bound(I, I + m, c);
          if (f != I + m && *f == c) {
            rcol.push_back((int)(f - I));
            rsrc.push_back((int)q);
          }
        }
        rptr.push_back((int)rcol.size());
      }
    }
    std::vector<int> own_dof(full_off[np], -1);
    for (int k : ref_patch)
      for (int i = 0; i < pm[k]; ++i)
        if (P.owned[P.ptr[k] + i]) own_dof[full_off[k] + i] = P.dof[P.ptr[k] + i];
    L.d_own_dof = dupload(own_dof.data(), (int64_t)own_dof.size(), own, st);
    L.yref0 = dalloc<float>(full_off[np], own);
    L.yref1 = dalloc<float>(full_off[np], own);
    // the blocks as one CSR over the refined rows: row full_off[k] + i,
    // columns full_off[k] + local column
    std::vector<int> growptr(full_off[np] + 1, 0), gcol(rcol.size());
    for (int k : ref_patch) {
      const int base = rptr_off[k];
      for (int i = 0; i < pm[k]; ++i) {
        growptr[full_off[k] + i + 1] = rptr[base + i + 1] - rptr[base + i];
        for (int q = rptr[base + i]; q < rptr[base + i + 1]; ++q) gcol[q] = full_off[k] + rcol[q];
      }
    }
    for (size_t r = 0; r + 1 < growptr.size(); ++r) growptr[r + 1] += growptr[r];
    // rows were appended in the same order as the refined rows, so the
    // entries keep their order: growptr[full_off[k] + i] == rptr[rptr_off[k] + i]
    L.ref_nnz = (int)rcol.size();
    L.ref_lpr = pick_lpr(L.ref_nnz, full_off[np]);
    L.d_ref_growptr = dupload(growptr.data(), (int64_t)growptr.size(), own, st);
    L.d_ref_gcol = dupload(gcol.data(), (int64_t)gcol.size(), own, st);
    L.d_ref_src = dupload(rsrc.data(), (int64_t)rsrc.size(), own, st);
    L.bref = dalloc<float>(L.ref_nnz, own);
    L.gref = dalloc<float>(full_off[np], own);
    L.rhoref = dalloc<float>(full_off[np], own);
  }
  // extraction map: one slot per CSR entry of every block row
  if (L.boff_total >= ((int64_t)1 << 31))
    throw Error(FSI_E_INVALID, "the blocks of one level exceed 2^31 entries");
  if (!ilu_patch.empty()) {
    // each ILU block's pattern (J's stored entries in the block, and the
    // diagonal) as L and U rows of local columns, the L columns' row lists
    // and a bit mask; the factors' positions in the dense blocks
    std::vector<int> row0, lptr{0}, uptr{0}, cptr{0}, lpos, upos, dpos, flev, flev_off{0}, blev, blev_off{0};
    std::vector<int16_t> lcol, ucol, crow, frow, brow;
    std::vector<uint32_t> mask;
    std::vector<int64_t> moff;
    int maxe = 0, nrows = 0;
    for (int k : ilu_patch) {
      const int32_t *I = P.dof + P.ptr[k];
      const int m = pm[k];
      row0.push_back(nrows);
      moff.push_back((int64_t)mask.size());
      mask.resize(mask.size() + ((int64_t)m * m + 31) / 32, 0u);
      uint32_t *mk = mask.data() + moff.back();
      std::vector<std::vector<int16_t>> lcols(m);   // L's rows below each column
      const int l0 = (int)lcol.size(), u0 = (int)ucol.size();
      std::vector<int> row_cols, flevel(m, 0), blevel(m, 0);
      for (int i = 0; i < m; ++i) {
        row_cols.clear();
        row_cols.push_back(i);
        const int g = I[i];
        for (int64_t q = J.rowptr[g]; q < J.rowptr[g + 1]; ++q) {
          const int32_t *f = std::lower_bound(I, I + m, J.colind[q]);
          if (f != I + m && *f == J.colind[q]) row_cols.push_back((int)(f - I));
        }
        std::sort(row_cols.begin(), row_cols.end());
        row_cols.erase(std::unique(row_cols.begin(), row_cols.end()), row_cols.end());
        for (int c : row_cols) {
          const int64_t bit = (int64_t)i * m + c;
          mk[bit >> 5] |= 1u << (bit & 31);
          const int pos = (int)(L.h_boff[k] + (int64_t)i * m + c);
          if (c < i) {
            lcol.push_back((int16_t)c);
            lpos.push_back(pos);
            lcols[c].push_back((int16_t)i);
            flevel[i] = std::max(flevel[i], flevel[c] + 1);
          } else if (c > i) {
            ucol.push_back((int16_t)c);
            upos.push_back(pos);
          } else {
            dpos.push_back(pos);
          }
        }
        lptr.push_back((int)lcol.size());
        uptr.push_back((int)ucol.size());
      }
      // rows arrive in ascending order, so every column's list is sorted
      for (int c = 0; c < m; ++c) {
        crow.insert(crow.end(), lcols[c].begin(), lcols[c].end());
        cptr.push_back((int)crow.size());
      }
      // levels: a row's L columns lie in earlier forward levels, its U
      // columns in earlier backward levels
      for (int i = m - 1; i >= 0; --i)
        for (int q = uptr[nrows + i]; q < uptr[nrows + i + 1]; ++q)
          blevel[i] = std::max(blevel[i], blevel[ucol[q]] + 1);
      // the block's rows by level (its segment of frow/brow) and its level
      // starts as indices into that array; a block's last level ends where
      // the next block's first begins (a closing entry follows the last block)
      auto order = [&](const std::vector<int> &lev, std::vector<int16_t> &rows, std::vector<int> &ptr,
                       std::vector<int> &off) {
        const int nlev = m ? *std::max_element(lev.begin(), lev.end()) + 1 : 0;
        std::vector<int> cnt(nlev + 1, 0);
        for (int i = 0; i < m; ++i) ++cnt[lev[i] + 1];
        for (int t = 0; t < nlev; ++t) cnt[t + 1] += cnt[t];
        std::vector<int16_t> byl(m);
        std::vector<int> fill(cnt.begin(), cnt.end() - 1);
        for (int i = 0; i < m; ++i) byl[fill[lev[i]]++] = (int16_t)i;
        rows.insert(rows.end(), byl.begin(), byl.end());
        for (int t = 0; t < nlev; ++t) ptr.push_back(nrows + cnt[t]);
        off.push_back((int)ptr.size());
      };
      order(flevel, frow, flev, flev_off);
      order(blevel, brow, blev, blev_off);
      nrows += m;
      maxe = std::max(maxe, (int)std::max(lcol.size() - l0, ucol.size() - u0));
    }
    flev.push_back(nrows);
    blev.push_back(nrows);
    L.nilu = (int)ilu_patch.size();
    L.ilu_rows = nrows;
    L.ilu_nl = (int64_t)lcol.size();
    L.ilu_nu = (int64_t)ucol.size();
    L.ilu_max_entries = maxe;
    L.d_ilu_patch = dupload(ilu_patch.data(), (int64_t)ilu_patch.size(), own, st);
    L.d_ilu_row0 = dupload(row0.data(), (int64_t)row0.size(), own, st);
    L.d_ilu_lptr = dupload(lptr.data(), (int64_t)lptr.size(), own, st);
    L.d_ilu_uptr = dupload(uptr.data(), (int64_t)uptr.size(), own, st);
    L.d_ilu_cptr = dupload(cptr.data(), (int64_t)cptr.size(), own, st);
    L.d_ilu_lcol = dupload(lcol.data(), (int64_t)lcol.size(), own, st);
    L.d_ilu_ucol = dupload(ucol.data(), (int64_t)ucol.size(), own, st);
    L.d_ilu_crow = dupload(crow.data(), (int64_t)crow.size(), own, st);
    L.d_ilu_frow = dupload(frow.data(), (int64_t)frow.size(), own, st);
    L.d_ilu_brow = dupload(brow.data(), (int64_t)brow.size(), own, st);
    L.d_ilu_flev = dupload(flev.data(), (int64_t)flev.size(), own, st);
    L.d_ilu_blev = dupload(blev.data(), (int64_t)blev.size(), own, st);
    L.d_ilu_flev_off = dupload(flev_off.data(), (int64_t)flev_off.size(), own, st);
    L.d_ilu_blev_off = dupload(blev_off.data(), (int64_t)blev_off.size(), own, st);
    L.d_ilu_lpos = dupload(lpos.data(), (int64_t)lpos.size(), own, st);
    L.d_ilu_upos = dupload(upos.data(), (int64_t)upos.size(), own, st);
    L.d_ilu_dpos = dupload(dpos.data(), (int64_t)dpos.size(), own, st);
    L.d_ilu_mask = dupload(mask.data(), (int64_t)mask.size(), own, st);
    L.d_ilu_moff = dupload(moff.data(), (int64_t)moff.size(), own, st);
  }
  std::vector<int64_t> slot_off(row_patch.size() + 1, 0);
  for (size_t t = 0; t < row_patch.size(); ++t) {
    const int g = P.dof[pdof_off[row_patch[t]] + row_local[t]];
    slot_off[t + 1] = slot_off[t] + (J.rowptr[g + 1] - J.rowptr[g]);
  }
  L.ext_nslots = slot_off.back();
  L.d_ext_slot_off = dupload(slot_off.data(), (int64_t)slot_off.size(), own, st);
  L.d_ext_src = dalloc<int>(L.ext_nslots, own);
  L.d_ext_dst = dalloc<int>(L.ext_nslots, own);
  launch_extract_map(L.J.v64(), L.d_pm, L.d_pdof_off, L.d_dof, L.d_boff, (int64_t)row_patch.size(),
                     L.d_row_patch, L.d_row_local, L.d_ext_slot_off, L.d_ext_src, L.d_ext_dst, st);
  hip_check(hipGetLastError(), "extraction map");
}

// the solid blocks' FP32 owned-row launch (the main view's arrays, the solid task list)
static RasView ras_view_solid(const Level &L) {
  RasView v = ras_view(L);
  v.ntask = L.ntask_s;
  v.task_patch = L.d_task_patch_s;
  v.task_row0 = L.d_task_row0_s;
  v.cscale = nullptr;
  return v;
}
static RefineView refine_view(const Level &L) {
  RefineView v;
  v.ntask = L.nftask;
  v.w16_kind = L.w16_kind;
  v.lpr = L.ref_lpr;
  v.task_patch = L.d_ftask_patch;
  v.task_row0 = L.d_ftask_row0;
  v.pm = L.d_pm;
  v.dof = L.d_dof;
  v.full_off = L.d_full_off;
  v.own_dof = L.d_own_dof;
  v.pdof_off = L.d_pdof_off;
  v.woff_full = L.d_woff_full;
  v.B = CsrView<float>{(int)L.full_rows, (int)L.full_rows, L.ref_nnz, L.d_ref_growptr, L.d_ref_gcol, L.bref};
  v.gfull = L.gref;
  v.rho = L.rhoref;
  v.rscale = L.Wscale_full;
  v.cscale = L.Cscale;
  v.unowned = L.d_unowned;
  v.nunowned = L.n_unowned;
  return v;
}

static IluView ilu_view(const Level &L) {
  IluView v;
  v.nblk = L.nilu;
  v.patch = L.d_ilu_patch;
  v.row0 = L.d_ilu_row0;
  v.pm = L.d_pm;
  v.dof = L.d_dof;
  v.out_off = L.d_out_off;
  v.own_local = L.d_own_local;
  v.out_idx = L.d_out_idx;
  v.pdof_off = L.d_pdof_off;
  v.boff = L.d_boff;
  v.lptr = L.d_ilu_lptr;
  v.uptr = L.d_ilu_uptr;
  v.cptr = L.d_ilu_cptr;
  v.lcol = L.d_ilu_lcol;
  v.ucol = L.d_ilu_ucol;
  v.crow = L.d_ilu_crow;
  v.frow = L.d_ilu_frow;
  v.brow = L.d_ilu_brow;
  v.flev = L.d_ilu_flev;
  v.flev_off = L.d_ilu_flev_off;
  v.blev = L.d_ilu_blev;
  v.blev_off = L.d_ilu_blev_off;
  v.mask = L.d_ilu_mask;
  v.moff = L.d_ilu_moff;
  v.unowned = L.d_unowned;
  v.nunowned = L.n_unowned;
  v.max_entries = L.ilu_max_entries;
  return v;
}

// ILU(0) of the level's fluid blocks in the dense block scratch (after the
// batched inversion, which skips them), then the factors compacted
template <typename T>
static void ilu_factor_level(MG &mg, Level &L, int l, T *blocks, hipStream_t st) {
  if (!L.nilu) return;
  int base = 0;
  for (int q = 1; q < l; ++q) base += mg.lv[q].npatch;
  launch_ilu_factor<T>(ilu_view(L), blocks, mg.status, base, st);
  T *&lv = std::is_same<T, double>::value ? reinterpret_cast<T *&>(L.ilu_l64) : reinterpret_cast<T *&>(L.ilu_l32);
  T *&uv = std::is_same<T, double>::value ? reinterpret_cast<T *&>(L.ilu_u64) : reinterpret_cast<T *&>(L.ilu_u32);
  T *&dv = std::is_same<T, double>::value ? reinterpret_cast<T *&>(L.ilu_d64) : reinterpret_cast<T *&>(L.ilu_d32);
  if (!lv) {
    lv = dalloc<T>(std::max<int64_t>(L.ilu_nl, 1), mg.owned);
    uv = dalloc<T>(std::max<int64_t>(L.ilu_nu, 1), mg.owned);
    dv = dalloc<T>(std::max<int64_t>(L.ilu_rows, 1), mg.owned);
  }
  launch_ilu_gather<T, T>(blocks, L.d_ilu_lpos, L.ilu_nl, lv, st);
  launch_ilu_gather<T, T>(blocks, L.d_ilu_upos, L.ilu_nu, uv, st);
  launch_ilu_gather<T, T>(blocks, L.d_ilu_dpos, L.ilu_rows, dv, st);
  hip_check(hipGetLastError(), "ilu launch");
}

// the 16-bit owned rows' view: the grouped layout's offsets
static RasView ras_view16(const Level &L);

RasView ras_view(const Level &L) {
  RasView v;
  v.ntask = L.ntask;
  v.task_patch = L.d_task_patch;
  v.task_row0 = L.d_task_row0;
  v.pm = L.d_pm;
  v.po = L.d_po;
  v.pdof_off = L.d_pdof_off;
  v.woff = L.d_woff;
  v.dof = L.d_dof;
  v.out_off = L.d_out_off;
  v.out_idx = L.d_out_idx;
  v.cscale = L.Cscale;
  v.unowned = L.d_unowned;
  v.nunowned = L.n_unowned;
  v.mmax = L.mmax;
  return v;
}

static RasView ras_view16(const Level &L) {
  RasView v = ras_view(L);
  v.woff = L.d_woff16;
  return v;
}

static void free_list(DevList &owned) {
  while (!owned.v.empty()) free_one(owned, owned.v.size() - 1);
}

// owned rows of every block inverse in the storage precision of the level
// (the inverted blocks of level L sit at mg.blk_scratch + L.blk_base)
template <typename TB>
static void pack_level_t(MG &mg, Level &L, const TB *B, hipStream_t st) {
  const int prec = mg.opts.precision;
  if (prec == FSI_PREC_FP64) {
    if (!L.W64) L.W64 = dalloc<double>(L.woff_total, mg.owned);
  } else if (prec == FSI_PREC_MIXED_FP32) {
    if (!L.W32) L.W32 = dalloc<float>(L.woff_total, mg.owned);
  } else {
    if (!L.W16) {
      // the grouped layout's padding columns stay zero (the packer never writes them)
      L.W16 = dalloc<uint16_t>(std::max<int64_t>(L.woff16_total, 1), mg.owned);
      hip_check(hipMemsetAsync(L.W16, 0, sizeof(uint16_t) * std::max<int64_t>(L.woff16_total, 1), st),
                "clear 16-bit storage");
      L.Wscale = dalloc<float>(L.total_owned, mg.owned);
      L.Cscale = dalloc<float>(L.sum_m, mg.owned);
    }
    L.w16_kind = prec == FSI_PREC_MIXED_BF16 ? 1 : 2;
    // column scales of the owned rows, and of every row of the refined
    // blocks when they are kept in 16 bits (one scale array, disjoint columns)
    const bool full16 = L.nftask && mg.opts.solid_precision != FSI_PREC_MIXED_FP32;
    launch_colscale(B, L.d_boff, L.d_pm, L.d_po, L.d_out_off, L.d_own_local, L.d_pdof_off,
                    L.d_task_patch, L.d_task_row0, L.ntask, L.sum_m, L.Cscale, mg.gj_perm + L.pm_base,
                    L.mmax, st, true, !full16);
    if (full16)
      launch_colscale(B, L.d_boff, L.d_pm, L.d_po_full, L.d_full_off, L.d_full_local, L.d_pdof_off,
                      L.d_ftask_patch, L.d_ftask_row0, L.nftask, L.sum_m, L.Cscale,
                      mg.gj_perm + L.pm_base, L.mmax, st, false, true);
  }
  launch_pack_owned(B, L.d_boff, L.d_pm, L.d_po, L.d_woff, L.d_out_off, L.d_own_local,
                    L.d_task_patch, L.d_task_row0, L.ntask, L.W64, L.W32, L.W16, L.w16_kind,
                    L.Wscale, L.d_pdof_off, L.Cscale, mg.gj_perm + L.pm_base, L.d_woff16, st);
  if (L.ntask_s) {   // solid blocks' owned rows in FP32
    if (!L.Ws) L.Ws = dalloc<float>(L.woff_solid, mg.owned);
    launch_pack_owned(B, L.d_boff, L.d_pm, L.d_po, L.d_woff, L.d_out_off, L.d_own_local,
                      L.d_task_patch_s, L.d_task_row0_s, L.ntask_s, (double *)nullptr, L.Ws,
                      (uint16_t *)nullptr, 0, (float *)nullptr, L.d_pdof_off, (const float *)nullptr,
                      mg.gj_perm + L.pm_base, (const int64_t *)nullptr, st);
  }
  if (L.nftask) {    // refined solid blocks: every row of the inverse, FP32 or 16-bit
    const bool full16 = prec != FSI_PREC_MIXED_FP32 && mg.opts.solid_precision != FSI_PREC_MIXED_FP32;
    if (full16) {
      if (!L.Wfull16) {
        L.Wfull16 = dalloc<uint16_t>(L.wfull_total, mg.owned);
        L.Wscale_full = dalloc<float>(L.full_rows, mg.owned);
      }
    } else if (!L.Wfull32) {
      L.Wfull32 = dalloc<float>(L.wfull_total, mg.owned);
    }
    launch_pack_owned(B, L.d_boff, L.d_pm, L.d_po_full, L.d_woff_full, L.d_full_off, L.d_full_local,
                      L.d_ftask_patch, L.d_ftask_row0, L.nftask, (double *)nullptr, full16 ? nullptr : L.Wfull32,
                      full16 ? L.Wfull16 : nullptr, L.w16_kind, L.Wscale_full, L.d_pdof_off,
                      full16 ? L.Cscale : nullptr, mg.gj_perm + L.pm_base, (const int64_t *)nullptr, st);
  }
  hip_check(hipGetLastError(), "pack launch");
}

static void pack_level(MG &mg, Level &L, hipStream_t st) {
  if (mg.mixed)
    pack_level_t(mg, L, reinterpret_cast<const float *>(mg.blk_scratch) + L.blk_base, st);
  else
    pack_level_t(mg, L, mg.blk_scratch + L.blk_base, st);
}
// coarsest operator: dense copy, Gauss-Jordan inverse written column-major
// for the GEMV (no sync)
static void enqueue_coarse(MG &mg, Level &L, hipStream_t st) {
  const int nf = mg.coarse_nf;
  double *A = mg.dense_scratch;
  const CsrView<double> J = L.J.v64();
  if (nf > 0) {
    launch_fill_f64(A, (int64_t)nf * mg.dense_ld, 0.0, st);
    launch_csr_to_dense(J, mg.coarse_fpos, A, mg.dense_ld, st);
  }
  launch_fill_i32(mg.status0, 1, 0, st);   // a kernel, not a memset: this chain is graph-captured
  CoarseSplit cs;
  cs.n = L.n;
  cs.nd = mg.coarse_nd;
  cs.fpos = mg.coarse_fpos;
  cs.dlist = mg.coarse_dlist;
  cs.rowptr = J.rowptr;
  cs.val = J.val;
  gj_coarse(A, nf, mg.dense_ld, cs, L.C0, mg.status0, reinterpret_cast<int *>(mg.gj_work), st);
  hip_check(hipGetLastError(), "coarse launch");
}

// B_k = J_l[I_k, I_k] of every smoothing level into the setup scratch: FP64
// blocks, or FP32 working matrices for the mixed forms (the same element
// offsets, the buffer read as floats)
static void extract_blocks(MG &mg, hipStream_t st) {
  if (mg.mixed) {
    float *B = reinterpret_cast<float *>(mg.blk_scratch);
    launch_fill_f32(B, mg.blk_total, 0.0f, st);
    for (int l = 1; l < mg.nlevels; ++l) {
      Level &L = mg.lv[l];
      launch_extract(L.J.val, L.ext_nslots, L.d_ext_src, L.d_ext_dst, B + L.blk_base, st);
    }
  } else {
    launch_fill_f64(mg.blk_scratch, mg.blk_total, 0.0, st);
    for (int l = 1; l < mg.nlevels; ++l) {
      Level &L = mg.lv[l];
      launch_extract(L.J.val, L.ext_nslots, L.d_ext_src, L.d_ext_dst, mg.blk_scratch + L.blk_base, st);
    }
  }
}

// the batched Gauss-Jordan inversion of every block (FP64, or FP32 for the mixed forms)
static void invert_blocks(MG &mg, int variant, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (mg.mixed)
    launch_gj_batched_f32(reinterpret_cast<float *>(mg.blk_scratch), mg.all_boff, mg.all_pm, mg.all_poff,
                          mg.gj_perm, mg.gj_used, mg.npatch_all, mg.mmax_all, mg.status, mg.gj_grid,
                          mg.gj_sched, st, variant, ev0, ev1);
  else
    launch_gj_batched(mg.blk_scratch, mg.all_boff, mg.all_pm, mg.all_poff, mg.gj_perm, mg.gj_used,
                      mg.npatch_all, mg.mmax_all, mg.status, mg.gj_grid, mg.gj_sched, st, variant, ev0,
                      ev1);
}

// the blocks above kMaxPatch dofs, one after another: a padded FP64 copy,
// the Gauss-Jordan chain (the inverse written un-permuted, row-major, straight
// into the block, or through an FP64 buffer for the FP32 working matrices of
// the mixed forms), identity permutations for the packing.  Runs after the
// batched launch, which wrote these blocks' statuses as 0.
static void invert_large(MG &mg, hipStream_t st) {
  for (const LargeBlock &b : mg.large) {
    launch_fill_f64(mg.large_A, (int64_t)b.m * mg.large_ld, 0.0, st);
    if (mg.mixed)
      launch_copy_block(reinterpret_cast<const float *>(mg.blk_scratch) + b.boff, b.m, mg.large_A, mg.large_ld, st);
    else
      launch_copy_block(mg.blk_scratch + b.boff, b.m, mg.large_A, mg.large_ld, st);
    CoarseSplit cs;
    cs.n = b.m;
    cs.fpos = mg.large_iota;
    double *C = mg.mixed ? mg.large_C : mg.blk_scratch + b.boff;
    gj_coarse(mg.large_A, b.m, mg.large_ld, cs, C, mg.status + b.q, mg.large_iwork, st);
    if (mg.mixed)
      launch_cast_d2f(mg.large_C, reinterpret_cast<float *>(mg.blk_scratch) + b.boff, (int)((int64_t)b.m * b.m), st);
    launch_iota_i32(mg.gj_perm + b.poff, b.m, st);
    launch_iota_i32(mg.gj_used + b.poff, b.m, st);
  }
  hip_check(hipGetLastError(), "large block launch");
}

// next event pair of a profiling list (created on first use)
static hipEvent_t *prof_event_pair(std::vector<std::pair<hipEvent_t, hipEvent_t>> &evs, size_t &used) {
  if (used == evs.size()) {
    hipEvent_t a, b;
    hip_check(hipEventCreate(&a), "event");
    hip_check(hipEventCreate(&b), "event");
    evs.push_back({a, b});
  }
  return &evs[used++].first;
}

// setup of a1-a3 from the device-resident operator values.  The blocks of
// all smoothing levels are extracted and inverted in one launch on the main
// stream; the coarsest inversion (a chain of ~n/16 small launches, replayed
// from a graph captured at the first refactor) runs beside it on a second
// stream, on the compute units the batched launch leaves free.
void refactor(MG &mg, hipStream_t st) {
  if (!mg.dense_scratch) throw Error(FSI_E_INVALID, "setup scratch released; refactor unavailable");
  auto t0 = std::chrono::steady_clock::now();
  // the coarsest inversion needs only the coarsest operator.  Its chain goes
  // on the side stream after the main stream's (short) extraction launches
  // and before the batched inversion, so that it starts early while the
  // host's graph launch overlaps the extraction
  hip_check(hipEventRecord(mg.ev_fork, st), "fork");
  if (mg.mixed)
    for (int l = 1; l < mg.nlevels; ++l) {
      Level &L = mg.lv[l];
      launch_cast_d2f(L.J.val, L.J.val32, L.J.nnz, st);
      if (L.nref) launch_gather_f32(L.J.val32, L.d_ref_src, L.ref_nnz, L.bref, st);   // refined blocks' B_k
    }
  if (mg.nlevels > 1) extract_blocks(mg, st);
  hip_check(hipStreamWaitEvent(mg.side_stream, mg.ev_fork, 0), "fork wait");
  if (mg.opts.use_graph) {
    if (!mg.coarse_graph) {
      hipGraph_t g;
      hip_check(hipStreamBeginCapture(mg.side_stream, hipStreamCaptureModeThreadLocal), "begin capture");
      enqueue_coarse(mg, mg.lv[0], mg.side_stream);
      hip_check(hipStreamEndCapture(mg.side_stream, &g), "end capture");
      hip_check(hipGraphInstantiate(&mg.coarse_graph, g, nullptr, nullptr, 0), "instantiate");
      (void)hipGraphDestroy(g);
    }
    hip_check(hipGraphLaunch(mg.coarse_graph, mg.side_stream), "graph launch");
  } else {
    enqueue_coarse(mg, mg.lv[0], mg.side_stream);
  }
  hip_check(hipEventRecord(mg.ev_join, mg.side_stream), "join");
  if (mg.nlevels > 1) {
    hipEvent_t *ev = mg.prof_on ? prof_event_pair(mg.prof_gj_ev, mg.prof_gj_used) : nullptr;
    invert_blocks(mg, mg.gj_variant, st, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
    hip_check(hipGetLastError(), "gj launch");
    invert_large(mg, st);
    for (int l = 1; l < mg.nlevels; ++l) {
      pack_level(mg, mg.lv[l], st);
      if (mg.mixed)
        ilu_factor_level(mg, mg.lv[l], l, reinterpret_cast<float *>(mg.blk_scratch) + mg.lv[l].blk_base, st);
      else
        ilu_factor_level(mg, mg.lv[l], l, mg.blk_scratch + mg.lv[l].blk_base, st);
    }
  }
  hip_check(hipStreamWaitEvent(st, mg.ev_join, 0), "join wait");
  std::vector<int> hs(mg.npatch_all + 1, 0);
  hip_check(hipMemcpyAsync(hs.data(), mg.status, sizeof(int) * (mg.npatch_all + 1), hipMemcpyDeviceToHost, st),
            "D2H status");
  hip_check(hipStreamSynchronize(st), "refactor");
  if (hs[mg.npatch_all]) {
    char buf[160];
    snprintf(buf, sizeof buf, "level 0 (coarsest): zero or non-finite pivot at step %d", hs[mg.npatch_all] - 1);
    throw Error(FSI_E_SINGULAR, buf);
  }
  for (int q = 0; q < mg.npatch_all; ++q)
    if (hs[q]) {
      int l = 1, k = q;
      while (l < mg.nlevels - 1 && k >= mg.lv[l].npatch) k -= mg.lv[l++].npatch;
      char buf[160];
      snprintf(buf, sizeof buf, "level %d patch %d: zero or non-finite pivot at step %d", l, k, hs[q] - 1);
      throw Error(FSI_E_SINGULAR, buf);
    }
  mg.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ------------------------------------------------------------------ V-cycle
// event pair recorded at the finest-level Schwarz kernel's start and end while profiling
static hipEvent_t *prof_pair(MG &mg, Level &L) {
  if (!mg.prof_on || &L != &mg.lv.back()) return nullptr;
  if (mg.prof_used == mg.prof_ev.size()) {
    hipEvent_t a, b;
    hip_check(hipEventCreate(&a), "event");
    hip_check(hipEventCreate(&b), "event");
    mg.prof_ev.push_back({a, b});
  }
  return &mg.prof_ev[mg.prof_used++].first;
}
// one FP64 Schwarz application: the explicit inverses' owned rows, then the
// ILU blocks (which clear the unowned dofs when no explicit block is left)
static void ras64_omega(MG &mg, Level &L, const double *s, double *e, double omega, bool add, hipStream_t st) {
  hipEvent_t *ev = prof_pair(mg, L);
  launch_ras_f64(ras_view(L), L.W64, s, e, omega, &L == &mg.lv.back(), add, st, ev ? ev[0] : nullptr,
                 ev ? ev[1] : nullptr);
  if (L.nilu)
    launch_ilu_apply<double>(ilu_view(L), L.ilu_l64, L.ilu_u64, L.ilu_d64, s, e, omega, add, L.ntask == 0, st);
}
static void ras64(MG &mg, Level &L, const double *s, double *e, bool add, hipStream_t st) {
  ras64_omega(mg, L, s, e, mg.opts.omega, add, st);
}
static void ras32(MG &mg, Level &L, const float *s, float *e, bool add, hipStream_t st,
                  double omega_d = -1.0) {
  hipEvent_t *ev = prof_pair(mg, L);
  const float omega = (float)(omega_d > 0.0 ? omega_d : mg.opts.omega);
  if (L.W32)
    launch_ras_f32(ras_view(L), L.W32, s, e, omega, &L == &mg.lv.back(), add, st,
                   ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
  else
    launch_ras_16(ras_view16(L), L.W16, L.w16_kind, L.Wscale, s, e, omega,
                  &L == &mg.lv.back(), add, st, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr);
  // the solid blocks apart: FP32 owned rows, or refined local solves
  if (L.ntask_s) launch_ras_f32(ras_view_solid(L), L.Ws, s, e, omega, false, add, st);
  if (L.nref)
    launch_ras_refine(refine_view(L), L.Wfull32, L.Wfull16, s, e, omega, add, mg.opts.refine_sweeps, L.yref0,
                      L.yref1, st);
  if (L.nilu)
    launch_ilu_apply<float>(ilu_view(L), L.ilu_l32, L.ilu_u32, L.ilu_d32, s, e, omega, add, L.ntask == 0, st);
}

// One V-cycle on level l for e = M_l^{-1} r (r and e distinct; the finest
// level works on the caller's vectors directly).  The first smoothing step
// starts from e = 0: it stores its correction and clears the dofs no patch
// owns (no zero fill), and without pre-smoothing the coarse correction is
// stored into e.
template <typename T>
struct VOps;
template <>
struct VOps<double> {
  static CsrView<double> J(Level &L) { return L.J.v64(); }
  static CsrView<double> R(Level &L) { return L.R.v64(); }
  static CsrView<double> P(Level &L) { return L.P.v64(); }
  static double *r(Level &L) { return L.r; }
  static double *e(Level &L) { return L.e; }
  static double *s(Level &L) { return L.s; }
  static void ras(MG &mg, Level &L, const double *s, double *e, bool add, hipStream_t st) {
    ras64(mg, L, s, e, add, st);
  }
};
template <>
struct VOps<float> {
  static CsrView<float> J(Level &L) { return L.J.v32(); }
  static CsrView<float> R(Level &L) { return L.R.v32(); }
  static CsrView<float> P(Level &L) { return L.P.v32(); }
  static float *r(Level &L) { return L.r32; }
  static float *e(Level &L) { return L.e32; }
  static float *s(Level &L) { return L.s32; }
  static void ras(MG &mg, Level &L, const float *s, float *e, bool add, hipStream_t st) {
    ras32(mg, L, s, e, add, st);
  }
};

// the coarsest solve: FP64 dense inverse (the mixed cycle converts around it)
static void coarse_solve(MG &mg, const double *r, double *e, hipStream_t st) {
  Level &L = mg.lv[0];
  launch_dense_gemv(L.C0, L.n, r, e, st);
}
static void coarse_solve(MG &mg, const float *r, float *e, hipStream_t st) {
  Level &L = mg.lv[0];
  launch_cast_f2d(r, L.r, L.n, st);
  launch_dense_gemv(L.C0, L.n, L.r, L.e, st);
  launch_cast_d2f(L.e, e, L.n, st);
}

template <typename T>
static void vcycle(MG &mg, int l, const T *r, T *e, hipStream_t st) {
  using O = VOps<T>;
  if (l == 0) {
    coarse_solve(mg, r, e, st);
    return;
  }
  Level &L = mg.lv[l];
  Level &C = mg.lv[l - 1];
  const auto J = O::J(L);
  T *s = O::s(L);
  const int nu_pre = mg.opts.nu_pre;
  for (int it = 0; it < nu_pre; ++it) {
    if (it == 0) {
      O::ras(mg, L, r, e, false, st);
    } else {
      launch_spmv(J, e, r, s, kSpmvResid, L.J.lpr, st);
      O::ras(mg, L, s, e, true, st);
    }
  }
  if (nu_pre == 0) {
    launch_spmv(O::R(L), r, (const T *)nullptr, O::r(C), kSpmvSet, L.R.lpr, st);
  } else {
    launch_spmv(J, e, r, s, kSpmvResid, L.J.lpr, st);
    launch_spmv(O::R(L), s, (const T *)nullptr, O::r(C), kSpmvSet, L.R.lpr, st);
  }
  vcycle<T>(mg, l - 1, O::r(C), O::e(C), st);
  launch_spmv(O::P(L), O::e(C), (const T *)nullptr, e, nu_pre == 0 ? kSpmvSet : kSpmvAdd,
              L.P.lpr, st);
  for (int it = 0; it < mg.opts.nu_post; ++it) {
    launch_spmv(J, e, r, s, kSpmvResid, L.J.lpr, st);
    O::ras(mg, L, s, e, true, st);
  }
}

// z = M^{-1} r (device FP64 vectors of the finest size)
void apply_vcycle(MG &mg, const double *r, double *z, hipStream_t st) {
  Level &F = mg.lv.back();
  if (r == z) {
    launch_copy_f64(F.n, r, F.r, st);
    r = F.r;
  }
  if (mg.mixed && mg.nlevels > 1) {
    launch_cast_d2f(r, F.r32, F.n, st);
    vcycle<float>(mg, mg.nlevels - 1, F.r32, F.e32, st);
    launch_cast_f2d(F.e32, z, F.n, st);
  } else {
    vcycle<double>(mg, mg.nlevels - 1, r, z, st);
  }
}

// ------------------------------------------------------------------ batched V-cycles
// The V-cycles of several systems, phase by phase, each phase one batched
// launch over the systems that have it (a system with fewer levels reaches
// its coarsest solve at a smaller depth and then waits for the ascent).
// Every system sees the operations of vcycle() in the same order with the
// same kernels' arithmetic, so its result equals its own V-cycle's.
template <typename T>
struct BatchLevel {
  MG *mg;
  int l;
  const T *r;
  T *e;
};

template <typename T>
static CsrView<T> csr_view(const DevCsr &A);
template <>
CsrView<double> csr_view<double>(const DevCsr &A) {
  return A.v64();
}
template <>
CsrView<float> csr_view<float>(const DevCsr &A) {
  return A.v32();
}

// y = op x (Set), y = r - op x (Resid) or y += op x (Add) for every entry:
// op = 0 J, 1 R, 2 P of the entry's level
template <typename T>
static void batch_spmv(const std::vector<BatchLevel<T>> &a, int op, const std::vector<const T *> &x,
                       const std::vector<const T *> &r, const std::vector<T *> &y, int mode, hipStream_t st) {
  std::vector<SpmvItem<T>> it(a.size());
  std::vector<int> lpr(a.size());
  for (size_t i = 0; i < a.size(); ++i) {
    const Level &L = a[i].mg->lv[a[i].l];
    const DevCsr &A = op == 0 ? L.J : (op == 1 ? L.R : L.P);
    it[i] = SpmvItem<T>{csr_view<T>(A), x[i], r[i], y[i]};
    lpr[i] = A.lpr;
  }
  launch_spmv_batch<T>(it.data(), lpr.data(), (int)it.size(), mode, st);
}

static void batch_ras(const std::vector<BatchLevel<double>> &a, const std::vector<const double *> &s,
                      const std::vector<double *> &e, bool add, hipStream_t st) {
  std::vector<RasItem<double, double>> it;
  for (size_t i = 0; i < a.size(); ++i) {
    const Level &L = a[i].mg->lv[a[i].l];
    it.push_back(RasItem<double, double>{ras_view(L), L.W64, 0, nullptr, s[i], e[i]});
  }
  launch_ras_batch_f64(it.data(), (int)it.size(), a[0].mg->opts.omega, add, st);
  for (size_t i = 0; i < a.size(); ++i) {   // ILU blocks: their own launches
    const Level &L = a[i].mg->lv[a[i].l];
    if (L.nilu)
      launch_ilu_apply<double>(ilu_view(L), L.ilu_l64, L.ilu_u64, L.ilu_d64, s[i], e[i], a[0].mg->opts.omega,
                               add, L.ntask == 0, st);
  }
}
static void batch_ras(const std::vector<BatchLevel<float>> &a, const std::vector<const float *> &s,
                      const std::vector<float *> &e, bool add, hipStream_t st) {
  std::vector<RasItem<float, float>> i32;
  std::vector<RasItem<uint16_t, float>> i16;
  for (size_t i = 0; i < a.size(); ++i) {
    const Level &L = a[i].mg->lv[a[i].l];
    if (L.W32)
      i32.push_back(RasItem<float, float>{ras_view(L), L.W32, 0, nullptr, s[i], e[i]});
    else
      i16.push_back(RasItem<uint16_t, float>{ras_view16(L), L.W16, L.w16_kind, L.Wscale, s[i], e[i]});
  }
  const float omega = (float)a[0].mg->opts.omega;
  if (!i32.empty()) launch_ras_batch_f32(i32.data(), (int)i32.size(), omega, add, st);
  if (!i16.empty()) launch_ras_batch_16(i16.data(), (int)i16.size(), omega, add, st);
  // the solid blocks kept apart (FP32 owned rows, refined solves): their own
  // launches, on owned dofs disjoint from the batched ones
  for (size_t i = 0; i < a.size(); ++i) {
    MG &mg = *a[i].mg;
    Level &L = mg.lv[a[i].l];
    if (L.ntask_s) launch_ras_f32(ras_view_solid(L), L.Ws, s[i], e[i], omega, false, add, st);
    if (L.nref)
      launch_ras_refine(refine_view(L), L.Wfull32, L.Wfull16, s[i], e[i], omega, add, mg.opts.refine_sweeps,
                        L.yref0, L.yref1, st);
    if (L.nilu)
      launch_ilu_apply<float>(ilu_view(L), L.ilu_l32, L.ilu_u32, L.ilu_d32, s[i], e[i], omega, add, L.ntask == 0,
                              st);
  }
}

static void batch_coarse(const std::vector<BatchLevel<double>> &c, hipStream_t st) {
  std::vector<GemvItem> g;
  for (auto &b : c) g.push_back(GemvItem{b.mg->lv[0].C0, b.mg->lv[0].n, b.r, b.e});
  launch_dense_gemv_batch(g.data(), (int)g.size(), st);
}
static void batch_coarse(const std::vector<BatchLevel<float>> &c, hipStream_t st) {
  std::vector<CastItem<float, double>> up;
  std::vector<GemvItem> g;
  std::vector<CastItem<double, float>> down;
  for (auto &b : c) {
    Level &L = b.mg->lv[0];
    up.push_back(CastItem<float, double>{b.r, L.r, L.n});
    g.push_back(GemvItem{L.C0, L.n, L.r, L.e});
    down.push_back(CastItem<double, float>{L.e, b.e, L.n});
  }
  launch_cast_batch<float, double>(up.data(), (int)up.size(), st);
  launch_dense_gemv_batch(g.data(), (int)g.size(), st);
  launch_cast_batch<double, float>(down.data(), (int)down.size(), st);
}

template <typename T>
static void batch_vcycle_levels(const std::vector<BatchLevel<T>> &cur, hipStream_t st) {
  using O = VOps<T>;
  std::vector<BatchLevel<T>> a, c;
  for (auto &b : cur) (b.l == 0 ? c : a).push_back(b);
  if (!c.empty()) batch_coarse(c, st);
  if (a.empty()) return;
  const int nu_pre = a[0].mg->opts.nu_pre, nu_post = a[0].mg->opts.nu_post;
  const size_t n = a.size();
  std::vector<const T *> r(n), sc(n), none(n, nullptr), ce_c(n);
  std::vector<T *> e(n), sv(n), cr(n);
  std::vector<BatchLevel<T>> next(n);
  for (size_t i = 0; i < n; ++i) {
    Level &L = a[i].mg->lv[a[i].l];
    Level &C = a[i].mg->lv[a[i].l - 1];
    r[i] = a[i].r;
    e[i] = a[i].e;
    sv[i] = O::s(L);
    sc[i] = O::s(L);
    cr[i] = O::r(C);
    ce_c[i] = O::e(C);
    next[i] = BatchLevel<T>{a[i].mg, a[i].l - 1, O::r(C), O::e(C)};
  }
  std::vector<const T *> e_c(e.begin(), e.end());
  for (int it = 0; it < nu_pre; ++it) {
    if (it == 0) {
      batch_ras(a, r, e, false, st);
    } else {
      batch_spmv<T>(a, 0, e_c, r, sv, kSpmvResid, st);
      batch_ras(a, sc, e, true, st);
    }
  }
  if (nu_pre == 0) {
    batch_spmv<T>(a, 1, r, none, cr, kSpmvSet, st);
  } else {
    batch_spmv<T>(a, 0, e_c, r, sv, kSpmvResid, st);
    batch_spmv<T>(a, 1, sc, none, cr, kSpmvSet, st);
  }
  batch_vcycle_levels<T>(next, st);
  batch_spmv<T>(a, 2, ce_c, none, e, nu_pre == 0 ? kSpmvSet : kSpmvAdd, st);
  for (int it = 0; it < nu_post; ++it) {
    batch_spmv<T>(a, 0, e_c, r, sv, kSpmvResid, st);
    batch_ras(a, sc, e, true, st);
  }
}

bool batch_compatible(const MG &a, const MG &b) {
  const bool fa = a.mixed && a.nlevels > 1, fb = b.mixed && b.nlevels > 1;
  return fa == fb && a.opts.nu_pre == b.opts.nu_pre && a.opts.nu_post == b.opts.nu_post &&
         a.opts.omega == b.opts.omega;
}

void batched_vcycle(const std::vector<BatchItem> &items, hipStream_t st) {
  if (items.empty()) return;
  for (size_t i = 0; i < items.size(); ++i) {
    const BatchItem &b = items[i];
    if (b.r == b.z || !batch_compatible(*b.mg, *items[0].mg))
      throw Error(FSI_E_INVALID, "batched V-cycle: aliased vectors or incompatible systems");
    for (size_t k = 0; k < i; ++k)   // one entry per system: its level vectors are the cycle's workspace
      if (items[k].mg == b.mg) throw Error(FSI_E_INVALID, "batched V-cycle: a system appears twice");
  }
  if (items[0].mg->mixed && items[0].mg->nlevels > 1) {
    std::vector<CastItem<double, float>> in;
    std::vector<CastItem<float, double>> out;
    std::vector<BatchLevel<float>> lv;
    for (auto &b : items) {
      Level &F = b.mg->lv.back();
      in.push_back(CastItem<double, float>{b.r, F.r32, F.n});
      out.push_back(CastItem<float, double>{F.e32, b.z, F.n});
      lv.push_back(BatchLevel<float>{b.mg, b.mg->nlevels - 1, F.r32, F.e32});
    }
    launch_cast_batch<double, float>(in.data(), (int)in.size(), st);
    batch_vcycle_levels<float>(lv, st);
    launch_cast_batch<float, double>(out.data(), (int)out.size(), st);
  } else {
    std::vector<BatchLevel<double>> lv;
    for (auto &b : items) lv.push_back(BatchLevel<double>{b.mg, b.mg->nlevels - 1, b.r, b.z});
    batch_vcycle_levels<double>(lv, st);
  }
  hip_check(hipGetLastError(), "batched V-cycle launch");
}

void run_vcycle(MG &mg, const double *r, double *z, hipStream_t st) {
  if (mg.opts.use_graph && !mg.prof_on) {
    // one graph per (input, output) pair; the Krylov loop reuses a small set of pairs
    GraphKey key{r, z};
    auto it = mg.graphs.find(key);
    if (it == mg.graphs.end()) {
      hipGraph_t g;
      hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
      apply_vcycle(mg, r, z, st);
      hip_check(hipStreamEndCapture(st, &g), "end capture");
      hipGraphExec_t ex;
      hip_check(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "instantiate");
      (void)hipGraphDestroy(g);
      it = mg.graphs.emplace(key, ex).first;
    }
    hip_check(hipGraphLaunch(it->second, st), "graph launch");
  } else {
    apply_vcycle(mg, r, z, st);
  }
}

// ------------------------------------------------------------------ Galerkin product on the device
// Section "Geometric Multigrid preconditioner": the coarse operators are the
// Galerkin products J_{l-1} = R_l J_l P_l.  The first call reads the
// patterns back and builds T_l = J_l P_l's pattern on the host, checks that
// R_l T_l's pattern lies in the given J_{l-1}'s, and finds the positions of
// J_{l-1}'s Dirichlet diagonals (the input flags, else the rows whose only
// entry is a unit diagonal); then every call is two products per level on
// the device, finest first, and a unit added on the Dirichlet diagonals
// (whose rows and columns R and P leave empty), as the coarse operators were
// formed.
template <typename T>
static std::vector<T> d2h(const T *d, int64_t n) {
  std::vector<T> h(std::max<int64_t>(n, 0));
  if (n > 0) hip_check(hipMemcpy(h.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost), "D2H");
  return h;
}
static void galerkin_prepare(MG &mg, hipStream_t st) {
  hip_check(hipStreamSynchronize(st), "galerkin");
  for (int l = mg.nlevels - 1; l >= 1; --l) {
    Level &L = mg.lv[l], &C = mg.lv[l - 1];
    const auto jrp = d2h(L.J.rowptr, L.n + 1), jc = d2h(L.J.col, L.J.nnz);
    const auto prp = d2h(L.P.rowptr, L.P.n + 1), pc = d2h(L.P.col, L.P.nnz);
    const auto rrp = d2h(L.R.rowptr, L.R.n + 1), rc = d2h(L.R.col, L.R.nnz);
    const auto crp = d2h(C.J.rowptr, C.n + 1), cc = d2h(C.J.col, C.J.nnz);
    // T = J P: union of P's rows over each J row
    std::vector<int> trp(L.n + 1, 0), tcol, mark(C.n, -1), list;
    for (int i = 0; i < L.n; ++i) {
      list.clear();
      for (int p = jrp[i]; p < jrp[i + 1]; ++p)
        for (int q = prp[jc[p]]; q < prp[jc[p] + 1]; ++q)
          if (mark[pc[q]] != i) {
            mark[pc[q]] = i;
            list.push_back(pc[q]);
          }
      std::sort(list.begin(), list.end());
      tcol.insert(tcol.end(), list.begin(), list.end());
      trp[i + 1] = (int)tcol.size();
    }
    // R T must land on the given coarse pattern
    std::fill(mark.begin(), mark.end(), -1);
    for (int r = 0; r < C.n; ++r) {
      for (int p = crp[r]; p < crp[r + 1]; ++p) mark[cc[p]] = r;
      for (int p = rrp[r]; p < rrp[r + 1]; ++p)
        for (int q = trp[rc[p]]; q < trp[rc[p] + 1]; ++q)
          if (mark[tcol[q]] != r) {
            char buf[160];
            snprintf(buf, sizeof buf, "level %d: R J P has an entry (%d, %d) outside the given coarse operator",
                     l - 1, r, tcol[q]);
            throw Error(FSI_E_INVALID, buf);
          }
    }
    // the coarse level's Dirichlet diagonals
    std::vector<int> dir = C.h_dir;
    if (!C.dir_known) {
      const auto cv = d2h(C.J.val, C.J.nnz);
      for (int r = 0; r < C.n; ++r)
        if (crp[r + 1] - crp[r] == 1 && cc[crp[r]] == r && cv[crp[r]] == 1.0) dir.push_back(r);
    }
    std::vector<int> pos;
    for (int r : dir) {
      const int *f = std::lower_bound(cc.data() + crp[r], cc.data() + crp[r + 1], r);
      if (f == cc.data() + crp[r + 1] || *f != r)
        throw Error(FSI_E_INVALID, "a Dirichlet row of a coarse operator holds no diagonal");
      pos.push_back((int)(f - cc.data()));
    }
    // the terms of every entry of T = J P, in the order a row-by-column product
    // sums them (ascending entries of J's row), then those of R T
    const auto pv = d2h(L.P.val, L.P.nnz), rv = d2h(L.R.val, L.R.nnz);
    std::vector<int> tpos(C.n, -1);
    std::vector<int> gt_ptr(tcol.size() + 1, 0), gt_idx;
    std::vector<double> gt_w;
    for (int i = 0; i < L.n; ++i) {
      for (int q = trp[i]; q < trp[i + 1]; ++q) tpos[tcol[q]] = q;
      for (int p = jrp[i]; p < jrp[i + 1]; ++p)
        for (int q = prp[jc[p]]; q < prp[jc[p] + 1]; ++q) ++gt_ptr[tpos[pc[q]] + 1];
    }
    for (size_t q = 0; q < tcol.size(); ++q) gt_ptr[q + 1] += gt_ptr[q];
    gt_idx.resize(gt_ptr.back());
    gt_w.resize(gt_ptr.back());
    {
      std::vector<int> fill(gt_ptr.begin(), gt_ptr.end() - 1);
      for (int i = 0; i < L.n; ++i) {
        for (int q = trp[i]; q < trp[i + 1]; ++q) tpos[tcol[q]] = q;
        for (int p = jrp[i]; p < jrp[i + 1]; ++p)
          for (int q = prp[jc[p]]; q < prp[jc[p] + 1]; ++q) {
            const int t = fill[tpos[pc[q]]]++;
            gt_idx[t] = p;
            gt_w[t] = pv[q];
          }
      }
    }
    std::vector<int> cpos(C.n, -1), gc_ptr(C.J.nnz + 1, 0), gc_idx;
    std::vector<double> gc_w;
    for (int r = 0; r < C.n; ++r) {
      for (int q = crp[r]; q < crp[r + 1]; ++q) cpos[cc[q]] = q;
      for (int p = rrp[r]; p < rrp[r + 1]; ++p)
        for (int q = trp[rc[p]]; q < trp[rc[p] + 1]; ++q) ++gc_ptr[cpos[tcol[q]] + 1];
    }
    for (int64_t q = 0; q < C.J.nnz; ++q) gc_ptr[q + 1] += gc_ptr[q];
    gc_idx.resize(gc_ptr.back());
    gc_w.resize(gc_ptr.back());
    {
      std::vector<int> fill(gc_ptr.begin(), gc_ptr.end() - 1);
      for (int r = 0; r < C.n; ++r) {
        for (int q = crp[r]; q < crp[r + 1]; ++q) cpos[cc[q]] = q;
        for (int p = rrp[r]; p < rrp[r + 1]; ++p)
          for (int q = trp[rc[p]]; q < trp[rc[p] + 1]; ++q) {
            const int t = fill[cpos[tcol[q]]]++;
            gc_idx[t] = q;
            gc_w[t] = rv[p];
          }
      }
    }
    L.gt_n = (int64_t)tcol.size();
    L.gc_n = C.J.nnz;
    L.d_gt_ptr = dupload(gt_ptr.data(), (int64_t)gt_ptr.size(), mg.owned, st);
    L.d_gt_idx = dupload(gt_idx.data(), std::max<int64_t>((int64_t)gt_idx.size(), 1), mg.owned, st);
    L.d_gt_w = dupload(gt_w.data(), std::max<int64_t>((int64_t)gt_w.size(), 1), mg.owned, st);
    L.d_gc_ptr = dupload(gc_ptr.data(), (int64_t)gc_ptr.size(), mg.owned, st);
    L.d_gc_idx = dupload(gc_idx.data(), std::max<int64_t>((int64_t)gc_idx.size(), 1), mg.owned, st);
    L.d_gc_w = dupload(gc_w.data(), std::max<int64_t>((int64_t)gc_w.size(), 1), mg.owned, st);
    L.d_t_val = dalloc<double>(std::max<int64_t>((int64_t)tcol.size(), 1), mg.owned);
    L.d_cdir_pos = dupload(pos.data(), (int64_t)pos.size(), mg.owned, st);
    L.n_cdir = (int)pos.size();
  }
  stage_drain();
  mg.galerkin_ready = true;
}

void galerkin(MG &mg, hipStream_t st) {
  if (!mg.galerkin_ready) galerkin_prepare(mg, st);
  for (int l = mg.nlevels - 1; l >= 1; --l) {
    Level &L = mg.lv[l], &C = mg.lv[l - 1];
    launch_gather_dot((int)L.gt_n, L.d_gt_ptr, L.d_gt_idx, L.d_gt_w, L.J.val, L.d_t_val, st);
    launch_gather_dot((int)L.gc_n, L.d_gc_ptr, L.d_gc_idx, L.d_gc_w, L.d_t_val, C.J.val, st);
    launch_add_at(C.J.val, L.d_cdir_pos, L.n_cdir, 1.0, st);
  }
  hip_check(hipGetLastError(), "galerkin launch");
}

// ------------------------------------------------------------------ setup
void alloc_level_vectors(MG &mg, Level &L) {
  L.r = dalloc<double>(L.n, mg.owned);
  L.e = dalloc<double>(L.n, mg.owned);
  L.s = dalloc<double>(L.n, mg.owned);
  if (mg.mixed) {
    L.r32 = dalloc<float>(L.n, mg.owned);
    L.e32 = dalloc<float>(L.n, mg.owned);
    L.s32 = dalloc<float>(L.n, mg.owned);
  }
}

static void validate_opts(const fsi_mg_opts *opts) {
  if (!opts) throw Error(FSI_E_INVALID, "no options");
  if (opts->nu_pre < 0 || opts->nu_post < 0 || !(opts->omega > 0.0) ||
      opts->precision < FSI_PREC_FP64 || opts->precision > FSI_PREC_MIXED_FP32)
    throw Error(FSI_E_INVALID, "invalid multigrid options");
  const bool mixed = opts->precision != FSI_PREC_FP64;
  if (opts->solid_precision != -1 && opts->solid_precision != opts->precision &&
      !(mixed && opts->solid_precision == FSI_PREC_MIXED_FP32))
    throw Error(FSI_E_INVALID,
                "solid_precision must be -1, equal to precision, or FSI_PREC_MIXED_FP32 in a mixed hierarchy");
  if (opts->refine_sweeps < 0 || opts->refine_sweeps > 4 || (opts->refine_sweeps > 0 && !mixed))
    throw Error(FSI_E_INVALID, "refine_sweeps must be 0..4, and 0 for an FP64 hierarchy");
  if (opts->fluid_ilu != 0 && opts->fluid_ilu != 1) throw Error(FSI_E_INVALID, "fluid_ilu must be 0 or 1");
}

static void validate_hierarchy(const fsi_level *levels, int nlevels, const std::vector<int64_t> &n) {
  for (int l = 0; l < nlevels; ++l) {
    if (n[l] < 1) throw Error(FSI_E_INVALID, "empty level");
    validate_csr(levels[l].J, n[l], n[l], "J", l);
    if (l > 0) {
      validate_csr(levels[l].P, n[l], n[l - 1], "P", l);
      validate_csr(levels[l].R, n[l - 1], n[l], "R", l);
      validate_patches(levels[l].patches, n[l], l);
    }
    if (levels[l].dirichlet) validate_dirichlet(levels[l], n[l], l);
  }
}

// The checks a server's submit makes before estimating the footprint and
// copying: options, dimensions across levels, CSR row offsets (monotone,
// spanning nnz) and patch offsets and dofs in range.  O(n + sum of patch
// sizes); the entries themselves are checked by validate_levels at setup.
// blocks above kMaxPatch dofs are inverted whole by the Gauss-Jordan chain;
// the ILU(0) factorization and the refinement sweeps keep the smaller limit
static void validate_large_blocks(const fsi_level *levels, int nlevels, const fsi_mg_opts &o) {
  const bool refine = solid_split(o) && o.refine_sweeps > 0;
  for (int l = 1; l < nlevels; ++l) {
    const fsi_patches &P = levels[l].patches;
    for (int k = 0; k < P.npatch; ++k) {
      if (P.ptr[k + 1] - P.ptr[k] <= kMaxPatch) continue;
      const int kind = P.kind ? P.kind[k] : 0;
      const char *why = (o.fluid_ilu && kind == 0) ? "an ILU(0) block" : (refine && kind == 1) ? "a refined block" : nullptr;
      if (why) {
        char buf[200];
        snprintf(buf, sizeof buf, "level %d patch %d: %s of %lld dofs; at most %d", l, k, why,
                 (long long)(P.ptr[k + 1] - P.ptr[k]), kMaxPatch);
        throw Error(FSI_E_INVALID, buf);
      }
    }
  }
}

void validate_levels_light(const fsi_level *levels, int nlevels, const fsi_mg_opts *opts) {
  if (!levels || nlevels < 1) throw Error(FSI_E_INVALID, "no levels");
  validate_opts(opts);
  auto rows = [&](const fsi_csr &A, int64_t nr, int64_t nc, const char *name, int l) {
    char buf[200];
    if (A.nrows != nr || A.ncols != nc || A.nnz < 0 || A.nnz >= ((int64_t)1 << 31) || !A.rowptr ||
        (A.nnz > 0 && (!A.colind || !A.val)) || A.rowptr[0] != 0 || A.rowptr[A.nrows] != A.nnz) {
      snprintf(buf, sizeof buf, "level %d %s: dimensions, arrays or row offsets invalid", l, name);
      throw Error(FSI_E_INVALID, buf);
    }
    for (int64_t r = 0; r < A.nrows; ++r)
      if (A.rowptr[r + 1] < A.rowptr[r]) {
        snprintf(buf, sizeof buf, "level %d %s: row offsets not monotone", l, name);
        throw Error(FSI_E_INVALID, buf);
      }
  };
  for (int l = 0; l < nlevels; ++l) {
    const int64_t n = levels[l].J.nrows;
    if (n < 1) throw Error(FSI_E_INVALID, "empty level");
    if (l == 0 && n > kMaxCoarse) throw Error(FSI_E_INVALID, "coarsest level too large for the direct solve");
    rows(levels[l].J, n, n, "J", l);
    if (l == 0) continue;
    const int64_t nc = levels[l - 1].J.nrows;
    rows(levels[l].P, n, nc, "P", l);
    rows(levels[l].R, nc, n, "R", l);
    const fsi_patches &P = levels[l].patches;
    if (P.npatch <= 0 || !P.ptr || !P.dof || !P.owned || P.ptr[0] != 0)
      throw Error(FSI_E_INVALID, "patches missing or malformed");
    for (int k = 0; k < P.npatch; ++k)
      if (P.ptr[k + 1] <= P.ptr[k] || P.ptr[k + 1] - P.ptr[k] > kMaxLargePatch)
        throw Error(FSI_E_INVALID, "patch offsets invalid or a patch larger than the supported block size");
    for (int64_t p = 0; p < P.ptr[P.npatch]; ++p)
      if (P.dof[p] < 0 || P.dof[p] >= n) throw Error(FSI_E_INVALID, "patch dof out of range");
  }
}

// host-side checks of the whole hierarchy (no device call)
void validate_levels(const fsi_level *levels, int nlevels, const fsi_mg_opts *opts) {
  if (!levels || nlevels < 1) throw Error(FSI_E_INVALID, "no levels");
  validate_opts(opts);
  std::vector<int64_t> n(nlevels);
  for (int l = 0; l < nlevels; ++l) n[l] = levels[l].J.nrows;
  if (n[0] > kMaxCoarse) {
    char buf[160];
    snprintf(buf, sizeof buf, "coarsest level has %lld unknowns; the dense direct solve takes at most %d",
             (long long)n[0], kMaxCoarse);
    throw Error(FSI_E_INVALID, buf);
  }
  validate_hierarchy(levels, nlevels, n);
  validate_large_blocks(levels, nlevels, *opts);
}


int autotune(MG &mg, const char *db_path, hipStream_t st);

MG *mg_setup(const fsi_level *levels, int nlevels, const fsi_mg_opts *opts, hipStream_t user_st,
             hipStream_t own_st, DevicePool *pool, hipStream_t side_st) {
  auto t0 = std::chrono::steady_clock::now();
  validate_levels(levels, nlevels, opts);
  std::vector<int64_t> n(nlevels);
  for (int l = 0; l < nlevels; ++l) n[l] = levels[l].J.nrows;
  MG *mg = new MG();
  mg->opts = *opts;
  mg->nlevels = nlevels;
  hip_check(hipGetDevice(&mg->device), "device");
  mg->mixed = opts->precision != FSI_PREC_FP64;
  mg->own_stream = own_st;
  mg->owned.pool = pool;
  mg->kry.owned.pool = pool;
  hipStream_t st = user_st ? user_st : own_st;
  try {
    mg->lv.resize(nlevels);
    for (int l = 0; l < nlevels; ++l) {
      Level &L = mg->lv[l];
      L.n = (int)n[l];
      upload_csr(levels[l].J, L.J, mg->mixed && l > 0, mg->owned, st);
      if (l > 0) {
        upload_csr(levels[l].P, L.P, mg->mixed, mg->owned, st);
        upload_csr(levels[l].R, L.R, mg->mixed, mg->owned, st);
        build_patch_layout(L, levels[l].patches, levels[l].J, *mg, st);
      }
      alloc_level_vectors(*mg, L);
      if (levels[l].dirichlet) {
        L.dir_known = true;
        for (int64_t i = 0; i < n[l]; ++i)
          if (levels[l].dirichlet[i]) L.h_dir.push_back((int)i);
      }
    }
    // all levels' blocks in one scratch; one offset/size table for the batched inversion
    std::vector<int64_t> all_boff, all_poff;
    std::vector<int> all_pm;
    int64_t base = 0, pbase = 0;
    mg->mmax_all = 1;
    for (int l = 1; l < nlevels; ++l) {
      Level &L = mg->lv[l];
      L.blk_base = base;
      L.pm_base = pbase;
      for (int k = 0; k < L.npatch; ++k) {
        all_boff.push_back(base + L.h_boff[k]);
        all_poff.push_back(pbase + L.h_ptr[k]);
        // an ILU block is factored apart, a block above kMaxPatch dofs is
        // inverted on its own: no work in the batched launch (size 0)
        const bool is_ilu = mg->opts.fluid_ilu && L.h_kind[k] == 0;
        const int m = (int)(L.h_ptr[k + 1] - L.h_ptr[k]);
        if (!is_ilu && m > kMaxPatch) {
          mg->large.push_back(LargeBlock{(int)all_pm.size(), m, base + L.h_boff[k], pbase + L.h_ptr[k]});
          mg->large_mmax = std::max(mg->large_mmax, m);
        }
        all_pm.push_back(is_ilu || m > kMaxPatch ? 0 : m);
        mg->mmax_all = std::max(mg->mmax_all, all_pm.back());
      }
      base += L.boff_total;
      pbase += L.sum_m;
    }
    mg->blk_total = base;
    mg->npatch_all = (int)all_pm.size();
    const int64_t n0 = mg->lv[0].n;
    // + 64: the batched inversion loads each panel slice whole from its row base
    mg->blk_scratch = dalloc<double>(base + 64, mg->owned);
    mg->all_boff = dupload(all_boff.data(), (int64_t)all_boff.size(), mg->owned, st);
    mg->all_pm = dupload(all_pm.data(), (int64_t)all_pm.size(), mg->owned, st);
    mg->all_poff = dupload(all_poff.data(), (int64_t)all_poff.size(), mg->owned, st);
    if (mg->npatch_all) {
      // room for the schedule of any grid up to one workgroup per block
      mg->h_all_pm = all_pm;
      mg->gj_grid = gj_batched_grid(mg->npatch_all);
      const std::vector<int> sched = gj_schedule(all_pm.data(), mg->npatch_all, mg->gj_grid);
      mg->gj_sched = dalloc<int>(2 * (int64_t)mg->npatch_all + 1, mg->owned);
      stage_copy(mg->gj_sched, sched.data(), sizeof(int) * sched.size(), st);
    }
    mg->gj_perm = dalloc<int>(std::max<int64_t>(pbase, 1), mg->owned);
    mg->gj_used = dalloc<int>(std::max<int64_t>(pbase, 1), mg->owned);
    // the blocks' statuses, then the coarsest operator's (one read-back)
    mg->status = dalloc<int>(mg->npatch_all + 1, mg->owned);
    mg->status0 = mg->status + mg->npatch_all;
    // coarsest operator: the dofs whose row and column hold only the
    // diagonal (D) are inverted by a reciprocal, the rest (F) densely
    {
      const fsi_csr &J0 = levels[0].J;
      std::vector<int> colcnt(n0, 0), fpos(n0, -1), dlist;
      for (int64_t p = 0; p < J0.nnz; ++p) ++colcnt[J0.colind[p]];
      int nf = 0;
      for (int64_t i = 0; i < n0; ++i) {
        const bool diag_only = J0.rowptr[i + 1] - J0.rowptr[i] == 1 && J0.colind[J0.rowptr[i]] == i &&
                               colcnt[i] == 1;
        if (diag_only)
          dlist.push_back((int)i);
        else
          fpos[i] = nf++;
      }
      mg->coarse_nf = nf;
      mg->coarse_nd = (int)dlist.size();
      mg->coarse_fpos = dupload(fpos.data(), n0, mg->owned, st);
      mg->coarse_dlist = dupload(dlist.data(), (int64_t)dlist.size(), mg->owned, st);
    }
    if (!mg->large.empty()) {
      // the chain's working copy: rows padded to a multiple of 16 doubles, + 64 past the end
      mg->large_ld = (mg->large_mmax + 15) / 16 * 16;
      mg->large_A = dalloc<double>((int64_t)mg->large_mmax * mg->large_ld + 64, mg->owned);
      if (mg->mixed) mg->large_C = dalloc<double>((int64_t)mg->large_mmax * mg->large_mmax, mg->owned);
      mg->large_iota = dalloc<int>(mg->large_mmax, mg->owned);
      launch_iota_i32(mg->large_iota, mg->large_mmax, st);
      mg->large_iwork = dalloc<int>(2 * (int64_t)mg->large_mmax + 64, mg->owned);
    }
    mg->dense_ld = (std::max(mg->coarse_nf, 1) + 15) / 16 * 16;
    mg->dense_scratch = dalloc<double>(std::max(mg->coarse_nf, 1) * mg->dense_ld, mg->owned);
    mg->gj_work = dalloc<double>(n0 + 64, mg->owned);
    mg->lv[0].C0 = dalloc<double>(n0 * n0, mg->owned);
    if (side_st) {
      mg->side_stream = side_st;
      mg->own_side = false;
    } else {
      hip_check(hipStreamCreateWithFlags(&mg->side_stream, hipStreamNonBlocking), "side stream");
    }
    hip_check(hipEventCreateWithFlags(&mg->ev_fork, hipEventDisableTiming), "event");
    hip_check(hipEventCreateWithFlags(&mg->ev_join, hipEventDisableTiming), "event");
    // the solve's host-coherent result slot and its event, taken here so that
    // fsi_fgmres_solve_noalloc allocates nothing; the static workspace's
    // address on this device (the device is current here)
    mg->kry.pinned = pinned_slot_acquire();
    hip_check(hipHostGetDevicePointer((void **)&mg->kry.pinned_dev, mg->kry.pinned, 0), "pinned address");
    hip_check(hipEventCreateWithFlags(&mg->kry.ev_done, hipEventDisableTiming), "event");
    mg->static_ws = scratch_address(mg->device);
    stage_drain();   // the uploads are complete and the staging buffer is free again
    hip_check(hipStreamSynchronize(st), "upload");
    refactor(*mg, st);
    if (opts->tuning_db) autotune(*mg, opts->tuning_db, st);
    mg->opts.tuning_db = nullptr;   // borrowed for the call only
  } catch (...) {
    try {
      stage_drain();   // no copy may still write into memory about to be released
    } catch (...) {
    }
    destroy_mg(mg);
    throw;
  }
  mg->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return mg;
}

// frees the setup scratch (dense blocks, coarse dense matrix); a later
// refactor is then refused.  Used by the server once a system is set up.
void release_setup_scratch(MG &mg) {
  auto drop = [&](void *p) {
    if (!p) return;
    for (size_t i = 0; i < mg.owned.v.size(); ++i)
      if (mg.owned.v[i].first == p) {
        free_one(mg.owned, i);
        return;
      }
  };
  drop(mg.blk_scratch);
  drop(mg.dense_scratch);
  mg.blk_scratch = nullptr;
  mg.dense_scratch = nullptr;
  for (Level &L : mg.lv) {
    drop(L.d_ext_src);
    drop(L.d_ext_dst);
    drop(L.d_ext_slot_off);
    L.d_ext_src = L.d_ext_dst = nullptr;
    L.d_ext_slot_off = nullptr;
  }
}

void destroy_mg(MG *mg) {
  if (!mg) return;
  if (mg->side_stream) {
    (void)hipStreamSynchronize(mg->side_stream);
    if (mg->own_side) (void)hipStreamDestroy(mg->side_stream);
  }
  if (mg->coarse_graph) (void)hipGraphExecDestroy(mg->coarse_graph);
  if (mg->ev_fork) (void)hipEventDestroy(mg->ev_fork);
  if (mg->ev_join) (void)hipEventDestroy(mg->ev_join);
  for (auto *list : {&mg->prof_ev, &mg->prof_gj_ev})
    for (auto &p : *list) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
  clear_graphs(*mg);
  free_list(mg->owned);
  free_list(mg->kry.owned);
  if (mg->kry.pinned) pinned_slot_release(mg->kry.pinned);
  if (mg->kry.ev_done) (void)hipEventDestroy(mg->kry.ev_done);
  delete mg;
}

// ------------------------------------------------------------------ FGMRES
void clear_graphs(MG &mg) {
  for (auto &kv : mg.graphs) (void)hipGraphExecDestroy(kv.second);
  mg.graphs.clear();
  // the per-step slots stay (a later solve with the same restart indexes them)
  for (auto &g : mg.kry.step_graphs) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

void ensure_krylov(MG &mg, int m) {
  Krylov &K = mg.kry;
  const int n = mg.lv.back().n;
  if (K.m == m && K.V) return;
  for (auto &g : K.step_graphs)
    if (g) (void)hipGraphExecDestroy(g);
  K.step_graphs.assign(m, nullptr);
  free_list(K.owned);
  K.m = m;
  K.V = dalloc<double>((int64_t)n * (m + 1), K.owned);
  K.Z = dalloc<double>((int64_t)n * m, K.owned);
  K.H = dalloc<double>((int64_t)(m + 1) * m, K.owned);
  K.cs = dalloc<double>(m + 1, K.owned);
  K.sn = dalloc<double>(m + 1, K.owned);
  K.g = dalloc<double>(m + 2, K.owned);
  K.y = dalloc<double>(m + 1, K.owned);
  K.h1 = dalloc<double>(m + 2, K.owned);
  K.partial = dalloc<double>((int64_t)2 * krylov_blocks(n) * kMaxKrylovCols, K.owned);
  K.npart = dalloc<double>(krylov_blocks(n), K.owned);
  K.nrm = dalloc<double>(4, K.owned);
  K.flags = dalloc<double>(4, K.owned);
  K.scal = dalloc<double>(4, K.owned);
  K.w = dalloc<double>(n, K.owned);
  if (!K.ev_done)
    hip_check(hipEventCreateWithFlags(&K.ev_done, hipEventDisableTiming), "event");
  if (!K.pinned) {
    K.pinned = pinned_slot_acquire();
    hip_check(hipHostGetDevicePointer((void **)&K.pinned_dev, K.pinned, 0), "pinned address");
  }
}

// The Krylov buffers in one region (sizes as ensure_krylov allocates them),
// each starting on a 256-byte boundary.
static int64_t krylov_layout(int n, int m, double *base, Krylov *K) {
  int64_t off = 0;
  auto take = [&](int64_t cnt) {
    double *p = base ? base + off : nullptr;
    off += (cnt + 31) / 32 * 32;
    return p;
  };
  double *V = take((int64_t)n * (m + 1)), *Z = take((int64_t)n * m), *H = take((int64_t)(m + 1) * m);
  double *cs = take(m + 1), *sn = take(m + 1), *g = take(m + 2), *y = take(m + 1), *h1 = take(m + 2);
  double *partial = take((int64_t)2 * krylov_blocks(n) * kMaxKrylovCols), *npart = take(krylov_blocks(n));
  double *nrm = take(4), *flags = take(4), *scal = take(4), *w = take(n);
  if (K) {
    K->V = V; K->Z = Z; K->H = H; K->cs = cs; K->sn = sn; K->g = g; K->y = y; K->h1 = h1;
    K->partial = partial; K->npart = npart; K->nrm = nrm; K->flags = flags; K->scal = scal; K->w = w;
  }
  return off;
}
int64_t krylov_doubles(int n, int m) { return krylov_layout(n, m, nullptr, nullptr); }
void bind_krylov(Krylov &K, const MG &mg, double *base, int n, int m) {
  krylov_layout(n, m, base, &K);
  K.m = m;
  K.pinned = mg.kry.pinned;
  K.pinned_dev = mg.kry.pinned_dev;
  K.ev_done = mg.kry.ev_done;
}

// ---- GMRES as a host state machine: enqueue() puts the next unit of work on
// the stream (ending with a small D2H copy into pinned memory), complete()
// runs after the stream has drained and decides what comes next.  The
// synchronous solve alternates the two; the server interleaves many systems.
void validate_krylov(const fsi_krylov_opts &ko) {
  if (ko.restart < 1 || ko.restart > 60) throw Error(FSI_E_INVALID, "restart must be in [1, 60]");
  if (!(ko.rtol >= 0.0) || ko.maxit < 1 || ko.fixed_iters < 0)
    throw Error(FSI_E_INVALID, "invalid Krylov options (rtol, maxit, fixed_iters)");
  if (ko.orth != FSI_ORTH_CGS2 && ko.orth != FSI_ORTH_CGS) throw Error(FSI_E_INVALID, "unknown orth");
  if (ko.side != FSI_SIDE_RIGHT && ko.side != FSI_SIDE_LEFT) throw Error(FSI_E_INVALID, "unknown side");
  if (ko.x0_nonzero != 0 && ko.x0_nonzero != 1) throw Error(FSI_E_INVALID, "x0_nonzero must be 0 or 1");
}

void FgmresRun::start(MG &mg_, const double *b_, double *x_, const fsi_krylov_opts &ko_,
                      hipStream_t st_, Krylov *ws) {
  mg = &mg_;
  b = b_;
  x = x_;
  ko = ko_;
  st = st_;
  validate_krylov(ko);
  left = ko.side == FSI_SIDE_LEFT;
  twice = ko.orth == FSI_ORTH_CGS2;
  t0 = std::chrono::steady_clock::now();
  if (ws) {
    K = ws;
    graphs = false;
  } else {
    ensure_krylov(*mg, ko.restart);
    K = &mg->kry;
    graphs = mg->opts.use_graph && !mg->prof_on;
    Krylov &G = *K;
    if (G.graph_side != ko.side || G.graph_orth != ko.orth ||   // the step graphs hold one variant
        (int)G.step_graphs.size() != ko.restart) {
      for (auto &g : G.step_graphs)
        if (g) (void)hipGraphExecDestroy(g);
      G.step_graphs.assign(ko.restart, nullptr);
      G.graph_side = ko.side;
      G.graph_orth = ko.orth;
    }
  }
  Krylov &K = *this->K;
  Level &F = mg->lv.back();
  const int n = F.n;
  fixed = ko.fixed_iters > 0;
  limit = fixed ? ko.fixed_iters : ko.maxit;
  iters = restarts = j = k = 0;
  converged = false;
  nhist = 0;
  est = NAN;
  true_res = 0.0;
  if (!ko.x0_nonzero) launch_fill_f64(x, n, 0.0, st);
  // |b|^2 and the monitored initial residual
  launch_kdot(n, b, n, 1, b, K.partial, K.nrm + 1, st);
  enqueue_residual();
  hip_check(hipMemcpyAsync(K.pinned, K.nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, st), "D2H");
  phase = kFirst;
}

// the monitored residual into K.w and its square norm into nrm[0]: b - J x
// (RIGHT) or M^{-1}(b - J x) (LEFT, through the first column of Z, which the
// left form does not otherwise use)
void FgmresRun::enqueue_residual() {
  Krylov &K = *this->K;
  Level &F = mg->lv.back();
  const int n = F.n;
  if (left) {
    launch_spmv(F.J.v64(), x, b, K.Z, kSpmvResid, F.J.lpr, st);
    apply_vcycle(*mg, K.Z, K.w, st);
  } else {
    launch_spmv(F.J.v64(), x, b, K.w, kSpmvResid, F.J.lpr, st);
  }
  launch_kdot(n, K.w, n, 1, K.w, K.partial, K.nrm, st);
}

// |b - J x|^2 into nrm[2] and the pinned slot (LEFT form, once at the end)
void FgmresRun::enqueue_true_residual() {
  Krylov &K = *this->K;
  Level &F = mg->lv.back();
  launch_spmv(F.J.v64(), x, b, K.Z, kSpmvResid, F.J.lpr, st);
  launch_kdot(F.n, K.Z, F.n, 1, K.Z, K.partial, K.nrm + 2, st);
  hip_check(hipMemcpyAsync(K.pinned, K.nrm + 2, sizeof(double), hipMemcpyDeviceToHost, st), "D2H");
}

// Arnoldi step j: RIGHT v_j -> z_j = M^{-1} v_j -> w = J z_j; LEFT v_j -> J v_j
// -> w = M^{-1} J v_j; then the orthogonalisation, the Givens column and
// v_{j+1}; |g_{j+1}| and the breakdown flag land in pinned memory
void FgmresRun::enqueue_step() {
  Krylov &K = *this->K;
  Level &F = mg->lv.back();
  const int n = F.n, m = ko.restart;
  if (j == 0) launch_start_cycle(n, K.w, K.nrm, K.V, K.g, m, st);
  double *vj = K.V + (int64_t)j * n;
  if (left) {
    launch_spmv(F.J.v64(), vj, (const double *)nullptr, K.Z, kSpmvSet, F.J.lpr, st);
    apply_vcycle(*mg, K.Z, K.w, st);
  } else {
    double *zj = K.Z + (int64_t)j * n;
    apply_vcycle(*mg, vj, zj, st);
    launch_spmv(F.J.v64(), zj, (const double *)nullptr, K.w, kSpmvSet, F.J.lpr, st);
  }
  launch_arnoldi_orth(n, K.V, n, j + 1, K.w, K.partial, K.h1, K.npart, K.V + (int64_t)(j + 1) * n,
                      K.H, m + 1, j, K.cs, K.sn, K.g, K.flags, K.scal, K.pinned_dev, st, twice);
}

// the step in two parts around an externally applied V-cycle (the server's
// batched V-cycles): the part before it, returning the V-cycle's input and
// output vectors, and the part after it
void FgmresRun::enqueue_step_pre(const double **vin, double **vout) {
  Krylov &K = *this->K;
  Level &F = mg->lv.back();
  const int n = F.n, m = ko.restart;
  reinterpret_cast<volatile double *>(K.pinned)[2] = 0.0;   // set again by the step's last kernel
  if (j == 0) launch_start_cycle(n, K.w, K.nrm, K.V, K.g, m, st);
  double *vj = K.V + (int64_t)j * n;
  if (left) {
    launch_spmv(F.J.v64(), vj, (const double *)nullptr, K.Z, kSpmvSet, F.J.lpr, st);
    *vin = K.Z;
    *vout = K.w;
  } else {
    *vin = vj;
    *vout = K.Z + (int64_t)j * n;
  }
  hip_check(hipGetLastError(), "arnoldi launch");
}
void FgmresRun::enqueue_step_post() {
  Krylov &K = *this->K;
  Level &F = mg->lv.back();
  const int n = F.n, m = ko.restart;
  if (!left) {
    double *zj = K.Z + (int64_t)j * n;
    launch_spmv(F.J.v64(), zj, (const double *)nullptr, K.w, kSpmvSet, F.J.lpr, st);
  }
  launch_arnoldi_orth(n, K.V, n, j + 1, K.w, K.partial, K.h1, K.npart, K.V + (int64_t)(j + 1) * n,
                      K.H, m + 1, j, K.cs, K.sn, K.g, K.flags, K.scal, K.pinned_dev, st, twice);
  hip_check(hipGetLastError(), "arnoldi launch");
}

void FgmresRun::enqueue() {
  if (phase != kIter) return;
  Krylov &K = *this->K;
  reinterpret_cast<volatile double *>(K.pinned)[2] = 0.0;   // set again by the step's last kernel
  if (graphs) {
    hipGraphExec_t &ex = K.step_graphs[j];
    if (!ex) {
      hipGraph_t g;
      hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture");
      enqueue_step();
      hip_check(hipStreamEndCapture(st, &g), "end capture");
      hip_check(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "instantiate");
      (void)hipGraphDestroy(g);
    }
    hip_check(hipGraphLaunch(ex, st), "graph launch");
  } else {
    enqueue_step();
  }
  hip_check(hipGetLastError(), "arnoldi launch");
}

// end of a cycle: y = H^{-1} g, x += Z y (RIGHT) or V y (LEFT), then the
// monitored residual of the new x decides exit or restart
void FgmresRun::finish_cycle() {
  Krylov &K = *this->K;
  Level &F = mg->lv.back();
  launch_backsolve(K.H, ko.restart + 1, K.g, k, K.y, st);
  launch_zupdate(F.n, left ? K.V : K.Z, F.n, k, K.y, x, st);
  ++restarts;
  enqueue_residual();
  hip_check(hipMemcpyAsync(K.pinned, K.nrm, sizeof(double), hipMemcpyDeviceToHost, st), "D2H");
  phase = kCheck;
}

// the solve is over: the right form already holds |b - J x|; the left form
// computes it in one more phase
bool FgmresRun::finish() {
  if (left) {
    enqueue_true_residual();
    phase = kFinal;
    return false;
  }
  true_res = beta;
  phase = kDone;
  return true;
}

void FgmresRun::add_hist(double v) {
  if (ko.history && nhist <= ko.maxit) ko.history[nhist] = v;
  ++nhist;
}

// decide after the stream drained; returns true when the solve is over
bool FgmresRun::complete() {
  Krylov &K = *this->K;
  const double tol = ko.rtol * ref;
  if (phase == kFirst) {
    const double bn2 = K.pinned[1];
    if (!std::isfinite(bn2)) throw Error(FSI_E_NONFINITE, "right-hand side has NaN/Inf");
    bnorm = std::sqrt(bn2);
    beta = std::sqrt(K.pinned[0]);
    if (!std::isfinite(beta)) throw Error(FSI_E_NONFINITE, "non-finite initial residual");
    beta0 = beta;
    ref = left ? beta : bnorm;
    add_hist(beta);
    const double tol0 = ko.rtol * ref;
    if ((!fixed && beta <= tol0) || iters >= limit || beta == 0.0) {
      converged = beta <= tol0;
      est = ref > 0 ? beta / ref : 0.0;
      return finish();
    }
    j = 0;
    phase = kIter;
    return false;
  }
  if (phase == kIter) {
    const double gj = K.pinned[0];
    const bool breakdown = K.pinned[1] != 0.0;
    if (!std::isfinite(gj)) throw Error(FSI_E_NONFINITE, "non-finite Krylov residual estimate");
    ++iters;
    est = gj / ref;
    add_hist(gj);
    k = j + 1;
    if ((!fixed && gj <= tol) || breakdown || iters >= limit || k == ko.restart) {
      finish_cycle();
    } else {
      ++j;
    }
    return false;
  }
  if (phase == kCheck) {
    beta = std::sqrt(K.pinned[0]);
    if (!std::isfinite(beta)) throw Error(FSI_E_NONFINITE, "non-finite residual");
    if ((!fixed && beta <= tol) || iters >= limit || beta == 0.0) {
      converged = beta <= tol;
      return finish();
    }
    j = 0;
    phase = kIter;
    return false;
  }
  if (phase == kFinal) {
    true_res = std::sqrt(K.pinned[0]);
    phase = kDone;
    return true;
  }
  return phase == kDone;
}

void FgmresRun::fill_info(fsi_solve_info *info) const {
  if (!info) return;
  info->iters = iters;
  info->restarts = restarts;
  info->converged = converged ? 1 : 0;
  info->true_relres = bnorm > 0 ? true_res / bnorm : 0.0;
  info->est_relres = est;
  info->setup_ms = mg->setup_ms;
  info->solve_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  // the monitored residual at exit over the initial one, per iteration
  info->rho = iters > 0 && beta0 > 0 ? std::pow(beta / beta0, 1.0 / iters) : 0.0;
}

fsi_status fgmres(MG &mg, const double *b, double *x, const fsi_krylov_opts &ko, fsi_solve_info *info,
                  hipStream_t st, Krylov *ws) {
  FgmresRun run;
  run.start(mg, b, x, ko, st, ws);
  // A phase's outcome is a few bytes in pinned memory.  The start and restart
  // phases copy it and are waited for by polling an event behind the copy; an
  // Arnoldi step's last kernel writes it itself with a ready mark, which the
  // host polls (the stream is queried now and then so that a failed launch
  // cannot leave the host waiting).
  auto wait_copy = [&](const char *what) {
    hip_check(hipEventRecord(run.K->ev_done, st), what);
    hipError_t e;
    while ((e = hipEventQuery(run.K->ev_done)) == hipErrorNotReady) {
    }
    hip_check(e, what);
  };
  auto wait_step = [&]() {
    volatile double *ready = run.K->pinned + 2;
    for (unsigned spin = 1; *ready == 0.0; ++spin) {
      if (spin % 4096 == 0) {
        const hipError_t e = hipStreamQuery(st);
        if (e == hipSuccess) {
          if (*ready != 0.0) break;
          throw Error(FSI_E_DEVICE, "Arnoldi step finished without its result");
        }
        if (e != hipErrorNotReady) hip_check(e, "fgmres step");
      }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
  };
  wait_copy("fgmres start");
  while (!run.complete()) {
    run.enqueue();
    if (run.phase == FgmresRun::kIter)
      wait_step();
    else
      wait_copy("fgmres restart");
  }
  run.fill_info(info);
  return run.converged ? FSI_OK : FSI_NOT_CONVERGED;
}

// ------------------------------------------------------------------ autotuner
// Lanes per row of every SpMV (J, P, R per level) and the panel width of the
// batched Gauss-Jordan, timed with events on the stream; results persist in a
// text database keyed by operator shape and precision.
static float time_events(hipStream_t st, const std::function<void()> &fn, int reps) {
  hipEvent_t a, b;
  hip_check(hipEventCreate(&a), "event");
  hip_check(hipEventCreate(&b), "event");
  fn();
  hip_check(hipEventRecord(a, st), "record");
  for (int i = 0; i < reps; ++i) fn();
  hip_check(hipEventRecord(b, st), "record");
  hip_check(hipEventSynchronize(b), "event sync");
  float ms = 0.f;
  hip_check(hipEventElapsedTime(&ms, a, b), "elapsed");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

// the batched inversion's workgroup count and its longest-first schedule
static void set_gj_grid(MG &mg, int grid, hipStream_t st) {
  grid = std::max(1, std::min(grid, mg.npatch_all));
  const std::vector<int> sched = gj_schedule(mg.h_all_pm.data(), mg.npatch_all, grid);
  hip_check(hipMemcpyAsync(mg.gj_sched, sched.data(), sizeof(int) * sched.size(), hipMemcpyHostToDevice, st),
            "schedule upload");
  hip_check(hipStreamSynchronize(st), "schedule upload");
  mg.gj_grid = grid;
}

int autotune(MG &mg, const char *db_path, hipStream_t st) {
  std::map<std::string, int> db;
  if (db_path) {
    if (FILE *f = fopen(db_path, "r")) {
      char key[256];
      int v;
      while (fscanf(f, "%255s %d", key, &v) == 2) db[key] = v;
      fclose(f);
    }
  }
  int measured = 0;
  const char *prec = mg.mixed ? "f32" : "f64";
  auto tune_csr = [&](DevCsr &A, const char *what, double *x64, double *y64, float *x32, float *y32,
                      bool use32) {
    char key[256];
    snprintf(key, sizeof key, "spmv:%s:%s:%d:%d:%d", what, use32 ? "f32" : "f64", A.n, A.m, A.nnz);
    auto it = db.find(key);
    if (it != db.end()) {
      A.lpr = it->second;
      return;
    }
    int best = A.lpr;
    float best_ms = 1e30f;
    for (int lpr : {2, 4, 8, 16, 32, 64}) {
      float ms;
      if (use32)
        ms = time_events(st, [&] { launch_spmv(A.v32(), x32, (const float *)nullptr, y32, kSpmvSet, lpr, st); }, 10);
      else
        ms = time_events(st, [&] { launch_spmv(A.v64(), x64, (const double *)nullptr, y64, kSpmvSet, lpr, st); }, 10);
      if (ms < best_ms) {
        best_ms = ms;
        best = lpr;
      }
    }
    A.lpr = best;
    db[key] = best;
    ++measured;
  };
  for (int l = 0; l < mg.nlevels; ++l) {
    Level &L = mg.lv[l];
    const bool use32 = mg.mixed && l > 0;
    launch_fill_f64(L.r, L.n, 1.0, st);
    if (use32) launch_fill_f32(L.r32, L.n, 1.0f, st);
    tune_csr(L.J, "J", L.r, L.s, L.r32, L.s32, use32);
    if (l > 0) {
      Level &C = mg.lv[l - 1];
      launch_fill_f64(C.r, C.n, 1.0, st);
      if (use32) launch_fill_f32(C.r32, C.n, 1.0f, st);
      tune_csr(L.P, "P", C.r, L.s, C.r32, L.s32, use32);
      tune_csr(L.R, "R", L.r, C.s, L.r32, C.s32, use32);
    }
  }
  if (mg.npatch_all && mg.blk_scratch) {
    // The batched inversion's kernel variant and grid, chosen together: a
    // variant on 256 threads fits two workgroups on a compute unit and wants
    // one workgroup per block, a 512-thread one the fewest rounds (which also
    // leaves the most room to the coarsest inversion beside it).  Every
    // (variant, grid) pair is timed on the extraction and inversion launches;
    // the best three are then timed on whole refactors (the coarse chain
    // overlaps the batched launch there).  The schedule changes which
    // workgroup inverts a block, not the result.
    char key[256], gkey[256];
    snprintf(key, sizeof key, "gj3:%s%d:%d:%lld", mg.mixed ? "f32:" : "", mg.mmax_all, mg.npatch_all,
             (long long)mg.blk_total);
    auto gj_key = [&](int var) {
      snprintf(gkey, sizeof gkey, "gjg:%s%d:%d:%lld:%d", mg.mixed ? "f32:" : "", mg.mmax_all,
               mg.npatch_all, (long long)mg.blk_total, var);
      return std::string(gkey);
    };
    auto it = db.find(key);
    if (it != db.end() && db.count(gj_key(it->second))) {
      mg.gj_variant = it->second;
      set_gj_grid(mg, db[gj_key(it->second)], st);
    } else {
      int dev = 0, ncu = 256;
      if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
      std::vector<int> grids;
      for (int g : {gj_batched_grid(mg.npatch_all), ncu - 64, ncu - 48, ncu - 40, 2 * ncu}) {
        g = std::max(1, std::min(g, mg.npatch_all));
        if (std::find(grids.begin(), grids.end(), g) == grids.end()) grids.push_back(g);
      }
      const std::vector<int> vars =
          mg.mixed ? std::vector<int>{kGjF64x512, kGjF32x512, kGjF32x256, kGjF32x512r2, kGjF48x512r2, kGjPF32x512}
                   : std::vector<int>{kGj16x256, kGj16x512, kGj32x512, kGjWideG, kGj24x512, kGjP32x512};
      std::vector<std::tuple<float, int, int>> timed;   // (ms, variant, grid)
      // every variant keeps at least 40 compute units free for the coarsest
      // inversion's chain on the side stream.  With more workgroups than
      // units the batched launch occupies every unit (the first ncu
      // workgroups go one to a unit, 256-thread ones too) until its last
      // block is dispatched, and whether the chain overlaps it then depends
      // on which launch reaches the device first: back to back here it
      // often does, after a solve it did not, and the refactor took the two
      // one after the other
      // (on a small device: at most half the units, and the smallest grid is
      // always allowed)
      const int gcap = std::max(ncu - 40, (ncu + 1) / 2);
      const int gmin = *std::min_element(grids.begin(), grids.end());
      auto grid_ok = [&](int, int g) { return g <= gcap || g == gmin; };
      for (int var : vars) {
        if (!gj_variant_ok(var, mg.mmax_all)) continue;
        for (int g : grids) {
          if (!grid_ok(var, g)) continue;
          set_gj_grid(mg, g, st);
          const float ms = time_events(st, [&] {
            extract_blocks(mg, st);
            invert_blocks(mg, var, st, nullptr, nullptr);
          }, 1);
          timed.emplace_back(ms, var, g);
        }
      }
      std::sort(timed.begin(), timed.end());
      int best_var = std::get<1>(timed[0]), best_grid = std::get<2>(timed[0]);
      // whole refactors decide among every grid of the two fastest variants
      // (a grid that speeds the batched launch up may starve the coarse chain)
      std::vector<std::pair<int, int>> finals;
      std::vector<int> top_vars;
      for (auto &t : timed)
        if (std::find(top_vars.begin(), top_vars.end(), std::get<1>(t)) == top_vars.end() && top_vars.size() < 2)
          top_vars.push_back(std::get<1>(t));
      for (int v : top_vars)
        for (int g : grids)
          if (grid_ok(v, g)) finals.push_back({v, g});
      double best_ms = 1e300;
      for (auto &fg : finals) {
        mg.gj_variant = fg.first;
        set_gj_grid(mg, fg.second, st);
        refactor(mg, st);
        for (int rep = 0; rep < 2; ++rep) {
          const auto a = std::chrono::steady_clock::now();
          refactor(mg, st);
          const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
          if (ms < best_ms) {
            best_ms = ms;
            best_var = mg.gj_variant;
            best_grid = mg.gj_grid;
          }
        }
      }
      mg.gj_variant = best_var;
      set_gj_grid(mg, best_grid, st);
      db[key] = best_var;
      db[gj_key(best_var)] = best_grid;
      ++measured;
      refactor(mg, st);   // the blocks were overwritten by the timing runs
    }
  }
  hip_check(hipGetLastError(), "autotune");
  clear_graphs(mg);
  if (db_path && measured) {
    if (FILE *f = fopen(db_path, "w")) {
      for (auto &kv : db) fprintf(f, "%s %d\n", kv.first.c_str(), kv.second);
      fclose(f);
    }
  }
  (void)prec;
  return measured;
}

}  // namespace fsi

// ==================================================================== C ABI
using namespace fsi;

#define FSI_GUARD(body)                               \
  try {                                               \
    body                                              \
  } catch (const Error &e) {                          \
    set_error(e.msg);                                 \
    return e.code;                                    \
  } catch (const std::exception &e) {                 \
    set_error(std::string("internal error: ") + e.what()); \
    return FSI_E_DEVICE;                              \
  }

extern "C" {

int32_t fsi_abi_version(void) { return FSI_ABI_VERSION; }

const char *fsi_status_string(fsi_status s) {
  switch (s) {
    case FSI_OK: return "ok";
    case FSI_NOT_CONVERGED: return "not converged";
    case FSI_PENDING: return "pending";
    case FSI_E_INVALID: return "invalid argument";
    case FSI_E_OOM: return "out of device memory";
    case FSI_E_SINGULAR: return "singular block";
    case FSI_E_DEVICE: return "device error";
    case FSI_E_NONFINITE: return "non-finite input";
    case FSI_E_CAPACITY: return "request exceeds capacity";
    case FSI_E_UNKNOWN_TICKET: return "unknown ticket";
    default: return "unknown status";
  }
}

const char *fsi_last_error(void) { return g_last_error.c_str(); }

fsi_status fsi_mg_setup(const fsi_level *levels, int32_t nlevels, const fsi_mg_opts *opts,
                        void *hip_stream, struct fsi_mg **out) {
  FSI_GUARD({
    if (!out) throw Error(FSI_E_INVALID, "null output handle");
    *out = nullptr;
    validate_levels(levels, nlevels, opts);
    hipStream_t own = nullptr;
    hip_check(hipStreamCreate(&own), "stream");
    try {
      MG *mg = mg_setup(levels, nlevels, opts, (hipStream_t)hip_stream, own);
      *out = reinterpret_cast<fsi_mg *>(mg);
    } catch (...) {
      (void)hipStreamDestroy(own);
      throw;
    }
    return FSI_OK;
  })
}

fsi_status fsi_mg_vcycle(struct fsi_mg *h, const double *r_dev, double *z_dev, void *hip_stream) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg || !r_dev || !z_dev) throw Error(FSI_E_INVALID, "null argument");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : mg->own_stream;
    run_vcycle(*mg, r_dev, z_dev, st);
    hip_check(hipGetLastError(), "vcycle launch");
    return FSI_OK;
  })
}

fsi_status fsi_mg_vcycle_batch(struct fsi_mg *const *mgs, int32_t count, const double *const *r_dev,
                               double *const *z_dev, void *hip_stream) {
  FSI_GUARD({
    if (!mgs || !r_dev || !z_dev || count < 1) throw Error(FSI_E_INVALID, "null argument or count < 1");
    std::vector<BatchItem> items;
    for (int i = 0; i < count; ++i) {
      MG *mg = reinterpret_cast<MG *>(mgs[i]);
      if (!mg || !r_dev[i] || !z_dev[i]) throw Error(FSI_E_INVALID, "null argument");
      items.push_back(BatchItem{mg, r_dev[i], z_dev[i]});
    }
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : items[0].mg->own_stream;
    batched_vcycle(items, st);
    return FSI_OK;
  })
}

fsi_status fsi_fgmres_solve(struct fsi_mg *h, const double *b_dev, double *x_dev,
                            const fsi_krylov_opts *kopts, fsi_solve_info *info, void *hip_stream) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg || !b_dev || !x_dev || !kopts) throw Error(FSI_E_INVALID, "null argument");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : mg->own_stream;
    return fgmres(*mg, b_dev, x_dev, *kopts, info, st);
  })
}

fsi_status fsi_fgmres_solve_noalloc(struct fsi_mg *h, const double *b_dev, double *x_dev,
                                    const fsi_krylov_opts *kopts, fsi_solve_info *info,
                                    void *hip_stream) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg || !b_dev || !x_dev || !kopts) throw Error(FSI_E_INVALID, "null argument");
    validate_krylov(*kopts);
    const int n = mg->lv.back().n;
    const int64_t need = krylov_doubles(n, kopts->restart) * 8;
    if (need > kStaticScratchBytes) {
      char buf[200];
      snprintf(buf, sizeof buf,
               "the Krylov workspace of %d unknowns at restart %d takes %lld bytes; the static "
               "workspace holds %lld",
               n, kopts->restart, (long long)need, (long long)kStaticScratchBytes);
      throw Error(FSI_E_CAPACITY, buf);
    }
    int dev = -1;
    hip_check(hipGetDevice(&dev), "device");
    if (dev != mg->device) throw Error(FSI_E_INVALID, "the handle's device is not the current device");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : mg->own_stream;
    Krylov ws;
    bind_krylov(ws, *mg, mg->static_ws, n, kopts->restart);
    return fgmres(*mg, b_dev, x_dev, *kopts, info, st, &ws);
  })
}

fsi_status fsi_mg_apply(struct fsi_mg *h, int32_t level, int32_t op, const double *x_dev,
                        const double *r_dev, double *y_dev, void *hip_stream) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg || !x_dev || !y_dev) throw Error(FSI_E_INVALID, "null argument");
    if (level < 0 || level >= mg->nlevels) throw Error(FSI_E_INVALID, "level out of range");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : mg->own_stream;
    Level &L = mg->lv[level];
    switch (op) {
      case 0: launch_spmv(L.J.v64(), x_dev, (const double *)nullptr, y_dev, kSpmvSet, L.J.lpr, st); break;
      case 1:
        if (!r_dev) throw Error(FSI_E_INVALID, "r required");
        launch_spmv(L.J.v64(), x_dev, r_dev, y_dev, kSpmvResid, L.J.lpr, st);
        break;
      case 2:
        if (level == 0) throw Error(FSI_E_INVALID, "no prolongation on level 0");
        launch_spmv(L.P.v64(), x_dev, (const double *)nullptr, y_dev, kSpmvSet, L.P.lpr, st);
        break;
      case 3:
        if (level == 0) throw Error(FSI_E_INVALID, "no restriction on level 0");
        launch_spmv(L.R.v64(), x_dev, (const double *)nullptr, y_dev, kSpmvSet, L.R.lpr, st);
        break;
      case 4:
        if (level == 0) throw Error(FSI_E_INVALID, "no patches on level 0");
        if (mg->mixed) throw Error(FSI_E_INVALID, "op 4 needs the FP64 precision");
        launch_fill_f64(y_dev, L.n, 0.0, st);
        ras64_omega(*mg, L, x_dev, y_dev, 1.0, true, st);
        break;
      case 5:
        if (level != 0) throw Error(FSI_E_INVALID, "direct solve only on level 0");
        launch_dense_gemv(L.C0, L.n, x_dev, y_dev, st);
        break;
      case 6:   // one Schwarz application as the V-cycle performs it (mixed: FP32 inside)
        if (level == 0) throw Error(FSI_E_INVALID, "no patches on level 0");
        if (!mg->mixed) {
          launch_fill_f64(y_dev, L.n, 0.0, st);
          ras64_omega(*mg, L, x_dev, y_dev, 1.0, true, st);
        } else {
          launch_cast_d2f(x_dev, L.s32, L.n, st);
          ras32(*mg, L, L.s32, L.e32, false, st, 1.0);
          launch_cast_f2d(L.e32, y_dev, L.n, st);
        }
        break;
      default: throw Error(FSI_E_INVALID, "unknown op");
    }
    hip_check(hipGetLastError(), "apply launch");
    return FSI_OK;
  })
}

fsi_status fsi_mg_refactor(struct fsi_mg *h, void *hip_stream) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg) throw Error(FSI_E_INVALID, "null handle");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : mg->own_stream;
    refactor(*mg, st);
    return FSI_OK;
  })
}

fsi_status fsi_mg_autotune(struct fsi_mg *h, const char *db_path, void *hip_stream,
                           int32_t *measured) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg) throw Error(FSI_E_INVALID, "null handle");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : mg->own_stream;
    const int m = autotune(*mg, db_path, st);
    if (measured) *measured = m;
    return FSI_OK;
  })
}

fsi_status fsi_mg_jvalues(struct fsi_mg *h, int32_t level, double **val_dev) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg || !val_dev || level < 0 || level >= mg->nlevels) throw Error(FSI_E_INVALID, "bad argument");
    *val_dev = mg->lv[level].J.val;
    return FSI_OK;
  })
}

fsi_status fsi_mg_set_jvalues(struct fsi_mg *h, int32_t level, const double *val_dev, void *hip_stream) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg || !val_dev || level < 0 || level >= mg->nlevels) throw Error(FSI_E_INVALID, "bad argument");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : mg->own_stream;
    Level &L = mg->lv[level];
    hip_check(hipMemcpyAsync(L.J.val, val_dev, sizeof(double) * L.J.nnz, hipMemcpyDeviceToDevice, st),
              "D2D values");
    return FSI_OK;
  })
}

fsi_status fsi_mg_galerkin(struct fsi_mg *h, void *hip_stream) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg) throw Error(FSI_E_INVALID, "null handle");
    galerkin(*mg, hip_stream ? (hipStream_t)hip_stream : mg->own_stream);
    return FSI_OK;
  })
}

fsi_status fsi_mg_profile(struct fsi_mg *h, int32_t enable, double out[4]) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg) throw Error(FSI_E_INVALID, "null handle");
    if (enable) {
      mg->prof_on = true;
      mg->prof_used = mg->prof_gj_used = 0;
      return FSI_OK;
    }
    auto total = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>> &evs, size_t used) {
      double tot = 0.0;
      for (size_t i = 0; i < used; ++i) {
        hip_check(hipEventSynchronize(evs[i].second), "event sync");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, evs[i].first, evs[i].second), "elapsed");
        tot += ms;
      }
      return tot;
    };
    const double ras_ms = total(mg->prof_ev, mg->prof_used);
    const double gj_ms = total(mg->prof_gj_ev, mg->prof_gj_used);
    if (out) {
      out[0] = ras_ms;
      out[1] = (double)mg->prof_used;
      out[2] = gj_ms;
      out[3] = (double)mg->prof_gj_used;
    }
    mg->prof_on = false;
    mg->prof_used = mg->prof_gj_used = 0;
    return FSI_OK;
  })
}

fsi_status fsi_stream_read(const double *x_dev, int64_t n, double *out_dev, void *hip_stream) {
  FSI_GUARD({
    if (!x_dev || !out_dev || n < 2 || (n & 1) || (reinterpret_cast<uintptr_t>(x_dev) & 15))
      throw Error(FSI_E_INVALID, "stream read needs an even n >= 2 and a 16-byte aligned x");
    launch_stream_read(x_dev, n, out_dev, (hipStream_t)hip_stream);
    hip_check(hipGetLastError(), "stream read launch");
    return FSI_OK;
  })
}

int32_t fsi_stream_read_blocks(void) { return kStreamReadBlocks; }

fsi_status fsi_mg_level_info(struct fsi_mg *h, int32_t level, int64_t out[8]) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg || !out || level < 0 || level >= mg->nlevels) throw Error(FSI_E_INVALID, "bad argument");
    Level &L = mg->lv[level];
    out[0] = L.n;
    out[1] = L.J.nnz;
    out[2] = L.npatch;
    out[3] = L.sum_m;
    out[4] = L.sum_m2;
    out[5] = L.sum_om;
    out[6] = L.nilu;
    out[7] = L.ilu_nl + L.ilu_nu + L.ilu_rows;
    return FSI_OK;
  })
}

fsi_status fsi_mg_export_patches(struct fsi_mg *h, int32_t level, int64_t *ptr, int32_t *dof,
                                 uint8_t *owned, double *blocks) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg || level < 1 || level >= mg->nlevels) throw Error(FSI_E_INVALID, "bad level");
    Level &L = mg->lv[level];
    hipStream_t st = mg->own_stream;
    if (ptr) std::copy(L.h_ptr.begin(), L.h_ptr.end(), ptr);
    if (dof)
      hip_check(hipMemcpy(dof, L.d_dof, sizeof(int32_t) * L.h_dof.size(), hipMemcpyDeviceToHost),
                "D2H dof");
    if (owned) std::copy(L.h_owned.begin(), L.h_owned.end(), owned);
    if (blocks) {
      if (!mg->blk_scratch) throw Error(FSI_E_INVALID, "setup scratch released");
      double *B = mg->blk_scratch + L.blk_base;
      launch_fill_f64(B, L.boff_total, 0.0, st);
      launch_extract(L.J.val, L.ext_nslots, L.d_ext_src, L.d_ext_dst, B, st);
      hip_check(hipMemcpyAsync(blocks, B, sizeof(double) * L.boff_total, hipMemcpyDeviceToHost, st),
                "D2H blocks");
      hip_check(hipStreamSynchronize(st), "export");
    }
    return FSI_OK;
  })
}

fsi_status fsi_mg_destroy(struct fsi_mg *h) {
  FSI_GUARD({
    MG *mg = reinterpret_cast<MG *>(h);
    if (!mg) return FSI_OK;
    hipStream_t own = mg->own_stream;
    (void)hipStreamSynchronize(own);
    destroy_mg(mg);
    (void)hipStreamDestroy(own);
    return FSI_OK;
  })
}

}  // extern "C"
