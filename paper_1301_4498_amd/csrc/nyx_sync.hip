// nyx_sync.hip -- synchronisation of two AMR levels after the fine level has
// been advanced (Sec. 4.3 Multilevel Algorithm, Steps 2 and 8): the coarse
// cells beside the fine level get the difference between the fine and the
// coarse fluxes through their shared faces, so that the sums over both
// levels stay conserved, and each covered coarse cell takes the mean of its
// eight children.
//
// The host plans once per pair of box layouts:
//   - the interface faces: coarse faces with exactly one side covered by the
//     fine level (periodic images included); each gets a register slot, one
//     record for the coarse step (its own flux, scale -1) and one for the
//     fine steps (the 2 x 2 fine faces, scale 1/4), both applied by the
//     steps' record kernel (nyx_step.hip) as scale * dt * flux;
//   - the reflux cells: uncovered coarse cells with at least one interface
//     face, each with its faces in the order x-, x+, y-, y+, z-, z+;
//   - the average-down rectangles: each fine box's coarsened region cut by
//     the coarse boxes.
// The device applies A += (sum over faces of +R (low face) or -R (high
// face)) / dx and sets each covered cell to the mean of its eight children,
// one lane per cell.  Built without contraction (equal to the CPU reference
// bit for bit).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "nyx_internal.h"

namespace nyx {

struct RefluxCell {
  int box;       // coarse box
  unsigned idx;  // padded cell index in that box
  int e0, ne;    // its entries
};

struct RefluxEnt {
  long long slot;
  int sign;  // +1: the face is the cell's low face, -1: its high face
  int pad_;
};

// Coarse cells clo + [0, ext) of coarse box cbox are covered by fine box
// fbox; the children of coarse local cell clo + x start at fine local cell
// flo + 2 x.
struct AvgRect {
  int cbox, fbox;
  int clo[3], ext[3], flo[3];
  int pad_;
  FastDiv dx, dxy;  // division by ext[0] and ext[0] * ext[1]
};

struct RefluxArgs {
  const RefluxCell* cells;
  const RefluxEnt* ents;
  long long ncells;
  const BoxDev* coarse;
  double* cstate;
  const double* reg;
  long long nslots;
  int ncomp;
};

struct AvgArgs {
  const AvgRect* rects;
  const int* prefix;  // cells before each rectangle, nrect + 1 entries
  int nrect;
  const BoxDev* coarse;
  const BoxDev* fine;
  double* cstate;
  const double* fstate;
  int ncomp;
};

__device__ __forceinline__ unsigned sync_pidx(const BoxDev& b, int i, int j, int k) {
  return ((unsigned)(k + b.ng) * (unsigned)b.py + (unsigned)(j + b.ng)) * (unsigned)b.px +
         (unsigned)(i + b.ng);
}

__global__ __launch_bounds__(kBlock) void k_reflux(RefluxArgs A) {
  const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (q >= A.ncells) return;
  const RefluxCell c = A.cells[q];
  const BoxDev& B = A.coarse[c.box];
  for (int v = 0; v < A.ncomp; ++v) {
    double delta = 0.0;
    for (int e = c.e0; e < c.e0 + c.ne; ++e) {
      const RefluxEnt E = A.ents[e];
      const double r = A.reg[(long long)v * A.nslots + E.slot];
      delta = delta + (E.sign > 0 ? r : -r);
    }
    double* u = A.cstate + B.soff + (long long)v * B.sstride;
    stu(u, c.idx, ldu(u, c.idx) + delta / B.dx);
  }
}

__global__ __launch_bounds__(kBlock) void k_average_down(AvgArgs A) {
  const unsigned q = blockIdx.x * (unsigned)kBlock + threadIdx.x;
  if (q >= (unsigned)A.prefix[A.nrect]) return;
  int lo = 0, hi = A.nrect;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((unsigned)A.prefix[mid] <= q) lo = mid;
    else hi = mid;
  }
  const AvgRect& R = A.rects[lo];
  const unsigned r = q - (unsigned)A.prefix[lo];
  const unsigned a = fast_div(r, R.dx), b = fast_div(r, R.dxy);
  const int x[3] = {(int)(r - a * (unsigned)R.ext[0]), (int)(a - b * (unsigned)R.ext[1]), (int)b};
  const BoxDev& C = A.coarse[R.cbox];
  const BoxDev& F = A.fine[R.fbox];
  const unsigned ci = sync_pidx(C, R.clo[0] + x[0], R.clo[1] + x[1], R.clo[2] + x[2]);
  const unsigned f0 = sync_pidx(F, R.flo[0] + 2 * x[0], R.flo[1] + 2 * x[1], R.flo[2] + 2 * x[2]);
  const unsigned sy = (unsigned)F.px, sz = (unsigned)F.px * (unsigned)F.py;
  const unsigned child[8] = {f0,      f0 + 1,      f0 + sy,      f0 + sy + 1,
                             f0 + sz, f0 + sz + 1, f0 + sz + sy, f0 + sz + sy + 1};
  // the fine level is read-only here and lives apart from the coarse state
  const double* __restrict__ fs = A.fstate;
  double* __restrict__ cs = A.cstate;
  for (int v = 0; v < A.ncomp; ++v) {
    const double* u = fs + F.soff + (long long)v * F.sstride;
    double s = ldu(u, child[0]);
    for (int k = 1; k < 8; ++k) s = s + ldu(u, child[k]);
    stu(cs + C.soff + (long long)v * C.sstride, ci, 0.125 * s);
  }
}

}  // namespace nyx

// ---------------------------------------------------------------------------
// host planning and the C ABI
// ---------------------------------------------------------------------------
using namespace nyx;

struct nyx_sync_plan {
  int ncoarse = 0, nfine = 0;
  long long nfaces = 0, ncells = 0, ncovered = 0;
  int nrect = 0, avg_blocks = 0;
  BoxDev* coarse = nullptr;
  BoxDev* fine = nullptr;
  FluxRec* recs[2] = {nullptr, nullptr};
  std::vector<long long> prefix[2];  // per box, host
  std::vector<int> shapes[2];        // 3 ints per box, host
  RefluxCell* cells = nullptr;
  RefluxEnt* ents = nullptr;
  AvgRect* rects = nullptr;
  int* rect_prefix = nullptr;
  size_t cstate_span = 0, fstate_span = 0;
};

namespace nyx {

int sync_level_view(const nyx_sync_plan* p, int level, SyncLevelView* out) {
  if (!p || !out) return NYX_E_NULL;
  if (level != 0 && level != 1) return NYX_E_PARAM;
  out->recs = p->recs[level];
  out->prefix = p->prefix[level].data();
  out->shapes = p->shapes[level].data();
  out->nbox = level == 0 ? p->ncoarse : p->nfine;
  out->nslots = p->nfaces;
  return NYX_OK;
}

}  // namespace nyx

namespace {

size_t r256(size_t x) { return (x + 255) / 256 * 256; }

int wrapi(int x, int m) {
  const int r = x % m;
  return r < 0 ? r + m : r;
}

struct SyncHost {
  std::vector<BoxDev> coarse, fine;
  std::vector<FluxRec> recs[2];
  std::vector<long long> prefix[2];
  std::vector<RefluxCell> cells;
  std::vector<RefluxEnt> ents;
  std::vector<AvgRect> rects;
  std::vector<int> rect_prefix;
  long long nfaces = 0, ncovered = 0;
  size_t cstate_span = 0, fstate_span = 0;
};

int check_boxes_in(int nbox, const nyx_box* boxes, const int32_t* lo, const int* dom, bool even) {
  if (nbox < 1 || nbox > (1 << 20)) return NYX_E_SHAPE;
  if (!boxes || !lo) return NYX_E_NULL;
  for (int b = 0; b < nbox; ++b) {
    int rc = validate_box(&boxes[b]);
    if (rc) return rc;
    for (int d = 0; d < 3; ++d) {
      if (lo[3 * b + d] < 0 || lo[3 * b + d] + boxes[b].n[d] > dom[d]) return NYX_E_SHAPE;
      if (even && ((lo[3 * b + d] & 1) || (boxes[b].n[d] & 1))) return NYX_E_SHAPE;
    }
  }
  return NYX_OK;
}

// box-index map over the coarse domain; NYX_E_SHAPE when two regions overlap
int paint(std::vector<int>& map, const int* cdom, int b, const int* lo, const int* ext) {
  for (int k = lo[2]; k < lo[2] + ext[2]; ++k)
    for (int j = lo[1]; j < lo[1] + ext[1]; ++j)
      for (int i = lo[0]; i < lo[0] + ext[0]; ++i) {
        int& m = map[((size_t)k * cdom[1] + j) * cdom[0] + i];
        if (m >= 0) return NYX_E_SHAPE;
        m = b;
      }
  return NYX_OK;
}

int plan_sync(int nfine, const nyx_box* fboxes, const int32_t* flo, const int32_t* dom,
              int ncoarse, const nyx_box* cboxes, const int32_t* clo, SyncHost& H) {
  if (!dom) return NYX_E_NULL;
  for (int d = 0; d < 3; ++d)
    if (dom[d] < 2 || (dom[d] & 1) || dom[d] > (1 << 24)) return NYX_E_SHAPE;
  const int fdom[3] = {dom[0], dom[1], dom[2]};
  const int cdom[3] = {dom[0] / 2, dom[1] / 2, dom[2] / 2};
  if ((double)cdom[0] * cdom[1] * cdom[2] > (double)(1 << 28)) return NYX_E_SHAPE;
  int rc = check_boxes_in(nfine, fboxes, flo, fdom, true);
  if (rc) return rc;
  if ((rc = check_boxes_in(ncoarse, cboxes, clo, cdom, false))) return rc;
  H.coarse.resize(ncoarse);
  for (int b = 0; b < ncoarse; ++b) {
    box_layout(cboxes[b], b, 0, &H.coarse[b]);
    H.cstate_span = std::max(H.cstate_span, (size_t)(cboxes[b].state_off +
                                                     5 * cboxes[b].comp_stride + H.coarse[b].P));
  }
  H.fine.resize(nfine);
  for (int b = 0; b < nfine; ++b) {
    box_layout(fboxes[b], b, 0, &H.fine[b]);
    H.fstate_span = std::max(H.fstate_span, (size_t)(fboxes[b].state_off +
                                                     5 * fboxes[b].comp_stride + H.fine[b].P));
  }
  const size_t ncc = (size_t)cdom[0] * cdom[1] * cdom[2];
  std::vector<int> cmap(ncc, -1), fmap(ncc, -1);
  for (int b = 0; b < ncoarse; ++b)
    if ((rc = paint(cmap, cdom, b, clo + 3 * b, cboxes[b].n))) return rc;
  for (int b = 0; b < nfine; ++b) {
    const int lo[3] = {flo[3 * b] / 2, flo[3 * b + 1] / 2, flo[3 * b + 2] / 2};
    const int ext[3] = {fboxes[b].n[0] / 2, fboxes[b].n[1] / 2, fboxes[b].n[2] / 2};
    if ((rc = paint(fmap, cdom, b, lo, ext))) return rc;
  }
  auto at = [&](const std::vector<int>& m, const int* g) {
    return m[((size_t)g[2] * cdom[1] + g[1]) * cdom[0] + g[0]];
  };
  // interface faces, visited from the fine side
  struct Ent {
    size_t cell;
    int order;
    long long slot;
    int sign;
  };
  std::vector<Ent> ents;
  for (int fb = 0; fb < nfine; ++fb) {
    const int* L = flo + 3 * fb;
    const int Rlo[3] = {L[0] / 2, L[1] / 2, L[2] / 2};
    const int Rn[3] = {fboxes[fb].n[0] / 2, fboxes[fb].n[1] / 2, fboxes[fb].n[2] / 2};
    for (int d = 0; d < 3; ++d) {
      const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      for (int hiside = 0; hiside < 2; ++hiside) {
        for (int b2 = 0; b2 < Rn[t2]; ++b2)
          for (int b1 = 0; b1 < Rn[t1]; ++b1) {
            int B[3];
            B[d] = hiside ? Rlo[d] + Rn[d] - 1 : Rlo[d];
            B[t1] = Rlo[t1] + b1;
            B[t2] = Rlo[t2] + b2;
            int A[3] = {B[0], B[1], B[2]};
            A[d] += hiside ? 1 : -1;
            for (int e = 0; e < 3; ++e) A[e] = wrapi(A[e], cdom[e]);
            if (at(fmap, A) >= 0) continue;  // fine on both sides
            const int cb = at(cmap, A);
            if (cb < 0) return NYX_E_SHAPE;  // improper nesting
            const long long slot = H.nfaces++;
            // the coarse record: A's face in A's box; the fine one: the 2 x 2
            // faces of B's children next to A
            FluxRec c{}, f{};
            c.box = cb;
            c.d = d;
            c.nsub = 1;
            c.scale = -1.0;
            c.slot = slot;
            f.box = fb;
            f.d = d;
            f.nsub = 2;
            f.scale = 0.25;
            f.slot = slot;
            for (int e = 0; e < 3; ++e) {
              c.f[e] = A[e] - clo[3 * cb + e];
              f.f[e] = 2 * B[e] - L[e];
            }
            // B below A (fine box's high side): A's low face, the children's
            // high faces; B above A: A's high face, the children's low faces
            if (hiside) f.f[d] += 2;
            else c.f[d] += 1;
            H.recs[0].push_back(c);
            H.recs[1].push_back(f);
            const size_t cell = ((size_t)A[2] * cdom[1] + A[1]) * cdom[0] + A[0];
            ents.push_back(Ent{cell, 2 * d + (hiside ? 0 : 1), slot, hiside ? 1 : -1});
          }
      }
    }
  }
  if (H.nfaces > (1ll << 31) - 1 - kBlock) return NYX_E_SHAPE;
  // records by box, prefix per box
  for (int lv = 0; lv < 2; ++lv) {
    auto& v = H.recs[lv];
    std::stable_sort(v.begin(), v.end(), [](const FluxRec& a, const FluxRec& b) {
      return a.box < b.box;
    });
    const int nb = lv == 0 ? ncoarse : nfine;
    H.prefix[lv].assign(nb + 1, 0);
    for (const FluxRec& r : v) H.prefix[lv][r.box + 1]++;
    for (int b = 0; b < nb; ++b) H.prefix[lv][b + 1] += H.prefix[lv][b];
  }
  // reflux cells, their faces in x-, x+, y-, y+, z-, z+ order
  std::sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) {
    return a.cell != b.cell ? a.cell < b.cell : a.order < b.order;
  });
  for (size_t i = 0; i < ents.size();) {
    size_t j = i;
    while (j < ents.size() && ents[j].cell == ents[i].cell) ++j;
    const size_t cell = ents[i].cell;
    const int g[3] = {(int)(cell % cdom[0]), (int)(cell / cdom[0] % cdom[1]),
                      (int)(cell / ((size_t)cdom[0] * cdom[1]))};
    const int cb = at(cmap, g);
    const BoxDev& C = H.coarse[cb];
    RefluxCell rc_{};
    rc_.box = cb;
    const int l[3] = {g[0] - clo[3 * cb], g[1] - clo[3 * cb + 1], g[2] - clo[3 * cb + 2]};
    rc_.idx = (unsigned)(((long long)(l[2] + C.ng) * C.py + (l[1] + C.ng)) * C.px + (l[0] + C.ng));
    rc_.e0 = (int)H.ents.size();
    rc_.ne = (int)(j - i);
    for (size_t k = i; k < j; ++k) H.ents.push_back(RefluxEnt{ents[k].slot, ents[k].sign, 0});
    H.cells.push_back(rc_);
    i = j;
  }
  // average-down rectangles: each fine box's coarsened region cut by the
  // coarse boxes; every covered cell must lie in one
  for (int fb = 0; fb < nfine; ++fb) {
    const int* L = flo + 3 * fb;
    const int Rlo[3] = {L[0] / 2, L[1] / 2, L[2] / 2};
    const int Rn[3] = {fboxes[fb].n[0] / 2, fboxes[fb].n[1] / 2, fboxes[fb].n[2] / 2};
    long long got = 0;
    for (int cb = 0; cb < ncoarse; ++cb) {
      int a[3], e[3];
      bool any = true;
      for (int d = 0; d < 3; ++d) {
        a[d] = std::max(Rlo[d], (int)clo[3 * cb + d]);
        e[d] = std::min(Rlo[d] + Rn[d], (int)clo[3 * cb + d] + cboxes[cb].n[d]) - a[d];
        any = any && e[d] > 0;
      }
      if (!any) continue;
      AvgRect R{};
      R.cbox = cb;
      R.fbox = fb;
      for (int d = 0; d < 3; ++d) {
        R.clo[d] = a[d] - clo[3 * cb + d];
        R.ext[d] = e[d];
        R.flo[d] = 2 * a[d] - L[d];
      }
      R.dx = make_fastdiv((unsigned)e[0]);
      R.dxy = make_fastdiv((unsigned)e[0] * (unsigned)e[1]);
      H.rects.push_back(R);
      got += (long long)e[0] * e[1] * e[2];
    }
    if (got != (long long)Rn[0] * Rn[1] * Rn[2]) return NYX_E_SHAPE;
    H.ncovered += got;
  }
  H.rect_prefix.assign(H.rects.size() + 1, 0);
  long long acc = 0;
  for (size_t i = 0; i < H.rects.size(); ++i) {
    H.rect_prefix[i] = (int)acc;
    acc += (long long)H.rects[i].ext[0] * H.rects[i].ext[1] * H.rects[i].ext[2];
    if (acc > (1ll << 31) - 1 - kBlock) return NYX_E_SHAPE;
  }
  H.rect_prefix[H.rects.size()] = (int)acc;
  return NYX_OK;
}

template <class T>
size_t bytes_of(const std::vector<T>& v) {
  return r256(sizeof(T) * std::max<size_t>(v.size(), 1));
}

size_t sync_bytes(const SyncHost& H) {
  return bytes_of(H.coarse) + bytes_of(H.fine) + bytes_of(H.recs[0]) + bytes_of(H.recs[1]) +
         bytes_of(H.cells) + bytes_of(H.ents) + bytes_of(H.rects) + bytes_of(H.rect_prefix);
}

template <class T>
bool upload(T*& dst, char*& w, const std::vector<T>& v, hipStream_t s) {
  dst = (T*)w;
  w += bytes_of(v);
  if (v.empty()) return true;
  return hipMemcpyAsync(dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s) ==
         hipSuccess;
}

bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + bn && y < x + an;
}

}  // namespace

extern "C" {

int nyx_sync_plan_bytes(int nfine, const nyx_box* fboxes, const int32_t* flo, const int32_t* dom,
                        int ncoarse, const nyx_box* cboxes, const int32_t* clo, size_t* bytes) {
  if (!bytes) return NYX_E_NULL;
  SyncHost H;
  int rc = plan_sync(nfine, fboxes, flo, dom, ncoarse, cboxes, clo, H);
  if (rc) return rc;
  *bytes = sync_bytes(H);
  return NYX_OK;
}

int nyx_sync_plan_create(int nfine, const nyx_box* fboxes, const int32_t* flo, const int32_t* dom,
                         int ncoarse, const nyx_box* cboxes, const int32_t* clo, void* workspace,
                         size_t ws_bytes, void* stream, nyx_sync_plan** out) {
  if (!out || !workspace) return NYX_E_NULL;
  *out = nullptr;
  if ((uintptr_t)workspace & 255) return NYX_E_WORKSPACE;
  SyncHost H;
  int rc = plan_sync(nfine, fboxes, flo, dom, ncoarse, cboxes, clo, H);
  if (rc) return rc;
  if (ws_bytes < sync_bytes(H)) return NYX_E_WORKSPACE;
  nyx_sync_plan* p = new (std::nothrow) nyx_sync_plan;
  if (!p) return NYX_E_HIP;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)workspace;
  bool ok = upload(p->coarse, w, H.coarse, s) && upload(p->fine, w, H.fine, s) &&
            upload(p->recs[0], w, H.recs[0], s) && upload(p->recs[1], w, H.recs[1], s) &&
            upload(p->cells, w, H.cells, s) && upload(p->ents, w, H.ents, s) &&
            upload(p->rects, w, H.rects, s) && upload(p->rect_prefix, w, H.rect_prefix, s);
  // the host vectors die with this call: the copies must have completed
  if (ok) ok = hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    delete p;
    return NYX_E_HIP;
  }
  p->ncoarse = ncoarse;
  p->nfine = nfine;
  p->nfaces = H.nfaces;
  p->ncells = (long long)H.cells.size();
  p->ncovered = H.ncovered;
  p->nrect = (int)H.rects.size();
  p->avg_blocks = (H.rect_prefix.back() + kBlock - 1) / kBlock;
  for (int lv = 0; lv < 2; ++lv) p->prefix[lv] = H.prefix[lv];
  p->shapes[0].resize(3 * (size_t)ncoarse);
  for (int b = 0; b < ncoarse; ++b)
    for (int d = 0; d < 3; ++d) p->shapes[0][3 * b + d] = cboxes[b].n[d];
  p->shapes[1].resize(3 * (size_t)nfine);
  for (int b = 0; b < nfine; ++b)
    for (int d = 0; d < 3; ++d) p->shapes[1][3 * b + d] = fboxes[b].n[d];
  p->cstate_span = H.cstate_span;
  p->fstate_span = H.fstate_span;
  *out = p;
  return NYX_OK;
}

int nyx_sync_plan_destroy(nyx_sync_plan* plan) {
  delete plan;
  return NYX_OK;
}

int nyx_sync_plan_counts(const nyx_sync_plan* plan, long long* faces, long long* reflux_cells,
                         long long* covered_cells) {
  if (!plan) return NYX_E_NULL;
  if (faces) *faces = plan->nfaces;
  if (reflux_cells) *reflux_cells = plan->ncells;
  if (covered_cells) *covered_cells = plan->ncovered;
  return NYX_OK;
}

int nyx_reflux(nyx_sync_plan* plan, double* coarse_state, const double* reg, int ncomp,
               void* stream) {
  if (!plan || !coarse_state || !reg) return NYX_E_NULL;
  if (ncomp < 1 || ncomp > 6) return NYX_E_PARAM;
  if (overlaps(coarse_state, plan->cstate_span * sizeof(double), reg,
               (size_t)plan->nfaces * 6 * sizeof(double)))
    return NYX_E_ALIAS;
  if (plan->ncells == 0) return NYX_OK;
  RefluxArgs A{};
  A.cells = plan->cells;
  A.ents = plan->ents;
  A.ncells = plan->ncells;
  A.coarse = plan->coarse;
  A.cstate = coarse_state;
  A.reg = reg;
  A.nslots = plan->nfaces;
  A.ncomp = ncomp;
  hipLaunchKernelGGL(k_reflux, dim3((unsigned)((plan->ncells + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, (hipStream_t)stream, A);
  return hipGetLastError() == hipSuccess ? NYX_OK : NYX_E_HIP;
}

int nyx_average_down(nyx_sync_plan* plan, double* coarse_state, const double* fine_state,
                     int ncomp, void* stream) {
  if (!plan || !coarse_state || !fine_state) return NYX_E_NULL;
  if (ncomp < 1 || ncomp > 16) return NYX_E_PARAM;
  if (overlaps(coarse_state, plan->cstate_span * sizeof(double), fine_state,
               plan->fstate_span * sizeof(double)))
    return NYX_E_ALIAS;
  if (plan->nrect == 0) return NYX_OK;
  AvgArgs A{};
  A.rects = plan->rects;
  A.prefix = plan->rect_prefix;
  A.nrect = plan->nrect;
  A.coarse = plan->coarse;
  A.fine = plan->fine;
  A.cstate = coarse_state;
  A.fstate = fine_state;
  A.ncomp = ncomp;
  hipLaunchKernelGGL(k_average_down, dim3(plan->avg_blocks), dim3(kBlock), 0,
                     (hipStream_t)stream, A);
  return hipGetLastError() == hipSuccess ? NYX_OK : NYX_E_HIP;
}

}  // extern "C"
