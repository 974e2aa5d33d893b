// nyx_fill.hip -- ghost fill of one AMR level (Sec. 4.1 Mesh Hierarchy:
// ghost cells hold data for the update of a grid's valid cells; the regrid
// procedure of the same section: data not covered by the level come from the coarser level
// through limited piecewise linear profiles whose values at the fine cell
// centres conserve the coarse averages).
//
// The host plans the fill once per box layout: every ghost region of every
// box is cut into rectangles, each either a copy from one box of the same
// level (periodic images included) or, where no box of the level covers it,
// a row segment interpolated from one box of the coarser level.  The device
// walks the rectangles with one thread per ghost cell.  Built without
// contraction (the interpolation equals the CPU reference bit for bit).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "nyx_internal.h"

namespace nyx {

// One rectangle of ghost cells of box `dst` (box-local coordinates, ghosts
// negative or >= n).  Copy: the source cell of box `src` is local + shift.
// Interpolation: the global fine index is local + shift (already wrapped
// into the domain), the coarse cell is (global >> 1) - clo in coarse box
// `src`, and par[d] = global & 1 selects the child.
struct FillTag {
  int dst, src;
  int lo[3];
  int ext[3];
  int shift[3];
  int clo[3];
  FastDiv dx, dxy;  // division by ext[0] and ext[0] * ext[1]
};

struct FillArgs {
  const FillTag* tags;
  const int* prefix;     // cells before each tag, ntags + 1 entries
  const int* btag;       // per workgroup: the tag of its first cell
  int ntags;
  const BoxDev* fine;    // fine boxes
  const BoxDev* coarse;  // coarse boxes (interpolation)
  double* state;
  const double* cstate;
  const double* cstate_new;  // or nullptr: coarse data interpolated in time
  double theta;
  int ncomp;
};

// The tag of this thread's cell and the cell's box-local coordinates; false
// for lanes past the last cell.  Every lane takes one ghost cell of the
// concatenated tags, so small tags do not leave lanes idle; the host stored
// the tag of each workgroup's first cell, and a lane walks forward from it
// (a workgroup's 256 cells span few tags).
__device__ __forceinline__ bool fill_locate(const FillArgs& A, const FillTag** tag, int* loc) {
  const unsigned q = blockIdx.x * (unsigned)kBlock + threadIdx.x;
  if (q >= (unsigned)A.prefix[A.ntags]) return false;
  int lo = A.btag[blockIdx.x];
  while ((unsigned)A.prefix[lo + 1] <= q) ++lo;
  const FillTag& t = A.tags[lo];
  *tag = &t;
  const unsigned r = q - (unsigned)A.prefix[lo];
  const unsigned a = fast_div(r, t.dx), c = fast_div(r, t.dxy);
  loc[0] = t.lo[0] + (int)(r - a * (unsigned)t.ext[0]);
  loc[1] = t.lo[1] + (int)(a - c * (unsigned)t.ext[1]);
  loc[2] = t.lo[2] + (int)c;
  return true;
}

__device__ __forceinline__ unsigned fill_pidx(const BoxDev& b, int i, int j, int k) {
  return ((unsigned)(k + b.ng) * (unsigned)b.py + (unsigned)(j + b.ng)) * (unsigned)b.px +
         (unsigned)(i + b.ng);
}

__global__ __launch_bounds__(kBlock) void k_fill_copy(FillArgs A) {
  int loc[3];
  const FillTag* tp;
  if (!fill_locate(A, &tp, loc)) return;
  const FillTag& t = *tp;
  const BoxDev& D = A.fine[t.dst];
  const BoxDev& S = A.fine[t.src];
  const unsigned di = fill_pidx(D, loc[0], loc[1], loc[2]);
  const unsigned si = fill_pidx(S, loc[0] + t.shift[0], loc[1] + t.shift[1], loc[2] + t.shift[2]);
  for (int c = 0; c < A.ncomp; ++c)
    stu(A.state + D.soff + (long long)c * D.sstride, di,
        ldu(A.state + S.soff + (long long)c * S.sstride, si));
}

__device__ __forceinline__ double mc_slope(double um, double u0, double up) {
  const double dp = up - u0, dm = u0 - um;
  const double c = 0.5 * (dp + dm);
  if (dp * dm > 0.0) {
    double m = fabs(c);
    m = fmin(m, 2.0 * fabs(dp));
    m = fmin(m, 2.0 * fabs(dm));
    return c > 0.0 ? m : -m;
  }
  return 0.0;
}

__global__ __launch_bounds__(kBlock) void k_fill_interp(FillArgs A) {
  int loc[3];
  const FillTag* tp;
  if (!fill_locate(A, &tp, loc)) return;
  const FillTag& t = *tp;
  const BoxDev& D = A.fine[t.dst];
  const BoxDev& C = A.coarse[t.src];
  int X[3], par[3];
  for (int d = 0; d < 3; ++d) {
    const int g = loc[d] + t.shift[d];  // global fine index, in the domain
    X[d] = (g >> 1) - t.clo[d];
    par[d] = g & 1;
  }
  const unsigned di = fill_pidx(D, loc[0], loc[1], loc[2]);
  const unsigned c0 = fill_pidx(C, X[0], X[1], X[2]);
  const unsigned st[3] = {1u, (unsigned)C.px, (unsigned)C.px * (unsigned)C.py};
  // the coarse level is read-only here and lives apart from the fine state
  const double* __restrict__ cs = A.cstate;
  const double* __restrict__ cn = A.cstate_new;
  double* __restrict__ fs = A.state;
  const double th = A.theta;
  for (int c = 0; c < A.ncomp; ++c) {
    const long long co = C.soff + (long long)c * C.sstride;
    const double* u = cs + co;
    const double* un = cn ? cn + co : nullptr;
    // a coarse value, at the fraction theta of the coarse step when a new
    // state is given (subcycling)
    auto cv = [&](unsigned i) {
      return un ? ldu(u, i) + th * (ldu(un, i) - ldu(u, i)) : ldu(u, i);
    };
    const double u0 = cv(c0);
    double s[3], lo = u0, hi = u0;
    for (int d = 0; d < 3; ++d) {
      const double um = cv(c0 - st[d]);
      const double up = cv(c0 + st[d]);
      s[d] = mc_slope(um, u0, up);
      lo = fmin(lo, fmin(um, up));
      hi = fmax(hi, fmax(um, up));
    }
    const double ext = 0.25 * ((fabs(s[0]) + fabs(s[1])) + fabs(s[2]));
    double alpha = 1.0;
    if (ext > 0.0) {
      if (u0 + ext > hi) alpha = fmin(alpha, (hi - u0) / ext);
      if (u0 - ext < lo) alpha = fmin(alpha, (u0 - lo) / ext);
    }
    double v = 0.0;
    for (int d = 0; d < 3; ++d) v = v + (par[d] ? 0.25 : -0.25) * s[d];
    stu(fs + D.soff + (long long)c * D.sstride, di, u0 + alpha * v);
  }
}

}  // namespace nyx

// ---------------------------------------------------------------------------
// host planning and the C ABI
// ---------------------------------------------------------------------------
using namespace nyx;

struct nyx_fill_plan {
  int nbox = 0, ncoarse = 0;
  int ncopy = 0, ninterp = 0;
  long long copied = 0, interpolated = 0;
  int copy_blocks = 0, interp_blocks = 0;
  BoxDev* fine = nullptr;
  BoxDev* coarse = nullptr;
  FillTag* copy_tags = nullptr;
  FillTag* interp_tags = nullptr;
  int* copy_prefix = nullptr;
  int* interp_prefix = nullptr;
  int* copy_btag = nullptr;
  int* interp_btag = nullptr;
  size_t state_span = 0, cstate_span = 0;
};

namespace {

size_t r256(size_t x) { return (x + 255) / 256 * 256; }

struct HostPlan {
  std::vector<BoxDev> fine, coarse;
  std::vector<FillTag> copy, interp;
  std::vector<int> copy_prefix, interp_prefix;
  std::vector<int> copy_btag, interp_btag;
  long long copied = 0, interpolated = 0;
  size_t state_span = 0, cstate_span = 0;
};

int wrapi(int x, int m) {
  const int r = x % m;
  return r < 0 ? r + m : r;
}

FillTag make_tag(int dst, int src, const int* lo, const int* ext, const int* shift,
                 const int* clo) {
  FillTag t{};
  t.dst = dst;
  t.src = src;
  for (int d = 0; d < 3; ++d) {
    t.lo[d] = lo[d];
    t.ext[d] = ext[d];
    t.shift[d] = shift[d];
    t.clo[d] = clo ? clo[d] : 0;
  }
  t.dx = make_fastdiv((unsigned)ext[0]);
  t.dxy = make_fastdiv((unsigned)ext[0] * (unsigned)ext[1]);
  return t;
}

// the tag holding the first cell of each workgroup of a launch over the
// prefix's cells
void block_tags(const std::vector<int>& pre, std::vector<int>& btag) {
  const int ntags = (int)pre.size() - 1;
  const int nblocks = (pre.back() + kBlock - 1) / kBlock;
  btag.assign(std::max(nblocks, 1), 0);
  int t = 0;
  for (int b = 0; b < nblocks; ++b) {
    const int q = b * kBlock;
    while (t + 1 < ntags && pre[t + 1] <= q) ++t;
    btag[b] = t;
  }
}

// cells before each tag; the launch covers prefix.back() cells
int prefix_of(const std::vector<FillTag>& tags, std::vector<int>& pre) {
  pre.assign(tags.size() + 1, 0);
  long long acc = 0;
  for (size_t i = 0; i < tags.size(); ++i) {
    pre[i] = (int)acc;
    acc += (long long)tags[i].ext[0] * tags[i].ext[1] * tags[i].ext[2];
    if (acc > (1ll << 31) - 1 - kBlock) return NYX_E_SHAPE;
  }
  pre[tags.size()] = (int)acc;
  return NYX_OK;
}

// Merge interpolation rows into rectangles: a row continues the previous
// tag along y (then along z) when it has the same box, coarse box, x range
// and index shifts (the same periodic image).
void merge_rows(std::vector<FillTag>& tags) {
  for (int axis = 1; axis <= 2; ++axis) {
    std::vector<FillTag> out;
    out.reserve(tags.size());
    for (const FillTag& t : tags) {
      bool merged = false;
      if (!out.empty()) {
        FillTag& u = out.back();
        const int o = 3 - axis;  // the other transverse axis
        merged = u.dst == t.dst && u.src == t.src && u.lo[0] == t.lo[0] && u.ext[0] == t.ext[0] &&
                 u.lo[o] == t.lo[o] && u.ext[o] == t.ext[o] &&
                 u.lo[axis] + u.ext[axis] == t.lo[axis] && u.shift[0] == t.shift[0] &&
                 u.shift[1] == t.shift[1] && u.shift[2] == t.shift[2];
        if (merged) u.ext[axis] += t.ext[axis];
      }
      if (!merged) out.push_back(t);
    }
    tags.swap(out);
    if (axis == 1) {
      // reorder so that equal rectangles of consecutive planes are adjacent
      std::stable_sort(tags.begin(), tags.end(), [](const FillTag& a, const FillTag& b) {
        if (a.dst != b.dst) return a.dst < b.dst;
        if (a.lo[1] != b.lo[1]) return a.lo[1] < b.lo[1];
        if (a.lo[0] != b.lo[0]) return a.lo[0] < b.lo[0];
        return a.lo[2] < b.lo[2];
      });
    }
  }
  for (FillTag& t : tags) {
    t.dx = make_fastdiv((unsigned)t.ext[0]);
    t.dxy = make_fastdiv((unsigned)t.ext[0] * (unsigned)t.ext[1]);
  }
}

int check_level(int nbox, const nyx_box* boxes, const int32_t* lo, const int32_t* dom) {
  if (nbox < 1 || nbox > (1 << 20)) return NYX_E_SHAPE;
  if (!boxes || !lo || !dom) return NYX_E_NULL;
  for (int d = 0; d < 3; ++d)
    if (dom[d] < 2 || (dom[d] & 1) || dom[d] > (1 << 24)) return NYX_E_SHAPE;
  const int ng = boxes[0].ng;
  for (int d = 0; d < 3; ++d)
    if (dom[d] < ng) return NYX_E_SHAPE;  // ghost regions reach at most one periodic image
  for (int b = 0; b < nbox; ++b) {
    int rc = validate_box(&boxes[b]);
    if (rc) return rc;
    if (boxes[b].ng != ng) return NYX_E_SHAPE;
    for (int d = 0; d < 3; ++d)
      if (lo[3 * b + d] < 0 || lo[3 * b + d] + boxes[b].n[d] > dom[d]) return NYX_E_SHAPE;
  }
  return NYX_OK;
}

// Build the tags.  Returns NYX_E_SHAPE for overlapping valid regions or a
// ghost cell covered by neither level.
int plan_level(int nbox, const nyx_box* boxes, const int32_t* lo, const int32_t* dom,
               int ncoarse, const nyx_box* cboxes, const int32_t* clo, HostPlan& H) {
  int rc = check_level(nbox, boxes, lo, dom);
  if (rc) return rc;
  int cdom[3] = {dom[0] / 2, dom[1] / 2, dom[2] / 2};
  if (ncoarse > 0) {
    if ((rc = check_level(ncoarse, cboxes, clo, cdom))) return rc;
    // the interpolation reads one coarse ghost layer
  } else if (ncoarse < 0) {
    return NYX_E_SHAPE;
  }
  H.fine.resize(nbox);
  for (int b = 0; b < nbox; ++b) {
    box_layout(boxes[b], b, 0, &H.fine[b]);
    const size_t end = (size_t)(boxes[b].state_off + 5 * boxes[b].comp_stride + H.fine[b].P);
    H.state_span = std::max(H.state_span, end);
  }
  H.coarse.resize(ncoarse);
  for (int b = 0; b < ncoarse; ++b) {
    box_layout(cboxes[b], b, 0, &H.coarse[b]);
    const size_t end = (size_t)(cboxes[b].state_off + 5 * cboxes[b].comp_stride + H.coarse[b].P);
    H.cstate_span = std::max(H.cstate_span, end);
  }
  // valid regions must not overlap
  for (int a = 0; a < nbox; ++a)
    for (int b = a + 1; b < nbox; ++b) {
      bool ov = true;
      for (int d = 0; d < 3; ++d)
        ov = ov && lo[3 * a + d] < lo[3 * b + d] + boxes[b].n[d] &&
             lo[3 * b + d] < lo[3 * a + d] + boxes[a].n[d];
      if (ov) return NYX_E_SHAPE;
    }
  // coarse cell -> box map over the coarse domain (for the interpolation)
  std::vector<int> cmap;
  if (ncoarse > 0) {
    cmap.assign((size_t)cdom[0] * cdom[1] * cdom[2], -1);
    for (int c = 0; c < ncoarse; ++c)
      for (int k = 0; k < cboxes[c].n[2]; ++k)
        for (int j = 0; j < cboxes[c].n[1]; ++j)
          for (int i = 0; i < cboxes[c].n[0]; ++i)
            cmap[((size_t)(clo[3 * c + 2] + k) * cdom[1] + (clo[3 * c + 1] + j)) * cdom[0] +
                 (clo[3 * c] + i)] = c;
  }
  for (int b = 0; b < nbox; ++b) {
    const int ng = boxes[b].ng;
    const int* n = boxes[b].n;
    const int* L = lo + 3 * b;
    const int gx = n[0] + 2 * ng, gy = n[1] + 2 * ng, gz = n[2] + 2 * ng;
    std::vector<unsigned char> covered((size_t)gx * gy * gz, 0);
    auto cov = [&](int i, int j, int k) -> unsigned char& {
      return covered[((size_t)(k + ng) * gy + (j + ng)) * gx + (i + ng)];
    };
    for (int k = 0; k < n[2]; ++k)
      for (int j = 0; j < n[1]; ++j)
        for (int i = 0; i < n[0]; ++i) cov(i, j, k) = 1;
    // copies: the grown box against every box's valid region and its images
    for (int s = 0; s < nbox; ++s) {
      // per axis, the intersections of the grown extent with the source's
      // valid extent shifted by -dom, 0, +dom (image index im)
      int ilo[3][3], ihi[3][3], iim[3][3], nsh[3];
      for (int d = 0; d < 3; ++d) {
        nsh[d] = 0;
        for (int m = -1; m <= 1; ++m) {
          const int slo = lo[3 * s + d] + m * dom[d], shi = slo + boxes[s].n[d];
          const int a = std::max(L[d] - ng, slo), e = std::min(L[d] + n[d] + ng, shi);
          if (a < e) {
            ilo[d][nsh[d]] = a;
            ihi[d][nsh[d]] = e;
            iim[d][nsh[d]] = m;
            nsh[d]++;
          }
        }
      }
      for (int p = 0; p < nsh[0]; ++p)
        for (int q = 0; q < nsh[1]; ++q)
          for (int r = 0; r < nsh[2]; ++r) {
            const int glo[3] = {ilo[0][p], ilo[1][q], ilo[2][r]};
            const int ghi[3] = {ihi[0][p], ihi[1][q], ihi[2][r]};
            const int im[3] = {iim[0][p], iim[1][q], iim[2][r]};
            int llo[3], ext[3], shift[3];
            for (int d = 0; d < 3; ++d) {
              llo[d] = glo[d] - L[d];
              ext[d] = ghi[d] - glo[d];
              // box-local in the destination -> box-local in the source image
              shift[d] = L[d] - im[d] * dom[d] - lo[3 * s + d];
            }
            if (s == b && shift[0] == 0 && shift[1] == 0 && shift[2] == 0) continue;  // own cells
            H.copy.push_back(make_tag(b, s, llo, ext, shift, nullptr));
            for (int k = llo[2]; k < llo[2] + ext[2]; ++k)
              for (int j = llo[1]; j < llo[1] + ext[1]; ++j)
                for (int i = llo[0]; i < llo[0] + ext[0]; ++i) cov(i, j, k) = 1;
            H.copied += (long long)ext[0] * ext[1] * ext[2];
          }
    }
    // the rest: row segments interpolated from the coarse level
    for (int k = -ng; k < n[2] + ng; ++k)
      for (int j = -ng; j < n[1] + ng; ++j) {
        int i = -ng;
        while (i < n[0] + ng) {
          if (cov(i, j, k)) {
            ++i;
            continue;
          }
          if (ncoarse == 0) return NYX_E_SHAPE;
          // a segment with one coarse box and one wrap of the global index
          const int gj = wrapi(L[1] + j, dom[1]), gk = wrapi(L[2] + k, dom[2]);
          const int off_x = wrapi(L[0] + i, dom[0]) - (L[0] + i);
          int c = -1, i0 = i;
          while (i < n[0] + ng && !cov(i, j, k)) {
            const int gi = L[0] + i + off_x;
            if (gi < 0 || gi >= dom[0]) break;  // the wrap changes: new segment
            const int cc = cmap[((size_t)(gk >> 1) * cdom[1] + (gj >> 1)) * cdom[0] + (gi >> 1)];
            if (cc < 0) return NYX_E_SHAPE;
            if (c >= 0 && cc != c) break;
            c = cc;
            ++i;
          }
          const int llo[3] = {i0, j, k};
          const int ext[3] = {i - i0, 1, 1};
          const int shift[3] = {L[0] + off_x, gj - j, gk - k};
          // the coarse cell is a valid cell of box c (the map says so), so its
          // face neighbours lie in c's padded region (ghost width >= 4)
          H.interp.push_back(make_tag(b, c, llo, ext, shift, clo + 3 * c));
          H.interpolated += ext[0];
        }
      }
  }
  merge_rows(H.interp);
  if ((rc = prefix_of(H.copy, H.copy_prefix))) return rc;
  if ((rc = prefix_of(H.interp, H.interp_prefix))) return rc;
  block_tags(H.copy_prefix, H.copy_btag);
  block_tags(H.interp_prefix, H.interp_btag);
  return NYX_OK;
}

size_t plan_bytes(const HostPlan& H) {
  return r256(sizeof(BoxDev) * H.fine.size()) + r256(sizeof(BoxDev) * std::max<size_t>(H.coarse.size(), 1)) +
         r256(sizeof(FillTag) * std::max<size_t>(H.copy.size(), 1)) +
         r256(sizeof(FillTag) * std::max<size_t>(H.interp.size(), 1)) +
         r256(sizeof(int) * H.copy_prefix.size()) + r256(sizeof(int) * H.interp_prefix.size()) +
         r256(sizeof(int) * H.copy_btag.size()) + r256(sizeof(int) * H.interp_btag.size());
}

}  // namespace

extern "C" {

int nyx_fill_plan_bytes(int nbox, const nyx_box* boxes, const int32_t* lo, const int32_t* dom,
                        int ncoarse, const nyx_box* cboxes, const int32_t* clo, size_t* bytes) {
  if (!bytes) return NYX_E_NULL;
  HostPlan H;
  int rc = plan_level(nbox, boxes, lo, dom, ncoarse, cboxes, clo, H);
  if (rc) return rc;
  *bytes = plan_bytes(H);
  return NYX_OK;
}

int nyx_fill_plan_create(int nbox, const nyx_box* boxes, const int32_t* lo, const int32_t* dom,
                         int ncoarse, const nyx_box* cboxes, const int32_t* clo, void* workspace,
                         size_t ws_bytes, void* stream, nyx_fill_plan** out) {
  if (!out || !workspace) return NYX_E_NULL;
  *out = nullptr;
  if ((uintptr_t)workspace & 255) return NYX_E_WORKSPACE;
  HostPlan H;
  int rc = plan_level(nbox, boxes, lo, dom, ncoarse, cboxes, clo, H);
  if (rc) return rc;
  if (ws_bytes < plan_bytes(H)) return NYX_E_WORKSPACE;
  nyx_fill_plan* p = new (std::nothrow) nyx_fill_plan;
  if (!p) return NYX_E_HIP;
  char* w = (char*)workspace;
  p->fine = (BoxDev*)w;
  w += r256(sizeof(BoxDev) * H.fine.size());
  p->coarse = (BoxDev*)w;
  w += r256(sizeof(BoxDev) * std::max<size_t>(H.coarse.size(), 1));
  p->copy_tags = (FillTag*)w;
  w += r256(sizeof(FillTag) * std::max<size_t>(H.copy.size(), 1));
  p->interp_tags = (FillTag*)w;
  w += r256(sizeof(FillTag) * std::max<size_t>(H.interp.size(), 1));
  p->copy_prefix = (int*)w;
  w += r256(sizeof(int) * H.copy_prefix.size());
  p->interp_prefix = (int*)w;
  w += r256(sizeof(int) * H.interp_prefix.size());
  p->copy_btag = (int*)w;
  w += r256(sizeof(int) * H.copy_btag.size());
  p->interp_btag = (int*)w;
  p->nbox = nbox;
  p->ncoarse = ncoarse;
  p->ncopy = (int)H.copy.size();
  p->ninterp = (int)H.interp.size();
  p->copied = H.copied;
  p->interpolated = H.interpolated;
  p->copy_blocks = (H.copy_prefix.back() + kBlock - 1) / kBlock;
  p->interp_blocks = (H.interp_prefix.back() + kBlock - 1) / kBlock;
  p->state_span = H.state_span;
  p->cstate_span = H.cstate_span;
  hipStream_t s = (hipStream_t)stream;
  bool ok = hipMemcpyAsync(p->fine, H.fine.data(), sizeof(BoxDev) * H.fine.size(),
                           hipMemcpyHostToDevice, s) == hipSuccess;
  if (ok && !H.coarse.empty())
    ok = hipMemcpyAsync(p->coarse, H.coarse.data(), sizeof(BoxDev) * H.coarse.size(),
                        hipMemcpyHostToDevice, s) == hipSuccess;
  if (ok && !H.copy.empty())
    ok = hipMemcpyAsync(p->copy_tags, H.copy.data(), sizeof(FillTag) * H.copy.size(),
                        hipMemcpyHostToDevice, s) == hipSuccess;
  if (ok && !H.interp.empty())
    ok = hipMemcpyAsync(p->interp_tags, H.interp.data(), sizeof(FillTag) * H.interp.size(),
                        hipMemcpyHostToDevice, s) == hipSuccess;
  if (ok)
    ok = hipMemcpyAsync(p->copy_prefix, H.copy_prefix.data(), sizeof(int) * H.copy_prefix.size(),
                        hipMemcpyHostToDevice, s) == hipSuccess;
  if (ok)
    ok = hipMemcpyAsync(p->interp_prefix, H.interp_prefix.data(),
                        sizeof(int) * H.interp_prefix.size(), hipMemcpyHostToDevice, s) == hipSuccess;
  if (ok)
    ok = hipMemcpyAsync(p->copy_btag, H.copy_btag.data(), sizeof(int) * H.copy_btag.size(),
                        hipMemcpyHostToDevice, s) == hipSuccess;
  if (ok)
    ok = hipMemcpyAsync(p->interp_btag, H.interp_btag.data(), sizeof(int) * H.interp_btag.size(),
                        hipMemcpyHostToDevice, s) == hipSuccess;
  // the host vectors die with this call: the copies must have completed
  if (ok) ok = hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    delete p;
    return NYX_E_HIP;
  }
  *out = p;
  return NYX_OK;
}

int nyx_fill_plan_destroy(nyx_fill_plan* plan) {
  delete plan;
  return NYX_OK;
}

int nyx_fill_plan_counts(const nyx_fill_plan* plan, long long* copied, long long* interpolated) {
  if (!plan) return NYX_E_NULL;
  if (copied) *copied = plan->copied;
  if (interpolated) *interpolated = plan->interpolated;
  return NYX_OK;
}

int nyx_fill_level(nyx_fill_plan* plan, double* state, const double* coarse_state, int ncomp,
                   void* stream) {
  return nyx_fill_level_time(plan, state, coarse_state, nullptr, 0.0, ncomp, stream);
}

int nyx_fill_level_time(nyx_fill_plan* plan, double* state, const double* coarse_state,
                        const double* coarse_state_new, double theta, int ncomp, void* stream) {
  if (!plan || !state) return NYX_E_NULL;
  if (ncomp < 1 || ncomp > 16) return NYX_E_PARAM;
  if (plan->ninterp > 0 && !coarse_state) return NYX_E_NULL;
  if (coarse_state_new && !(theta >= 0.0 && theta <= 1.0)) return NYX_E_PARAM;
  hipStream_t s = (hipStream_t)stream;
  FillArgs A{};
  A.fine = plan->fine;
  A.coarse = plan->coarse;
  A.state = state;
  A.cstate = coarse_state;
  A.cstate_new = coarse_state_new;
  A.theta = theta;
  A.ncomp = ncomp;
  if (plan->ncopy > 0) {
    A.tags = plan->copy_tags;
    A.prefix = plan->copy_prefix;
    A.btag = plan->copy_btag;
    A.ntags = plan->ncopy;
    hipLaunchKernelGGL(k_fill_copy, dim3(plan->copy_blocks), dim3(kBlock), 0, s, A);
    if (hipGetLastError() != hipSuccess) return NYX_E_HIP;
  }
  if (plan->ninterp > 0) {
    A.tags = plan->interp_tags;
    A.prefix = plan->interp_prefix;
    A.btag = plan->interp_btag;
    A.ntags = plan->ninterp;
    hipLaunchKernelGGL(k_fill_interp, dim3(plan->interp_blocks), dim3(kBlock), 0, s, A);
    if (hipGetLastError() != hipSuccess) return NYX_E_HIP;
  }
  return NYX_OK;
}

}  // extern "C"
