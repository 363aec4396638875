// capi.cpp -- C ABI and host runtime of libhydro (see include/hydro.h).
//
// The runtime validates descriptors, lays out the caller's workspace,
// chooses a kernel configuration per sweep axis (built-in default, forced
// text, cached autotune result, or a timing search), builds the batched
// work lists, captures the even/odd step graphs and enqueues steps on the
// caller's stream.  It never allocates device memory.
#include <hip/hip_runtime.h>
#include <sys/stat.h>

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/hydro.h"
#include "launch.hpp"
#include "layout.hpp"

using namespace hydro;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(HYDRO_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kScalarBytes = 256;
constexpr int kReduceBlock = 256;
constexpr int kMaxChunks = 1024;
constexpr int kBatchChunks = 4;
constexpr int kMaxBlock = 512;  // launch bound of the sweep kernels
static_assert(sizeof(DevScalars) <= kScalarBytes, "scalar block");

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int chunks_for(int64_t cells) {
  int64_t c = (cells + int64_t(kReduceBlock) * 8 - 1) / (int64_t(kReduceBlock) * 8);
  return int(std::max<int64_t>(1, std::min<int64_t>(kMaxChunks, c)));
}

// ------------------------------------------------------------------------
// descriptor checks
// ------------------------------------------------------------------------

int check_common(const hydro_desc* d) {
  if (!d) return fail(HYDRO_EINVAL, "null descriptor");
  if (!(d->gamma > 1.0) || !std::isfinite(d->gamma)) return fail(HYDRO_EINVAL, "gamma must be > 1");
  if (!(d->cfl > 0.0 && d->cfl <= 1.0)) return fail(HYDRO_EINVAL, "cfl must be in (0, 1]");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(d->grav[a])) return fail(HYDRO_EINVAL, "gravity must be finite");
  for (int a = 0; a < 3; ++a) {
    int lo = d->bc[2 * a], hi = d->bc[2 * a + 1];
    if (lo < 0 || lo > 2 || hi < 0 || hi > 2) return fail(HYDRO_EINVAL, "unknown boundary condition");
    if ((lo == HYDRO_BC_PERIODIC) != (hi == HYDRO_BC_PERIODIC))
      return fail(HYDRO_EINVAL, "periodic boundary set on one side only");
  }
  if (d->precision != HYDRO_FP32 && d->precision != HYDRO_FP64)
    return fail(HYDRO_EINVAL, "unknown precision");
  return HYDRO_OK;
}

int check_extent(const int32_t n[3], int32_t ng, const double dx[3]) {
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1) return fail(HYDRO_EINVAL, "cell counts must be >= 1");
    if (n[a] == 1) continue;  // inactive axis
    if (n[a] > (1 << 24)) return fail(HYDRO_EINVAL, "axis too long");
  }
  for (int a = 0; a < 3; ++a)
    if (!finite_pos(dx[a])) return fail(HYDRO_EINVAL, "cell widths must be > 0");
  if (ng < 0 || ng > 64) return fail(HYDRO_EINVAL, "ghost layers must be in [0, 64]");
  return HYDRO_OK;
}

PatchDev make_patch(const int32_t n[3], int32_t ng, const double dx[3], int64_t offset) {
  PatchDev P;
  int64_t sx = n[0] + 2 * ng, sy = n[1] + 2 * ng, sz = n[2] + 2 * ng;
  P.plane = sx * sy * sz;
  P.sy = int32_t(sx);
  P.sz = int32_t(sx * sy);
  P.base0 = offset + ng + ng * sx + ng * sx * sy;
  P.ng = ng;
  for (int a = 0; a < 3; ++a) {
    P.n[a] = n[a];
    P.dx[a] = dx[a];
    P.idx[a] = n[a] > 1 ? 1.0 / dx[a] : 0.0;
  }
  return P;
}

// The sweep kernels address a plane with 32-bit byte offsets from its
// interior origin, up to one z layer past the last cell (a column march's
// clamped prefetch steps there before clamping).
bool plane_fits(const PatchDev& P, int64_t esz) {
  return (P.plane + int64_t(P.sz)) * esz < (int64_t(1) << 32);
}

// Patch geometry from a hydro_patch (defaults or explicit pitches); returns
// false on an inconsistent layout.  *len receives the elements the patch
// spans in the pool (5 planes).
bool patch_from(const hydro_patch& p, PatchDev* out, int64_t* len) {
  const int32_t n[3] = {p.nx, p.ny, p.nz};
  const double dx[3] = {p.dx, p.dy, p.dz};
  const int64_t ng = p.ng;
  const int64_t rp = p.row_pitch ? p.row_pitch : n[0] + 2 * ng;
  const int64_t sp = p.slab_pitch ? p.slab_pitch : rp * (n[1] + 2 * ng);
  const int64_t pp = p.plane_pitch ? p.plane_pitch : sp * (n[2] + 2 * ng);
  const int64_t io = p.interior_offset ? p.interior_offset : ng * (1 + rp + sp);
  if (rp < n[0] + 2 * ng || sp < rp * (n[1] + 2 * ng) || pp < sp * (n[2] + 2 * ng))
    return false;
  if (io < ng * (1 + rp + sp)) return false;
  // the last stored cell of a plane (interior plus ng beyond) inside the plane
  const int64_t lastc = io + (n[0] - 1 + ng) + (n[1] - 1 + ng) * rp + (n[2] - 1 + ng) * sp;
  if (lastc >= pp) return false;
  if (rp > INT32_MAX || sp > INT32_MAX) return false;
  PatchDev P;
  P.plane = pp;
  P.sy = int32_t(rp);
  P.sz = int32_t(sp);
  P.base0 = p.offset_elems + io;
  P.ng = p.ng;
  for (int a = 0; a < 3; ++a) {
    P.n[a] = n[a];
    P.dx[a] = dx[a];
    P.idx[a] = n[a] > 1 ? 1.0 / dx[a] : 0.0;
  }
  *out = P;
  *len = 5 * pp;
  return true;
}

// ------------------------------------------------------------------------
// kernel configurations
// ------------------------------------------------------------------------

struct Config {
  SweepCfg ax[3];
  int32_t batch_blocks = 0;  // persistent launches: workgroups
  int32_t batch_dyn = 1;     // persistent launches: ticket (1) or static (0) items
  int32_t batch_fuse = 0;    // batches: x and y sweeps fused per patch z-plane (1)
  int32_t batch_zplane = 0;  // batches: z swept as lane runs over x-z planes in LDS (1)
  SweepCfg plane{kLaneRunKind, 4, 512, 0, 0, 0};  // fused plane kernel: V, threads
  SweepCfg zplane{kLaneRunKind, 2, 512, 0, 0, 0};  // x-z plane kernel: V, threads
};

// A lane run of v cells is loaded and stored as one vector access, so every
// row of the patch must start on a multiple of the vector's element count
// (the pool itself is 16-byte aligned).
bool x_cfg_ok(const SweepCfg& c, const PatchDev& P, int fp64) {
  if (c.kind != kLaneRunKind && c.kind != kXMarchKind) return false;
  if (c.v != 1 && c.v != 2 && c.v != 4) return false;
  const int nx = P.n[0];
  if (nx % c.v) return false;
  int lpp = nx / c.v;
  if (c.block < 64 || c.block > kMaxBlock || c.block % 64) return false;
  if (c.kind == kLaneRunKind && lpp > 64 && c.block % (64 * ((lpp + 63) / 64)))
    return false;  // whole pencils per workgroup
  if (c.kind == kXMarchKind && fp64 && c.v == 4) return false;  // not built (spills)
  if (c.kind == kLaneRunKind && c.q != 0) return false;            // no grid cap
  if (c.q < 0) return false;
  if (x_pencils_per_tile(P, c) < 1) return false;
  const int esz = fp64 ? 8 : 4;
  const int a = std::min(c.v, 16 / esz);
  if (P.base0 % a || P.sy % a || P.sz % a || P.plane % a) return false;
  return true;
}

bool x_cfg_ok_all(const SweepCfg& c, const std::vector<PatchDev>& ps, int fp64) {
  for (auto& P : ps)
    if (!x_cfg_ok(c, P, fp64)) return false;
  return true;
}

bool col_cfg_ok(const SweepCfg& c) {
  if (c.kind != kColumnKind || c.q < 1 || c.s < 1) return false;
  int b = c.q * c.s;
  return b >= 64 && b <= kMaxBlock && b % 64 == 0 && c.q % 64 == 0 && c.s <= 16;
}

SweepCfg default_x(const std::vector<PatchDev>& ps, int fp64) {
  SweepCfg c{};
  c.kind = kLaneRunKind;
  for (int v : {4, 2, 1}) {
    c.v = v;
    int lpp = 1;
    for (auto& P : ps) lpp = std::max(lpp, P.n[0] / v);
    const int wpp = (lpp + 63) / 64;      // waves per pencil
    c.block = 64 * wpp * std::max(1, 4 / wpp);
    if (c.block > kMaxBlock) c.block = 64 * wpp;
    if (x_cfg_ok_all(c, ps, fp64)) return c;
  }
  c.v = 0;  // none fits
  return c;
}

SweepCfg default_col(int n) {
  SweepCfg c{};
  c.kind = kColumnKind;
  c.q = 64;
  int s = (n + 63) / 64;
  c.s = std::max(1, std::min(kMaxBlock / c.q, s));
  return c;
}

std::string cfg_text(const Config& cf) {
  std::ostringstream o;
  o << "x:v=" << cf.ax[0].v << ",b=" << cf.ax[0].block;
  if (cf.ax[0].kind == kXMarchKind) {
    o << ",m=1";
    if (cf.ax[0].q) o << ",g=" << cf.ax[0].q;
  }
  o << ";y:q=" << cf.ax[1].q << ",s=" << cf.ax[1].s;
  o << ";z:q=" << cf.ax[2].q << ",s=" << cf.ax[2].s;
  if (cf.batch_blocks) {
    o << ";p:g=" << cf.batch_blocks << ",d=" << cf.batch_dyn << ",f=" << cf.batch_fuse;
    if (cf.batch_zplane) o << ",z=1";
    if (cf.batch_fuse) o << ";w:v=" << cf.plane.v << ",b=" << cf.plane.block;
    if (cf.batch_zplane) o << ";u:v=" << cf.zplane.v << ",b=" << cf.zplane.block;
  } else if (cf.batch_fuse) {
    o << ";p:f=1;w:v=" << cf.plane.v << ",b=" << cf.plane.block;  // single grid, fused x+y
  }
  return o.str();
}

// parse "x:v=4,b=256[,m=1];y:q=64,s=4;z:q=64,s=2;p:g=2048" (any subset) into
// cf; m=1 selects the chunked x march, m=0 (or no m) the lane-run x sweep
bool parse_cfg(const std::string& text, Config& cf) {
  std::stringstream ss(text);
  std::string part;
  while (std::getline(ss, part, ';')) {
    if (part.empty()) continue;
    if (part.size() < 3 || part[1] != ':') return false;
    char ax = part[0];
    if (ax == 'x') {
      cf.ax[0].kind = kLaneRunKind;
      cf.ax[0].q = 0;
    }
    std::stringstream kv(part.substr(2));
    std::string item;
    while (std::getline(kv, item, ',')) {
      auto eq = item.find('=');
      if (eq == std::string::npos) return false;
      std::string k = item.substr(0, eq);
      char* end = nullptr;
      long v = std::strtol(item.c_str() + eq + 1, &end, 10);
      if (!end || *end) return false;
      if (ax == 'x') {
        if (k == "v") cf.ax[0].v = int(v);
        else if (k == "b") cf.ax[0].block = int(v);
        else if (k == "m" && (v == 0 || v == 1)) cf.ax[0].kind = v ? kXMarchKind : kLaneRunKind;
        else if (k == "g" && v >= 0 && v <= (1 << 24)) cf.ax[0].q = int(v);
        else return false;
      } else if (ax == 'y' || ax == 'z') {
        SweepCfg& c = cf.ax[ax == 'y' ? 1 : 2];
        if (k == "q") c.q = int(v);
        else if (k == "s") c.s = int(v);
        else return false;
      } else if (ax == 'w') {
        if (k == "v") cf.plane.v = int(v);
        else if (k == "b") cf.plane.block = int(v);
        else return false;
      } else if (ax == 'u') {
        if (k == "v") cf.zplane.v = int(v);
        else if (k == "b") cf.zplane.block = int(v);
        else return false;
      } else if (ax == 'p') {
        if (k == "g") cf.batch_blocks = int(v);
        else if (k == "d" && (v == 0 || v == 1)) cf.batch_dyn = int(v);
        else if (k == "f" && (v == 0 || v == 1)) cf.batch_fuse = int(v);
        else if (k == "z" && (v == 0 || v == 1)) cf.batch_zplane = int(v);
        else return false;
      } else {
        return false;
      }
    }
  }
  return true;
}

// ------------------------------------------------------------------------
// autotune cache (flat JSON object of string -> string)
// ------------------------------------------------------------------------

std::mutex g_cache_mu;

std::string cache_path() {
  const char* p = std::getenv("HYDRO_TUNE_CACHE");
  if (p && *p) return p;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/hydro_mi355x_tune.json";
}

std::map<std::string, std::string> cache_read() {
  std::map<std::string, std::string> m;
  std::ifstream f(cache_path());
  if (!f) return m;
  std::stringstream buf;
  buf << f.rdbuf();
  std::string s = buf.str();
  size_t i = 0;
  auto str = [&](std::string& out) {
    while (i < s.size() && s[i] != '"') ++i;
    if (i >= s.size()) return false;
    size_t j = s.find('"', i + 1);
    if (j == std::string::npos) return false;
    out = s.substr(i + 1, j - i - 1);
    i = j + 1;
    return true;
  };
  std::string k, v;
  while (str(k) && str(v)) m[k] = v;
  return m;
}

void cache_write(const std::map<std::string, std::string>& m) {
  std::string path = cache_path();
  size_t slash = path.find_last_of('/');
  if (slash != std::string::npos && slash > 0) {
    // create the cache directory if missing (best effort, one level)
    ::mkdir(path.substr(0, slash).c_str(), 0755);
  }
  std::string tmp = path + ".tmp";
  std::ofstream f(tmp);
  if (!f) return;
  f << "{\n";
  size_t i = 0;
  for (auto& kv : m) {
    f << "  \"" << kv.first << "\": \"" << kv.second << "\"" << (++i < m.size() ? "," : "")
      << "\n";
  }
  f << "}\n";
  f.close();
  std::rename(tmp.c_str(), path.c_str());
}

}  // namespace

// ------------------------------------------------------------------------
// context
// ------------------------------------------------------------------------

struct hydro_ctx {
  hydro_desc desc{};
  bool batch = false;
  int fp64 = 0;
  void* pool = nullptr;
  size_t pool_bytes = 0;     // size of the state (grid) or pool (batch) buffer
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  DevScalars* scal = nullptr;
  double* partials = nullptr;          // totals partials (fused and standalone)
  double* tslice = nullptr;            // first level of the totals reduction
  double* profile_partials = nullptr;  // single grid: slab profile partial sums
  PatchDev single{};
  // batch
  int32_t npatch = 0;
  std::vector<PatchDev> patches;
  PatchDev* d_patches = nullptr;
  // single grid, fused x+y step (HYDRO_FLAG_FUSE_XY): the windows of a
  // z-plane and a second buffer laid out like the state (null: not eligible)
  WinDev* d_wins = nullptr;
  int32_t nwin = 0;
  void* shadow = nullptr;
  // x, y, z, z-planes (fused x+y), x-z planes (z in LDS)
  WorkItem* d_items[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int32_t nitems[5] = {0, 0, 0, 0, 0};
  int64_t max_patch_cells = 0;
  // run state
  int64_t step = 0;
  double t_host = 0.0;
  double t_end = 0.0;
  bool dt_valid = false;
  bool totals_valid = false;  // scal->totals hold the totals of the current state
  // HYDRO_BATCH_PER_PATCH_DT: patch p has its own time pt[p] and dt pdt[p],
  // and its sweeps fold their CFL maximum into psmax[p]; pp_live turns this
  // off while the tuner times sweeps with dt = 0
  bool per_patch = false;
  bool pp_live = false;
  double* pt = nullptr;
  double* pdt = nullptr;
  unsigned long long* psmax = nullptr;
  Config cfg;
  Config items_cfg;          // configuration the batch work lists were built for
  bool active[3] = {false, false, false};
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int cu_count = 0;
  std::string arch;
};

namespace {

int rebuild_items(hydro_ctx* c);

// The persistent sweeps read (patch, tile) lists whose tiles depend on the
// configuration; launching with lists built for another configuration would
// silently skip or repeat work, so every batched launch path checks this.
bool items_current(const hydro_ctx* c) {
  return !c->batch || std::memcmp(c->items_cfg.ax, c->cfg.ax, sizeof(c->cfg.ax)) == 0;
}

constexpr int64_t kTotCellsPerBlock = 24576;

LaunchSweep sweep_launch(const hydro_ctx* c, int axis, int do_cfl) {
  LaunchSweep L{};
  L.pool = c->pool;
  L.patches = c->d_patches;
  L.single = c->single;
  L.items = c->d_items[axis];
  L.nitems = c->nitems[axis];
  L.nblocks = c->cfg.batch_blocks;
  L.dyn = c->cfg.batch_dyn;
  L.axis = axis;
  L.bc_lo = c->desc.bc[2 * axis];
  L.bc_hi = c->desc.bc[2 * axis + 1];
  L.do_cfl = do_cfl;
  L.grav = c->desc.grav[axis];
  for (int a = 0; a < 3; ++a) L.gvec[a] = c->desc.grav[a];
  L.gamma = c->desc.gamma;
  L.scal = c->scal;
  L.cfg = c->cfg.ax[axis];
  L.persistent = c->batch ? 1 : 0;
  L.fp64 = c->fp64;
  // totals: the direct x launches stride their workgroups over the tiles so
  // that one partial covers many pencils: about kTotCellsPerBlock cells per
  // workgroup (measured best from 16.8 M to 453 M cells), as a power of two
  // from 2 to 64 workgroups per CU (the same number on every CU)
  {
    const int cu = std::max(1, c->cu_count);
    const double cells = double(c->single.n[0]) * c->single.n[1] * c->single.n[2];
    const double per_cu = cells / (double(kTotCellsPerBlock) * cu);
    int m = 2;
    while (m < 64 && per_cu > 1.4142135623730951 * m) m *= 2;  // nearest power of two
    L.tot_cap = m * cu;
  }
  if (c->pp_live) {
    L.pdt = c->pdt;
    L.psmax = c->psmax;
  }
  if (c->cfg.ax[0].kind == kXMarchKind) {
    L.xmode = kXMarch;
  } else {
    bool wave = true;
    if (c->batch) {
      for (auto& P : c->patches) wave = wave && x_wave_ok(P.n[0], c->cfg.ax[0].v);
    } else {
      wave = x_wave_ok(c->single.n[0], c->cfg.ax[0].v);
    }
    L.xmode = wave ? kXPacked : kXMulti;
  }
  return L;
}

LaunchReduce reduce_launch(const hydro_ctx* c) {
  LaunchReduce L{};
  L.pool = c->pool;
  L.patches = c->batch ? c->d_patches : nullptr;
  L.single = c->single;
  L.npatch = c->batch ? c->npatch : 1;
  L.chunks = c->batch ? kBatchChunks
                      : chunks_for(int64_t(c->single.n[0]) * c->single.n[1] * c->single.n[2]);
  L.gamma = c->desc.gamma;
  for (int a = 0; a < 3; ++a) L.grav[a] = c->desc.grav[a];
  L.scal = c->scal;
  L.partials = c->partials;
  L.fp64 = c->fp64;
  if (c->pp_live) L.psmax = c->psmax;
  return L;
}

// Fused plane sweeps apply to a batch whose x and y axes are both active
// and whose every z-plane fits the kernel: an LDS share of at most
// kPlaneLdsBytes, lane runs of the x configuration's V along x and along y
// (n / V <= 64), and rows aligned for its vector copies.
bool plane_ok(const hydro_ctx* c, const Config& cf) {
  if (!c->batch || !c->active[0] || !c->active[1]) return false;
  const int v = cf.plane.v;
  if (v != 1 && v != 2 && v != 4) return false;
  if (cf.plane.block < 64 || cf.plane.block > kMaxBlock || cf.plane.block % 64) return false;
  const int esz = c->fp64 ? 8 : 4;
  const int a = std::min(v, 16 / esz);
  for (auto& P : c->patches) {
    if (P.n[0] == 1 || P.n[1] == 1) return false;
    if (P.n[0] % v || P.n[1] % v || P.n[0] / v > 64 || P.n[1] / v > 64) return false;
    if (plane_lds_bytes(P, c->fp64) == 0) return false;
    if (P.base0 % a || P.sy % a || P.sz % a || P.plane % a) return false;
  }
  return true;
}

// The z sweep over patch x-z planes in LDS applies when every patch has z
// active and an x-z plane within a workgroup's LDS share, with lane runs of
// V cells along x and z.
bool zplane_ok(const hydro_ctx* c, const Config& cf) {
  if (!c->batch || !c->active[2]) return false;
  const int v = cf.zplane.v;
  if (v != 1 && v != 2 && v != 4) return false;
  if (cf.zplane.block < 64 || cf.zplane.block > kMaxBlock || cf.zplane.block % 64) return false;
  const int esz = c->fp64 ? 8 : 4;
  const int a = std::min(v, 16 / esz);
  for (auto& P : c->patches) {
    if (P.n[0] == 1 || P.n[2] == 1) return false;
    if (P.n[0] % v || P.n[2] % v || P.n[0] / v > 64 || P.n[2] / v > 64) return false;
    if (plane_lds_bytes(P, c->fp64, 2) == 0) return false;
    if (P.base0 % a || P.sy % a || P.sz % a || P.plane % a) return false;
  }
  return true;
}

// The z sweep of every patch x-z plane in LDS (replaces the z march).
LaunchSweep zplane_launch(const hydro_ctx* c, int do_cfl) {
  LaunchSweep L = sweep_launch(c, 2, do_cfl);
  L.plane = kZPlane;
  L.cfg = c->cfg.zplane;
  L.items = c->d_items[4];
  L.nitems = c->nitems[4];
  // the plane's first axis is x, its second z
  L.bc_lo = c->desc.bc[0];
  L.bc_hi = c->desc.bc[1];
  L.grav = c->desc.grav[0];
  L.bc_lo_y = c->desc.bc[4];
  L.bc_hi_y = c->desc.bc[5];
  L.grav_y = c->desc.grav[2];
  int lds = 0;
  for (auto& P : c->patches) lds = std::max(lds, plane_lds_bytes(P, c->fp64, 2));
  L.plane_lds = lds;
  return L;
}

// The fused x and y sweeps of every patch z-plane (x first on even steps).
LaunchSweep plane_launch(const hydro_ctx* c, bool xfirst, int do_cfl) {
  LaunchSweep L = sweep_launch(c, 0, do_cfl);
  L.plane = xfirst ? kPlaneXY : kPlaneYX;
  L.cfg = c->cfg.plane;
  L.items = c->d_items[3];
  L.nitems = c->nitems[3];
  L.bc_lo_y = c->desc.bc[2];
  L.bc_hi_y = c->desc.bc[3];
  L.grav_y = c->desc.grav[1];
  int lds = 0;
  for (auto& P : c->patches) lds = std::max(lds, plane_lds_bytes(P, c->fp64));
  L.plane_lds = lds;
  return L;
}

// The fused x+y step of a single grid applies (see fuse_eligible) with a
// window kernel of V = 1 or 2 cells per lane.
bool win_ok(const hydro_ctx* c, const Config& cf) {
  if (c->batch || !c->shadow) return false;
  const int v = cf.plane.v;
  if (v != 1 && v != 2) return false;
  return cf.plane.block >= 64 && cf.plane.block <= kMaxBlock && cf.plane.block % 64 == 0;
}

// The fused x and y sweeps of a single grid, window by window, from src to
// dst (x first on even steps): two resident workgroups per CU take the
// windows of every z-plane round robin.
LaunchSweep window_launch(const hydro_ctx* c, bool xfirst, int do_cfl, void* src, void* dst) {
  LaunchSweep L = sweep_launch(c, 0, do_cfl);
  L.plane = xfirst ? kWinXY : kWinYX;
  L.cfg = c->cfg.plane;
  L.pool = src;
  L.dst = dst;
  L.wins = c->d_wins;
  L.nwin = c->nwin;
  L.nitems = c->nwin * c->single.n[2];
  L.nblocks = 2 * std::max(1, c->cu_count);
  L.bc_lo_y = c->desc.bc[2];
  L.bc_hi_y = c->desc.bc[3];
  L.grav_y = c->desc.grav[1];
  return L;
}

// One launch of a step and the profile slot it reports in (0: x, or x and y
// fused; 1: y; 2: z).
struct StepOp {
  LaunchSweep L;
  int slot;
};

// The launches of a step in Strang order (x, y, z on even steps, z, y, x on
// odd ones; with fusion the x and y sweeps are one launch), the last folding
// the CFL maximum.
std::vector<StepOp> step_ops(const hydro_ctx* c, int parity) {
  static const int even[3] = {0, 1, 2}, odd[3] = {2, 1, 0};
  const int* order = parity ? odd : even;
  const bool fuse = c->cfg.batch_fuse && c->nitems[3] > 0 && plane_ok(c, c->cfg);
  std::vector<int> seq;  // axes; -1 for the fused plane sweeps
  for (int i = 0; i < 3; ++i) {
    const int ax = order[i];
    if (!c->active[ax] || (c->batch && c->nitems[ax] == 0)) continue;
    if (fuse && ax < 2) {
      if (std::find(seq.begin(), seq.end(), -1) == seq.end()) seq.push_back(-1);
      continue;
    }
    seq.push_back(ax);
  }
  std::vector<StepOp> ops;
  if (!c->batch && c->cfg.batch_fuse && win_ok(c, c->cfg)) {
    // single grid, x and y fused: x+y from the state into the second buffer
    // and z back (even steps), or z into it and y+x back (odd steps)
    void* st = c->pool;
    void* sh = c->shadow;
    if (parity == 0) {
      ops.push_back(StepOp{window_launch(c, true, 0, st, sh), 0});
      LaunchSweep Z = sweep_launch(c, 2, 1);
      Z.pool = sh;
      Z.dst = st;
      ops.push_back(StepOp{Z, 2});
    } else {
      LaunchSweep Z = sweep_launch(c, 2, 0);
      Z.dst = sh;
      ops.push_back(StepOp{Z, 2});
      ops.push_back(StepOp{window_launch(c, false, 1, sh, st), 0});
    }
    ops.back().L.tpart = c->partials;
    return ops;
  }
  const bool zp = c->cfg.batch_zplane && c->nitems[4] > 0 && zplane_ok(c, c->cfg);
  for (size_t i = 0; i < seq.size(); ++i) {
    const int cfl = i + 1 == seq.size() ? 1 : 0;
    if (seq[i] < 0)
      ops.push_back(StepOp{plane_launch(c, parity == 0, cfl), 0});
    else if (seq[i] == 2 && zp)
      ops.push_back(StepOp{zplane_launch(c, cfl), 2});
    else
      ops.push_back(StepOp{sweep_launch(c, seq[i], cfl), seq[i]});
  }
  // the last sweep also folds the FP64 totals of the updated cells
  if (!ops.empty()) ops.back().L.tpart = c->partials;
  return ops;
}

// The end of a step after its sweep launches `ops`: the fixed-order sum of
// the totals partials the last sweep wrote, then t += dt and the next dt.
// With nothing to sweep the CFL maximum and the totals come from standalone
// reductions of the state.
hipError_t finish_step_launches(const hydro_ctx* c, const std::vector<StepOp>& ops,
                                hipStream_t st) {
  hipError_t e = hipSuccess;
  if (ops.empty()) {
    // nothing to sweep: the CFL maximum and the totals of the state itself
    LaunchReduce R = reduce_launch(c);
    R.fold_only = 1;
    e = launch_cfl(R, st);
    if (e == hipSuccess) e = launch_totals(reduce_launch(c), st);
    if (e == hipSuccess && !c->pp_live) e = launch_finish_step(c->scal, st);
  } else {
    e = launch_totals_finish(c->partials, sweep_parts(ops.back().L), c->tslice, c->scal,
                             c->pp_live ? 0 : 1, st);
  }
  // a dt per patch: each patch's t advances by its dt, then its next dt
  if (e == hipSuccess && c->pp_live)
    e = launch_patch_dt(c->pt, c->pdt, c->psmax, c->npatch, c->scal, 1, st);
  return e;
}

// dt of the next step on the device: `dt` (> 0) for every patch, or the CFL
// dt of the current state (one, or one per patch)
hipError_t set_step_dt(const hydro_ctx* c, double dt, hipStream_t st) {
  if (dt > 0.0)
    return c->pp_live ? launch_fill(c->pdt, c->npatch, dt, st) : launch_set_dt(c->scal, dt, st);
  hipError_t e = launch_cfl(reduce_launch(c), st);
  if (e == hipSuccess && c->pp_live)
    e = launch_patch_dt(c->pt, c->pdt, c->psmax, c->npatch, c->scal, 0, st);
  return e;
}

// The launches of a step, then the step bookkeeping.
hipError_t enqueue_step_kernels(const hydro_ctx* c, int parity, hipStream_t st) {
  if (!items_current(c)) return hipErrorInvalidValue;
  const std::vector<StepOp> ops = step_ops(c, parity);
  for (const StepOp& op : ops) {
    hipError_t e = launch_sweep(op.L, st);
    if (e != hipSuccess) return e;
  }
  return finish_step_launches(c, ops, st);
}

void destroy_graphs(hydro_ctx* c) {
  for (int p = 0; p < 2; ++p) {
    if (c->graph[p]) (void)hipGraphExecDestroy(c->graph[p]);
    c->graph[p] = nullptr;
  }
}

int capture_graphs(hydro_ctx* c) {
  destroy_graphs(c);
  // a graph freezes the work-list lengths: rebuild the lists for the current
  // configuration first, so the captured counts and the lists always agree
  if (c->batch) {
    int rc = rebuild_items(c);
    if (rc) return rc;
  }
  if (c->desc.flags & HYDRO_FLAG_NO_GRAPH) return HYDRO_OK;
  for (int p = 0; p < 2; ++p) {
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_step_kernels(c, p, c->cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(HYDRO_EDEVICE, std::string("graph capture: ") +
                                     hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipError_t e3 = hipGraphInstantiate(&c->graph[p], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) return fail(HYDRO_EDEVICE, std::string("graph instantiate: ") +
                                                        hipGetErrorString(e3));
  }
  return HYDRO_OK;
}

// Mean ms per launch of one sweep (dt on the device must already be 0).
int time_launch(hydro_ctx* c, const LaunchSweep& L, int reps, double* ms);
int time_sweep(hydro_ctx* c, int axis, int reps, double* ms) {
  return time_launch(c, sweep_launch(c, axis, 1), reps, ms);
}

int time_launch(hydro_ctx* c, const LaunchSweep& L, int reps, double* ms) {
  if (!items_current(c)) return fail(HYDRO_ESTATE, "batch work lists out of date");
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  auto run = [&]() -> hipError_t {
    hipError_t e = launch_sweep(L, c->stream);
    if (e == hipSuccess && c->batch) e = launch_reset_tickets(c->scal, c->stream);
    return e;
  };
  int rc = HYDRO_OK;
  for (int i = 0; i < 2 && rc == HYDRO_OK; ++i)
    if (run() != hipSuccess) rc = fail(HYDRO_EDEVICE, "sweep launch failed");
  if (rc == HYDRO_OK && hipEventRecord(a, c->stream) != hipSuccess) rc = HYDRO_EDEVICE;
  for (int i = 0; i < reps && rc == HYDRO_OK; ++i)
    if (run() != hipSuccess) rc = fail(HYDRO_EDEVICE, "sweep launch failed");
  if (rc == HYDRO_OK && hipEventRecord(b, c->stream) != hipSuccess) rc = HYDRO_EDEVICE;
  if (rc == HYDRO_OK && hipEventSynchronize(b) != hipSuccess) rc = HYDRO_EDEVICE;
  float t = 0.f;
  if (rc == HYDRO_OK && hipEventElapsedTime(&t, a, b) != hipSuccess) rc = HYDRO_EDEVICE;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc == HYDRO_OK) *ms = double(t) / reps;
  return rc == HYDRO_EDEVICE && g_last_error.empty() ? fail(rc, "timing failed") : rc;
}

// Mean time of one even plus one odd step's sweep launches, run back to back
// in step order as a captured step runs them (one step pair of warm-up).
int time_steps(hydro_ctx* c, int reps, double* ms) {
  if (!items_current(c)) return fail(HYDRO_ESTATE, "batch work lists out of date");
  std::vector<StepOp> ops = step_ops(c, 0);
  for (const StepOp& op : step_ops(c, 1)) ops.push_back(op);
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  auto run = [&]() -> hipError_t {
    for (const StepOp& op : ops) {
      hipError_t e = launch_sweep(op.L, c->stream);
      if (e == hipSuccess && c->batch) e = launch_reset_tickets(c->scal, c->stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  int rc = HYDRO_OK;
  if (run() != hipSuccess) rc = fail(HYDRO_EDEVICE, "sweep launch failed");
  if (rc == HYDRO_OK && hipEventRecord(a, c->stream) != hipSuccess) rc = HYDRO_EDEVICE;
  for (int i = 0; i < reps && rc == HYDRO_OK; ++i)
    if (run() != hipSuccess) rc = fail(HYDRO_EDEVICE, "sweep launch failed");
  if (rc == HYDRO_OK && hipEventRecord(b, c->stream) != hipSuccess) rc = HYDRO_EDEVICE;
  if (rc == HYDRO_OK && hipEventSynchronize(b) != hipSuccess) rc = HYDRO_EDEVICE;
  float t = 0.f;
  if (rc == HYDRO_OK && hipEventElapsedTime(&t, a, b) != hipSuccess) rc = HYDRO_EDEVICE;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc == HYDRO_OK) *ms = double(t) / reps;
  return rc == HYDRO_EDEVICE && g_last_error.empty() ? fail(rc, "timing failed") : rc;
}

std::string shape_key(const hydro_ctx* c, int axis) {
  std::ostringstream o;
  o << c->arch << ":cu" << c->cu_count << ":" << (c->fp64 ? "fp64" : "fp32") << ":ax" << axis
    << ":k7";
  if (c->batch) {
    o << ":batch" << c->npatch << "x" << c->max_patch_cells;
  } else {
    o << ":" << c->single.n[0] << "x" << c->single.n[1] << "x" << c->single.n[2] << ":s"
      << c->single.sy << "x" << c->single.sz;
  }
  return o.str();
}

std::vector<SweepCfg> candidates(const hydro_ctx* c, int axis) {
  std::vector<SweepCfg> out;
  if (axis == 0) {
    const std::vector<PatchDev> ps = c->batch ? c->patches : std::vector<PatchDev>{c->single};
    int nx_min = 1 << 30;
    for (auto& P : ps) nx_min = std::min(nx_min, P.n[0]);
    for (int v : {1, 2, 4})
      for (int b : {64, 128, 192, 256, 384, 448, 512}) {
        SweepCfg s{};
        s.kind = kLaneRunKind;
        s.v = v;
        s.block = b;
        if (x_cfg_ok_all(s, ps, c->fp64)) out.push_back(s);
        // the march only pays where every pencil spans more than one wave;
        // direct launches also try capped grids (a wave then marches
        // several pencils, prefetching the next one's first chunk)
        s.kind = kXMarchKind;
        if (nx_min / v > 64 && x_cfg_ok_all(s, ps, c->fp64)) {
          out.push_back(s);
          if (!c->batch)
            for (int g : {2, 4, 8}) {
              s.q = g * c->cu_count;
              out.push_back(s);
            }
          s.q = 0;
        }
      }
  } else {
    int n = c->batch ? 64 : c->single.n[axis];
    for (int q : {64, 128, 256})
      for (int s : {1, 2, 4, 8, 16}) {
        SweepCfg k{};
        k.kind = kColumnKind;
        k.q = q;
        k.s = s;
        if (!col_cfg_ok(k)) continue;
        if (s > 1 && (n + s - 1) / s < 8) continue;  // segments shorter than 8 cells
        out.push_back(k);
      }
  }
  return out;
}

int rebuild_items(hydro_ctx* c);

// Index of the fastest of n candidates.  Every candidate is timed once per
// round, in forward order on even rounds and reverse order on odd ones, and
// keeps its fastest round: a slow stretch of the device (clock or power
// transients) then costs every candidate alike instead of whichever ran
// during it.  apply(i) selects candidate i; measure(&ms) times it.
// With HYDRO_TUNE_LOG set, every timing goes to stderr as
// "tune <what> <candidate> <round> <ms>".
template <class Apply, class Measure>
int fastest_of(const char* what, int n, int rounds, Apply apply, Measure measure, int* best,
               std::vector<double>* times = nullptr) {
  const char* lg = std::getenv("HYDRO_TUNE_LOG");
  const bool log = lg && *lg && std::strcmp(lg, "0") != 0;
  std::vector<double> t(size_t(n), 1e30);
  for (int r = 0; r < rounds; ++r)
    for (int k = 0; k < n; ++k) {
      const int i = (r & 1) ? n - 1 - k : k;
      int rc = apply(i);
      double ms = 0.0;
      if (rc == HYDRO_OK) rc = measure(&ms);
      if (rc != HYDRO_OK) return rc;
      t[size_t(i)] = std::min(t[size_t(i)], ms);
      if (log) std::fprintf(stderr, "tune %s %d %d %.4f\n", what, i, r, ms);
    }
  *best = int(std::min_element(t.begin(), t.end()) - t.begin());
  if (times) *times = t;
  return HYDRO_OK;
}

// Pick each axis' configuration: HYDRO_FORCE_CONFIG, then the cache, then a
// timing search (dt = 0 leaves the state unchanged bit for bit).
int choose_config(hydro_ctx* c) {
  Config cf = c->cfg;
  const char* forced = std::getenv("HYDRO_FORCE_CONFIG");
  if (forced && *forced) {
    if (!parse_cfg(forced, cf)) return fail(HYDRO_EINVAL, "bad HYDRO_FORCE_CONFIG");
    c->cfg = cf;
    return HYDRO_OK;
  }
  if (c->desc.flags & HYDRO_FLAG_NO_TUNE) return HYDRO_OK;
  std::map<std::string, std::string> cache;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    cache = cache_read();
  }
  bool dirty = false;
  for (int axis = 0; axis < 3; ++axis) {
    if (!c->active[axis]) continue;
    std::string key = shape_key(c, axis);
    auto it = cache.find(key);
    if (it != cache.end()) {
      Config tmp = c->cfg;
      if (parse_cfg(it->second, tmp)) {
        bool ok = axis == 0 ? true : col_cfg_ok(tmp.ax[axis]);
        if (axis == 0)
          ok = x_cfg_ok_all(tmp.ax[0],
                            c->batch ? c->patches : std::vector<PatchDev>{c->single}, c->fp64);
        if (ok) {
          c->cfg.ax[axis] = tmp.ax[axis];
          if (c->batch) {
            int rc = rebuild_items(c);
            if (rc) return rc;
          }
          continue;
        }
      }
    }
    // timing search
    int rc = HYDRO_OK;
    if (launch_timing_begin(c->scal, c->stream) != hipSuccess)
      return fail(HYDRO_EDEVICE, "timing setup failed");
    SweepCfg best_cfg = c->cfg.ax[axis];
    const std::vector<SweepCfg> cands = candidates(c, axis);
    int bi = 0;
    if (!cands.empty()) {
      static const char* const names[3] = {"x", "y", "z"};
      std::vector<double> iso;
      rc = fastest_of(
          names[axis], int(cands.size()), 2,
          [&](int i) {
            c->cfg.ax[axis] = cands[size_t(i)];
            return c->batch ? rebuild_items(c) : HYDRO_OK;
          },
          [&](double* ms) { return time_sweep(c, axis, 5, ms); }, &bi, &iso);
      if (rc == HYDRO_OK && !c->batch && cands.size() > 1) {
        // A sweep repeated alone runs in a different cache state from the
        // same sweep inside a step (it follows another axis' writes), and
        // the ranking can differ: the fastest few alone are timed again
        // over whole even + odd steps.
        static const char* const step_names[3] = {"x-in-step", "y-in-step", "z-in-step"};
        std::vector<int> idx(cands.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = int(i);
        std::sort(idx.begin(), idx.end(),
                  [&](int a, int b) { return iso[size_t(a)] < iso[size_t(b)]; });
        const int top = std::min<int>(3, int(idx.size()));
        int bs = 0;
        rc = fastest_of(
            step_names[axis], top, 3,
            [&](int i) {
              c->cfg.ax[axis] = cands[size_t(idx[size_t(i)])];
              return HYDRO_OK;
            },
            [&](double* ms) { return time_steps(c, 2, ms); }, &bs);
        if (rc == HYDRO_OK) bi = idx[size_t(bs)];
      }
      if (rc == HYDRO_OK) best_cfg = cands[size_t(bi)];
    }
    c->cfg.ax[axis] = best_cfg;
    if (launch_timing_end(c->scal, c->stream) != hipSuccess)
      return fail(HYDRO_EDEVICE, "timing teardown failed");
    if (rc != HYDRO_OK) return rc;
    if (c->batch && (rc = rebuild_items(c)) != HYDRO_OK) return rc;
    Config one{};
    one.ax[axis] = best_cfg;
    std::string txt = cfg_text(one);
    // keep only this axis' part
    std::string part;
    {
      std::stringstream ss(txt);
      std::string p;
      const char tag = "xyz"[axis];
      while (std::getline(ss, p, ';'))
        if (!p.empty() && p[0] == tag) part = p;
    }
    cache[key] = part;
    dirty = true;
  }
  if (!c->batch && c->shadow) {
    // single grid with the fused x+y step available: keep it when whole
    // steps (an even and an odd one, as they will run) are faster than with
    // the separate sweeps
    const std::string key = shape_key(c, 4);
    auto it = cache.find(key);
    Config tmp = c->cfg;
    if (it != cache.end() && parse_cfg(it->second, tmp) && (!tmp.batch_fuse || win_ok(c, tmp))) {
      c->cfg.batch_fuse = tmp.batch_fuse;
      c->cfg.plane = tmp.plane;
    } else {
      if (launch_timing_begin(c->scal, c->stream) != hipSuccess)
        return fail(HYDRO_EDEVICE, "timing setup failed");
      std::vector<SweepCfg> wins;  // candidate i > 0: window configuration i - 1
      for (int v : {1, 2})
        for (int b : {256, 512}) {
          Config trial = c->cfg;
          trial.plane.v = v;
          trial.plane.block = b;
          if (win_ok(c, trial)) wins.push_back(trial.plane);
        }
      const SweepCfg keep = c->cfg.plane;
      int bi = 0;
      int rc = fastest_of(
          "fuse", int(wins.size()) + 1, 3,
          [&](int i) {
            c->cfg.batch_fuse = i > 0 ? 1 : 0;
            if (i > 0) c->cfg.plane = wins[size_t(i - 1)];
            return HYDRO_OK;
          },
          [&](double* ms) { return time_steps(c, 2, ms); }, &bi);
      if (launch_timing_end(c->scal, c->stream) != hipSuccess)
        return fail(HYDRO_EDEVICE, "timing teardown failed");
      if (rc) return rc;
      c->cfg.plane = bi > 0 ? wins[size_t(bi - 1)] : keep;
      c->cfg.batch_fuse = bi > 0 ? 1 : 0;
      std::ostringstream o;
      o << "p:f=" << c->cfg.batch_fuse << ";w:v=" << c->cfg.plane.v << ",b=" << c->cfg.plane.block;
      cache[key] = o.str();
      dirty = true;
    }
  }
  if (c->batch) {
    // fuse the x and y sweeps per patch z-plane when that is faster than the
    // two sweeps: the fastest valid plane configuration (both Strang orders
    // timed) against x + y
    const std::string key = shape_key(c, 4);
    auto it = cache.find(key);
    Config tmp = c->cfg;
    if (it != cache.end() && parse_cfg(it->second, tmp) && (!tmp.batch_fuse || plane_ok(c, tmp))) {
      c->cfg.batch_fuse = tmp.batch_fuse;
      c->cfg.plane = tmp.plane;
    } else {
      if (launch_timing_begin(c->scal, c->stream) != hipSuccess)
        return fail(HYDRO_EDEVICE, "timing setup failed");
      // candidate 0: the separate sweeps (x + y); candidate i > 0: plane
      // configuration i - 1 (mean of its x-first and y-first launches)
      std::vector<SweepCfg> planes;
      for (int v : {1, 2, 4})
        for (int b : {256, 512}) {
          Config trial = c->cfg;
          trial.plane.v = v;
          trial.plane.block = b;
          if (plane_ok(c, trial)) planes.push_back(trial.plane);
        }
      const SweepCfg keep = c->cfg.plane;
      int sel = 0, bi = 0;
      int rc = fastest_of(
          "plane", int(planes.size()) + 1, 3,
          [&](int i) {
            sel = i;
            if (i > 0) c->cfg.plane = planes[size_t(i - 1)];
            return HYDRO_OK;
          },
          [&](double* ms) {
            double t0 = 0.0, t1 = 0.0;
            int r = sel ? time_launch(c, plane_launch(c, true, 1), 5, &t0)
                        : time_sweep(c, 0, 5, &t0);
            if (r == HYDRO_OK)
              r = sel ? time_launch(c, plane_launch(c, false, 1), 5, &t1)
                      : time_sweep(c, 1, 5, &t1);
            *ms = sel ? 0.5 * (t0 + t1) : t0 + t1;
            return r;
          },
          &bi);
      if (launch_timing_end(c->scal, c->stream) != hipSuccess)
        return fail(HYDRO_EDEVICE, "timing teardown failed");
      if (rc) return rc;
      c->cfg.plane = bi > 0 ? planes[size_t(bi - 1)] : keep;
      c->cfg.batch_fuse = bi > 0 ? 1 : 0;
      std::ostringstream o;
      o << "p:f=" << c->cfg.batch_fuse << ";w:v=" << c->cfg.plane.v << ",b="
        << c->cfg.plane.block;
      cache[key] = o.str();
      dirty = true;
    }
  }
  if (c->batch) {
    // persistent grid size (workgroups per CU) and scheduling, timed over
    // the launches of one even and one odd step as they will run
    const std::string key = shape_key(c, 3);
    auto it = cache.find(key);
    Config tmp = c->cfg;
    if (it != cache.end() && parse_cfg(it->second, tmp) && tmp.batch_blocks > 0 &&
        tmp.batch_blocks <= 65536) {
      c->cfg.batch_blocks = tmp.batch_blocks;
      c->cfg.batch_dyn = tmp.batch_dyn;
    } else {
      if (launch_timing_begin(c->scal, c->stream) != hipSuccess)
        return fail(HYDRO_EDEVICE, "timing setup failed");
      // 2, 4, 8, 16 workgroups per CU, each with the ticket and round robin
      auto apply = [&](int i) {
        c->cfg.batch_blocks = (2 << (i % 4)) * c->cu_count;
        c->cfg.batch_dyn = i < 4 ? 1 : 0;
        return HYDRO_OK;
      };
      int bi = 0;
      int rc = fastest_of("grid", 8, 3, apply, [&](double* ms) { return time_steps(c, 2, ms); }, &bi);
      if (rc == HYDRO_OK) apply(bi);
      const int best_g = c->cfg.batch_blocks, best_d = c->cfg.batch_dyn;
      if (launch_timing_end(c->scal, c->stream) != hipSuccess)
        return fail(HYDRO_EDEVICE, "timing teardown failed");
      if (rc) return rc;
      cache[key] = "p:g=" + std::to_string(best_g) + ",d=" + std::to_string(best_d);
      dirty = true;
    }
  }
  if (c->batch && c->active[2]) {
    // the z sweep over x-z planes in LDS against the z march, timed over the
    // launches of one even and one odd step
    const std::string key = shape_key(c, 5);
    auto it = cache.find(key);
    Config tmp = c->cfg;
    if (it != cache.end() && parse_cfg(it->second, tmp) &&
        (!tmp.batch_zplane || zplane_ok(c, tmp))) {
      c->cfg.batch_zplane = tmp.batch_zplane;
      c->cfg.zplane = tmp.zplane;
    } else {
      if (launch_timing_begin(c->scal, c->stream) != hipSuccess)
        return fail(HYDRO_EDEVICE, "timing setup failed");
      std::vector<SweepCfg> zps;  // candidate i > 0: x-z plane configuration i - 1
      for (int v : {1, 2, 4})
        for (int b : {256, 512}) {
          Config trial = c->cfg;
          trial.zplane.v = v;
          trial.zplane.block = b;
          if (zplane_ok(c, trial)) zps.push_back(trial.zplane);
        }
      const SweepCfg keep = c->cfg.zplane;
      int bi = 0;
      int rc = fastest_of(
          "zplane", int(zps.size()) + 1, 3,
          [&](int i) {
            c->cfg.batch_zplane = i > 0 ? 1 : 0;
            if (i > 0) c->cfg.zplane = zps[size_t(i - 1)];
            return HYDRO_OK;
          },
          [&](double* ms) { return time_steps(c, 2, ms); }, &bi);
      if (launch_timing_end(c->scal, c->stream) != hipSuccess)
        return fail(HYDRO_EDEVICE, "timing teardown failed");
      if (rc) return rc;
      c->cfg.zplane = bi > 0 ? zps[size_t(bi - 1)] : keep;
      c->cfg.batch_zplane = bi > 0 ? 1 : 0;
      std::ostringstream o;
      o << "p:z=" << c->cfg.batch_zplane << ";u:v=" << c->cfg.zplane.v << ",b="
        << c->cfg.zplane.block;
      cache[key] = o.str();
      dirty = true;
    }
  }
  if (dirty) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto merged = cache_read();
    for (auto& kv : cache) merged[kv.first] = kv.second;
    cache_write(merged);
  }
  return HYDRO_OK;
}

int device_info(hydro_ctx* c) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  c->cu_count = prop.multiProcessorCount;
  c->arch = prop.gcnArchName;
  auto colon = c->arch.find(':');
  if (colon != std::string::npos) c->arch = c->arch.substr(0, colon);
  return HYDRO_OK;
}

int common_init(hydro_ctx* c) {
  int rc = device_info(c);
  if (rc) return rc;
  HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  HIP_TRY(launch_init_scalars(c->scal, c->desc.cfl, 0.0, 0.0, c->stream));
  rc = choose_config(c);
  if (rc) return rc;
  HIP_TRY(launch_init_scalars(c->scal, c->desc.cfl, 0.0, 0.0, c->stream));
  if (c->per_patch) {
    c->pp_live = true;
    HIP_TRY(launch_fill(c->pt, c->npatch, 0.0, c->stream));
    HIP_TRY(launch_fill(c->pdt, c->npatch, 0.0, c->stream));
    HIP_TRY(launch_fill(reinterpret_cast<double*>(c->psmax), c->npatch, 0.0, c->stream));
  }
  rc = capture_graphs(c);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->step = 0;
  c->t_host = 0.0;
  c->dt_valid = false;
  return HYDRO_OK;
}

int read_scalars(hydro_ctx* c, DevScalars* out) {
  HIP_TRY(hipMemcpyAsync(out, c->scal, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return HYDRO_OK;
}

// Totals partials of a single grid: the most workgroups any valid
// configuration launches for a sweep (x: one pencil per workgroup; y, z: 64
// columns per tile), and at least the standalone reduction's chunks.
// Windows of the fused x+y step along an axis of n cells for windows of
// `edge` cells: written chunks of edge - 2 kWinHalo cells.
int32_t win_count(int32_t n, int edge) {
  const int w = edge - 2 * kWinHalo;
  return n >= edge ? (n + w - 1) / w : 0;
}

int64_t grid_parts(const int32_t n[3]) {
  int64_t m = kMaxChunks;
  m = std::max<int64_t>(m, int64_t(win_count(n[0], kWinEdge)) * win_count(n[1], win_rows(true)) *
                               n[2]);
  if (n[0] > 1) m = std::max<int64_t>(m, int64_t(n[1]) * n[2]);
  if (n[1] > 1) m = std::max<int64_t>(m, (int64_t(n[0]) * n[2] + 63) / 64);
  if (n[2] > 1) m = std::max<int64_t>(m, (int64_t(n[0]) * n[1] + 63) / 64);
  return m;
}

// Single-grid workspace: scalars, totals partials and the first level of
// their reduction, then the partial sums of the slab profiles
// (kProfileChunksX per slab of the longest axis, 5 values each).
size_t grid_totals_bytes(const int32_t n[3]) {
  return align_up(size_t(grid_parts(n)) * 6 * sizeof(double), 256) +
         align_up(size_t(kTotalsSlices) * 6 * sizeof(double), 256);
}
size_t grid_workspace_bytes(const int32_t n[3]) {
  const int64_t nmax = std::max(n[0], std::max(n[1], n[2]));
  return kScalarBytes + grid_totals_bytes(n) +
         align_up(size_t(nmax) * kProfileChunksX * 5 * sizeof(double), 256);
}

// The fused x+y step of a single grid applies to grids with x and y extents
// even and at least a window's (kWinEdge along x, win_rows() along y) and
// an active z axis, whose rows allow runs of two cells (even strides).
bool fuse_eligible(const hydro_desc& d) {
  if (!(d.flags & HYDRO_FLAG_FUSE_XY)) return false;
  const bool fp64 = d.precision == HYDRO_FP64;
  if (d.nx < kWinEdge || d.ny < win_rows(fp64) || d.nx % 2 || d.ny % 2 || d.nz < 2) return false;
  int32_t n[3] = {d.nx, d.ny, d.nz};
  double dx[3] = {d.dx, d.dy, d.dz};
  const PatchDev P = make_patch(n, d.ng, dx, 0);
  return P.base0 % 2 == 0 && P.sy % 2 == 0 && P.sz % 2 == 0 && P.plane % 2 == 0;
}

// Workspace of the fused step after the grid's own: the window table, then
// the second state buffer.
size_t fuse_bytes(const hydro_desc& d) {
  if (!fuse_eligible(d)) return 0;
  int32_t n[3] = {d.nx, d.ny, d.nz};
  double dx[3] = {d.dx, d.dy, d.dz};
  const PatchDev P = make_patch(n, d.ng, dx, 0);
  const bool fp64 = d.precision == HYDRO_FP64;
  const size_t nwin = size_t(win_count(d.nx, kWinEdge)) * win_count(d.ny, win_rows(fp64));
  return align_up(nwin * sizeof(WinDev), 256) +
         align_up(size_t(P.plane) * 5 * (fp64 ? 8 : 4), 256);
}

// The windows of a z-plane: along each axis, written chunks [w i, w (i+1))
// (the last one shorter), w = edge - 2 kWinHalo with edge = kWinEdge along
// x and win_rows() along y; a window starts
// kWinHalo cells before its chunk, wrapped on a periodic axis, or clamped
// into the domain on a non-periodic one, where its pencil ends at a domain
// edge take the boundary condition (elsewhere the ends are discarded).
std::vector<WinDev> build_windows(const int32_t n[3], const int32_t bc[6], bool fp64) {
  struct Span { int32_t start, lo, hi, blo, bhi; };
  auto spans = [&](int axis) {
    std::vector<Span> out;
    const int edge = axis == 0 ? kWinEdge : win_rows(fp64);
    const int N = n[axis], w = edge - 2 * kWinHalo;
    const bool per = bc[2 * axis] == HYDRO_BC_PERIODIC;
    for (int o = 0; o < N; o += w) {
      const int e = std::min(N, o + w);
      const int start = per ? o - kWinHalo : std::max(0, std::min(o - kWinHalo, N - edge));
      Span sp{start, o - start, e - start, HYDRO_BC_PERIODIC, HYDRO_BC_PERIODIC};
      if (!per && start == 0) sp.blo = bc[2 * axis];
      if (!per && start + edge == N) sp.bhi = bc[2 * axis + 1];
      out.push_back(sp);
    }
    return out;
  };
  std::vector<WinDev> wins;
  for (const Span& y : spans(1))
    for (const Span& x : spans(0))
      wins.push_back(WinDev{x.start, y.start, x.lo, x.hi, y.lo, y.hi, x.blo, x.bhi, y.blo, y.bhi});
  return wins;
}

// layout of a batch workspace
struct BatchLayout {
  size_t partials, slice, patches, items[5], pt, pdt, psmax, total;
};

// totals partials: one per work item of any sweep launch, and at least the
// standalone reduction's chunks
BatchLayout batch_layout(int32_t n, const int32_t items[5]) {
  BatchLayout L;
  size_t o = kScalarBytes;
  L.partials = o;
  int64_t parts = int64_t(n) * kBatchChunks;
  for (int a = 0; a < 5; ++a) parts = std::max<int64_t>(parts, items[a]);
  o += align_up(size_t(parts) * 6 * sizeof(double), 256);
  L.slice = o;
  o += align_up(size_t(kTotalsSlices) * 6 * sizeof(double), 256);
  L.patches = o;
  o += align_up(size_t(n) * sizeof(PatchDev), 256);
  for (int a = 0; a < 5; ++a) {
    L.items[a] = o;
    o += align_up(size_t(std::max(1, items[a])) * sizeof(WorkItem), 256);
  }
  // time, dt and CFL maximum per patch (HYDRO_BATCH_PER_PATCH_DT)
  L.pt = o;
  o += align_up(size_t(n) * sizeof(double), 256);
  L.pdt = o;
  o += align_up(size_t(n) * sizeof(double), 256);
  L.psmax = o;
  o += align_up(size_t(n) * sizeof(unsigned long long), 256);
  L.total = o;
  return L;
}

// The most tiles a patch list can need per axis under any valid config
// (x: v = 1 with one pencil per workgroup; columns: 64 columns per tile),
// its z-planes (fused plane sweeps) and its x-z planes (z sweep in LDS).
void max_items(const std::vector<PatchDev>& ps, int32_t out[5]) {
  int64_t acc[5] = {0, 0, 0, 0, 0};
  for (auto& P : ps) {
    acc[0] += int64_t(P.n[1]) * P.n[2];
    acc[1] += (int64_t(P.n[0]) * P.n[2] + 63) / 64;
    acc[2] += (int64_t(P.n[0]) * P.n[1] + 63) / 64;
    acc[3] += P.n[2];
    acc[4] += P.n[1];
  }
  for (int a = 0; a < 5; ++a) out[a] = int32_t(std::min<int64_t>(acc[a], INT32_MAX));
}

int rebuild_items(hydro_ctx* c) {
  // work items per axis, largest patches first (longest-processing-time
  // order keeps the persistent workgroups busy until the end)
  std::vector<int32_t> order(c->npatch);
  for (int32_t i = 0; i < c->npatch; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    const PatchDev &A = c->patches[a], &B = c->patches[b];
    return int64_t(A.n[0]) * A.n[1] * A.n[2] > int64_t(B.n[0]) * B.n[1] * B.n[2];
  });
  int32_t cap[5];
  max_items(c->patches, cap);
  for (int axis = 0; axis < 5; ++axis) {
    std::vector<WorkItem> items;
    if (axis == 4) {
      // x-z planes of the z sweep in LDS (patches with z active)
      if (c->active[2])
        for (int32_t p : order) {
          const PatchDev& P = c->patches[p];
          if (P.n[2] == 1) continue;
          for (int32_t y = 0; y < P.n[1]; ++y) items.push_back(WorkItem{p, y});
        }
    } else if (axis == 3) {
      // z-planes of the fused plane sweeps (patches with both x and y active)
      if (c->active[0] && c->active[1])
        for (int32_t p : order) {
          const PatchDev& P = c->patches[p];
          if (P.n[0] == 1 || P.n[1] == 1) continue;
          for (int32_t z = 0; z < P.n[2]; ++z) items.push_back(WorkItem{p, z});
        }
    } else if (c->active[axis]) {
      for (int32_t p : order) {
        const PatchDev& P = c->patches[p];
        if (P.n[axis] == 1) continue;
        int64_t nt = axis == 0 ? x_tiles(P, c->cfg.ax[0]) : col_tiles(P, axis, c->cfg.ax[axis]);
        for (int64_t t = 0; t < nt; ++t) items.push_back(WorkItem{p, int32_t(t)});
      }
    }
    if (int64_t(items.size()) > cap[axis]) return fail(HYDRO_EINVAL, "work list overflow");
    c->nitems[axis] = int32_t(items.size());
    if (!items.empty())
      HIP_TRY(hipMemcpyAsync(c->d_items[axis], items.data(), items.size() * sizeof(WorkItem),
                             hipMemcpyHostToDevice, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::memcpy(&c->items_cfg, &c->cfg, sizeof(Config));
  return HYDRO_OK;
}

}  // namespace

// ------------------------------------------------------------------------
// exported API
// ------------------------------------------------------------------------

extern "C" {

int hydro_abi_version(void) { return HYDRO_ABI_VERSION; }

const char* hydro_strerror(int s) {
  switch (s) {
    case HYDRO_OK: return "HYDRO_OK";
    case HYDRO_EINVAL: return "HYDRO_EINVAL: invalid argument";
    case HYDRO_EDEVICE: return "HYDRO_EDEVICE: HIP runtime error";
    case HYDRO_ENUMERIC: return "HYDRO_ENUMERIC: non-physical or non-finite state";
    case HYDRO_ESTATE: return "HYDRO_ESTATE: call out of order";
    default: return "unknown hydro status";
  }
}

const char* hydro_last_error(void) { return g_last_error.c_str(); }

int hydro_workspace_bytes(const hydro_desc* d, size_t* bytes) {
  if (!d || !bytes) return fail(HYDRO_EINVAL, "null argument");
  int rc = check_common(d);
  if (rc) return rc;
  int32_t n[3] = {d->nx, d->ny, d->nz};
  double dx[3] = {d->dx, d->dy, d->dz};
  rc = check_extent(n, d->ng, dx);
  if (rc) return rc;
  *bytes = grid_workspace_bytes(n) + fuse_bytes(*d);
  return HYDRO_OK;
}

int hydro_init(const hydro_desc* d, void* state, size_t state_bytes, void* workspace,
               size_t ws_bytes, void* stream, hydro_ctx** out) {
  g_last_error.clear();
  if (!out) return fail(HYDRO_EINVAL, "null output pointer");
  *out = nullptr;
  size_t need = 0;
  int rc = hydro_workspace_bytes(d, &need);
  if (rc) return rc;
  if (!state || !workspace) return fail(HYDRO_EINVAL, "null device pointer");
  if ((reinterpret_cast<uintptr_t>(state) & 15) || (reinterpret_cast<uintptr_t>(workspace) & 15))
    return fail(HYDRO_EINVAL, "device pointers must be 16-byte aligned");
  if (ws_bytes < need) return fail(HYDRO_EINVAL, "workspace too small");
  int32_t n[3] = {d->nx, d->ny, d->nz};
  double dx[3] = {d->dx, d->dy, d->dz};
  PatchDev P = make_patch(n, d->ng, dx, 0);
  const int64_t esz = d->precision == HYDRO_FP64 ? 8 : 4;
  if (!plane_fits(P, esz)) return fail(HYDRO_EINVAL, "a state plane must be smaller than 4 GiB");
  if (state_bytes < size_t(P.plane) * 5 * size_t(esz))
    return fail(HYDRO_EINVAL, "state buffer too small");
  hydro_ctx* c = new (std::nothrow) hydro_ctx();
  if (!c) return fail(HYDRO_EINVAL, "out of host memory");
  c->desc = *d;
  c->fp64 = d->precision == HYDRO_FP64;
  c->pool = state;
  c->pool_bytes = size_t(P.plane) * 5 * size_t(esz);
  c->ws = static_cast<char*>(workspace);
  c->ws_bytes = ws_bytes;
  c->stream = static_cast<hipStream_t>(stream);
  c->scal = reinterpret_cast<DevScalars*>(c->ws);
  c->partials = reinterpret_cast<double*>(c->ws + kScalarBytes);
  c->tslice = reinterpret_cast<double*>(
      c->ws + kScalarBytes + align_up(size_t(grid_parts(n)) * 6 * sizeof(double), 256));
  c->profile_partials = reinterpret_cast<double*>(c->ws + kScalarBytes + grid_totals_bytes(n));
  c->single = P;
  for (int a = 0; a < 3; ++a) c->active[a] = n[a] > 1;
  c->cfg.ax[0] = default_x({P}, c->fp64);
  c->cfg.ax[1] = default_col(n[1]);
  c->cfg.ax[2] = default_col(n[2]);
  if (c->cfg.ax[0].v == 0 && c->active[0]) {
    delete c;
    return fail(HYDRO_EINVAL, "no valid x-sweep configuration for this width");
  }
  if (fuse_eligible(*d)) {
    const std::vector<WinDev> wins = build_windows(n, d->bc, d->precision == HYDRO_FP64);
    char* f = c->ws + grid_workspace_bytes(n);
    c->d_wins = reinterpret_cast<WinDev*>(f);
    c->nwin = int32_t(wins.size());
    c->shadow = f + align_up(wins.size() * sizeof(WinDev), 256);
    if (hipMemcpyAsync(c->d_wins, wins.data(), wins.size() * sizeof(WinDev),
                       hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      delete c;
      return fail(HYDRO_EDEVICE, "window table upload failed");
    }
  }
  rc = common_init(c);
  if (rc) {
    hydro_destroy(c);
    return rc;
  }
  *out = c;
  return HYDRO_OK;
}

int hydro_batch_workspace_bytes(const hydro_patch* p, int32_t n, const hydro_desc* common,
                                size_t* bytes) {
  if (!p || !common || !bytes || n < 1) return fail(HYDRO_EINVAL, "bad batch arguments");
  int rc = check_common(common);
  if (rc) return rc;
  std::vector<PatchDev> ps;
  ps.reserve(n);
  for (int32_t i = 0; i < n; ++i) {
    int32_t nn[3] = {p[i].nx, p[i].ny, p[i].nz};
    double dx[3] = {p[i].dx, p[i].dy, p[i].dz};
    rc = check_extent(nn, p[i].ng, dx);
    if (rc) return rc;
    PatchDev P;
    int64_t len = 0;
    if (!patch_from(p[i], &P, &len))
      return fail(HYDRO_EINVAL, "patch " + std::to_string(i) + " has an inconsistent layout");
    if (!plane_fits(P, common->precision == HYDRO_FP64 ? 8 : 4))
      return fail(HYDRO_EINVAL, "patch " + std::to_string(i) + ": a plane must be smaller than 4 GiB");
    ps.push_back(P);
  }
  int32_t cap[5];
  max_items(ps, cap);
  *bytes = batch_layout(n, cap).total;
  return HYDRO_OK;
}

int hydro_batch_init(const hydro_patch* p, int32_t n, const hydro_desc* common, void* pool,
                     size_t pool_bytes, void* workspace, size_t ws_bytes, void* stream,
                     hydro_ctx** out) {
  g_last_error.clear();
  if (!out) return fail(HYDRO_EINVAL, "null output pointer");
  *out = nullptr;
  size_t need = 0;
  int rc = hydro_batch_workspace_bytes(p, n, common, &need);
  if (rc) return rc;
  if (!pool || !workspace) return fail(HYDRO_EINVAL, "null device pointer");
  if ((reinterpret_cast<uintptr_t>(pool) & 15) || (reinterpret_cast<uintptr_t>(workspace) & 15))
    return fail(HYDRO_EINVAL, "device pointers must be 16-byte aligned");
  if (ws_bytes < need) return fail(HYDRO_EINVAL, "workspace too small");
  const size_t esz = common->precision == HYDRO_FP64 ? 8 : 4;
  const int64_t pool_elems = int64_t(pool_bytes / esz);
  hydro_ctx* c = new (std::nothrow) hydro_ctx();
  if (!c) return fail(HYDRO_EINVAL, "out of host memory");
  c->desc = *common;
  c->batch = true;
  c->fp64 = common->precision == HYDRO_FP64;
  c->pool = pool;
  c->pool_bytes = pool_bytes;
  c->npatch = n;
  // patch extents: inside the pool, aligned, non-overlapping
  std::vector<std::pair<int64_t, int64_t>> spans;
  for (int32_t i = 0; i < n; ++i) {
    int32_t nn[3] = {p[i].nx, p[i].ny, p[i].nz};
    PatchDev P;
    int64_t len = 0;
    (void)patch_from(p[i], &P, &len);  // validated by hydro_batch_workspace_bytes
    if (P.plane * int64_t(esz) >= (int64_t(1) << 32)) {
      delete c;
      return fail(HYDRO_EINVAL, "a patch plane must be smaller than 4 GiB");
    }
    if (p[i].offset_elems < 0 || p[i].offset_elems + len > pool_elems) {
      delete c;
      return fail(HYDRO_EINVAL, "patch " + std::to_string(i) + " lies outside the pool");
    }
    if ((p[i].offset_elems * int64_t(esz)) % 16) {
      delete c;
      return fail(HYDRO_EINVAL, "patch offsets must be 16-byte aligned");
    }
    spans.push_back({p[i].offset_elems, p[i].offset_elems + len});
    c->patches.push_back(P);
    c->max_patch_cells = std::max<int64_t>(c->max_patch_cells, int64_t(nn[0]) * nn[1] * nn[2]);
    for (int a = 0; a < 3; ++a) c->active[a] = c->active[a] || nn[a] > 1;
  }
  std::sort(spans.begin(), spans.end());
  for (size_t i = 1; i < spans.size(); ++i)
    if (spans[i].first < spans[i - 1].second) {
      delete c;
      return fail(HYDRO_EINVAL, "patches overlap in the pool");
    }
  c->ws = static_cast<char*>(workspace);
  c->ws_bytes = ws_bytes;
  c->stream = static_cast<hipStream_t>(stream);
  c->scal = reinterpret_cast<DevScalars*>(c->ws);
  int32_t cap[5];
  max_items(c->patches, cap);
  BatchLayout L = batch_layout(n, cap);
  c->partials = reinterpret_cast<double*>(c->ws + L.partials);
  c->tslice = reinterpret_cast<double*>(c->ws + L.slice);
  c->pt = reinterpret_cast<double*>(c->ws + L.pt);
  c->pdt = reinterpret_cast<double*>(c->ws + L.pdt);
  c->psmax = reinterpret_cast<unsigned long long*>(c->ws + L.psmax);
  c->per_patch = (common->flags & HYDRO_BATCH_PER_PATCH_DT) != 0;
  c->d_patches = reinterpret_cast<PatchDev*>(c->ws + L.patches);
  for (int a = 0; a < 5; ++a) c->d_items[a] = reinterpret_cast<WorkItem*>(c->ws + L.items[a]);
  c->single = c->patches[0];
  // batch defaults: 4 cells per lane where every width allows, whole
  // columns per thread (patches are short), 8 workgroups per CU
  SweepCfg x = default_x(c->patches, c->fp64);
  if (x.v == 0 && c->active[0]) {
    delete c;
    return fail(HYDRO_EINVAL, "no x-sweep configuration fits every patch width");
  }
  c->cfg.ax[0] = x;
  for (int a = 1; a < 3; ++a) {
    SweepCfg s{};
    s.kind = kColumnKind;
    s.q = 256;
    s.s = 1;
    c->cfg.ax[a] = s;
  }
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      delete c;
      return fail(HYDRO_EDEVICE, "device query failed");
    }
    c->cfg.batch_blocks = prop.multiProcessorCount * 8;
  }
  if (hipMemcpyAsync(c->d_patches, c->patches.data(), c->patches.size() * sizeof(PatchDev),
                     hipMemcpyHostToDevice, c->stream) != hipSuccess) {
    delete c;
    return fail(HYDRO_EDEVICE, "patch table upload failed");
  }
  rc = rebuild_items(c);
  if (rc == HYDRO_OK) rc = common_init(c);
  if (rc == HYDRO_OK) rc = rebuild_items(c);
  if (rc) {
    hydro_destroy(c);
    return rc;
  }
  *out = c;
  return HYDRO_OK;
}

static int step_common(hydro_ctx* c, double dt, bool want_batch) {
  if (!c) return fail(HYDRO_EINVAL, "null context");
  if (!items_current(c)) return fail(HYDRO_ESTATE, "batch work lists out of date");
  if (c->batch != want_batch)
    return fail(HYDRO_ESTATE, want_batch ? "not a batch context" : "batch context: use hydro_batch_step");
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(HYDRO_EINVAL, "dt must be >= 0 and finite");
  if (dt > 0.0 || !c->dt_valid) HIP_TRY(set_step_dt(c, dt, c->stream));
  const int parity = int(c->step & 1);
  if (c->graph[parity]) {
    HIP_TRY(hipGraphLaunch(c->graph[parity], c->stream));
  } else {
    HIP_TRY(enqueue_step_kernels(c, parity, c->stream));
  }
  c->step += 1;
  c->dt_valid = true;
  c->totals_valid = true;
  return HYDRO_OK;
}

int hydro_step(hydro_ctx* c, double dt) { return step_common(c, dt, false); }

int hydro_batch_step(hydro_ctx* c, double dt) { return step_common(c, dt, true); }

}  // extern "C"

// ------------------------------------------------------------------------
// a step that allocates nothing (hydro_step_noalloc)
// ------------------------------------------------------------------------

// Device memory of hydro_step_noalloc: the scalar block, then the first
// level of the totals reduction, then the totals partials.  Every GPU the
// library runs on holds its own copy until the process ends; the calls on
// one GPU share it.  In host code its name stands for no device address:
// only the per-device address from hipGetSymbolAddress is ever used.
static __device__ __align__(256) unsigned char scratch[HYDRO_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kNoallocSlices = kScalarBytes;
constexpr size_t kNoallocParts =
    kNoallocSlices + (size_t(kTotalsSlices) * 6 * sizeof(double) + 255) / 256 * 256;
constexpr int64_t kNoallocMaxParts =
    int64_t((HYDRO_NOALLOC_SCRATCH_BYTES - kNoallocParts) / (6 * sizeof(double)));

struct NoallocDevice {
  void* ptr = nullptr;  // device address of this GPU's scratch
  int cu_count = 0;
};

std::mutex g_noalloc_mu;
std::map<int, NoallocDevice> g_noalloc;  // by device ordinal

// The current device's scratch address (looked up once per device, with the
// device current) and CU count.
int noalloc_device(NoallocDevice* out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc.find(dev);
  if (it == g_noalloc.end()) {
    NoallocDevice d;
    HIP_TRY(hipGetSymbolAddress(&d.ptr, HIP_SYMBOL(scratch)));
    if (!d.ptr) return fail(HYDRO_EDEVICE, "no device address for the static scratch");
    HIP_TRY(hipDeviceGetAttribute(&d.cu_count, hipDeviceAttributeMultiprocessorCount, dev));
    it = g_noalloc.emplace(dev, d).first;
  }
  *out = it->second;
  return HYDRO_OK;
}

}  // namespace

extern "C" {

int hydro_step_noalloc(const hydro_desc* d, void* state, size_t state_bytes, double dt,
                       int64_t step, void* stream, double* out) {
  g_last_error.clear();
  if (!d || !state) return fail(HYDRO_EINVAL, "null argument");
  int rc = check_common(d);
  if (rc) return rc;
  const int32_t n[3] = {d->nx, d->ny, d->nz};
  const double dx[3] = {d->dx, d->dy, d->dz};
  rc = check_extent(n, d->ng, dx);
  if (rc) return rc;
  if (reinterpret_cast<uintptr_t>(state) & 15)
    return fail(HYDRO_EINVAL, "the state must be 16-byte aligned");
  if (out && (reinterpret_cast<uintptr_t>(out) & 7))
    return fail(HYDRO_EINVAL, "out must be 8-byte aligned");
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(HYDRO_EINVAL, "dt must be >= 0 and finite");
  if (step < 0) return fail(HYDRO_EINVAL, "step must be >= 0");
  const PatchDev P = make_patch(n, d->ng, dx, 0);
  const int64_t esz = d->precision == HYDRO_FP64 ? 8 : 4;
  if (!plane_fits(P, esz)) return fail(HYDRO_EINVAL, "a state plane must be smaller than 4 GiB");
  if (state_bytes < size_t(P.plane) * 5 * size_t(esz))
    return fail(HYDRO_EINVAL, "state buffer too small");
  NoallocDevice nd;
  rc = noalloc_device(&nd);
  if (rc) return rc;
  // a host-side description of the grid; it owns nothing on the device
  hydro_ctx c;
  c.desc = *d;
  c.fp64 = d->precision == HYDRO_FP64;
  c.pool = state;
  c.pool_bytes = size_t(P.plane) * 5 * size_t(esz);
  c.stream = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(nd.ptr);
  c.scal = reinterpret_cast<DevScalars*>(base);
  c.tslice = reinterpret_cast<double*>(base + kNoallocSlices);
  c.partials = reinterpret_cast<double*>(base + kNoallocParts);
  c.single = P;
  for (int a = 0; a < 3; ++a) c.active[a] = n[a] > 1;
  c.cfg.ax[0] = default_x({P}, c.fp64);
  c.cfg.ax[1] = default_col(n[1]);
  c.cfg.ax[2] = default_col(n[2]);
  if (c.cfg.ax[0].v == 0 && c.active[0])
    return fail(HYDRO_EINVAL, "no valid x-sweep configuration for this width");
  c.cu_count = nd.cu_count;
  const int parity = int(step & 1);
  const std::vector<StepOp> ops = step_ops(&c, parity);
  const int64_t need = ops.empty() ? int64_t(chunks_for(int64_t(n[0]) * n[1] * n[2]))
                                   : sweep_parts(ops.back().L);
  if (need > kNoallocMaxParts)
    return fail(HYDRO_EINVAL, "this grid's totals need " + std::to_string(need) +
                                  " partial sums; the static scratch holds " +
                                  std::to_string(kNoallocMaxParts));
  hipStream_t st = c.stream;
  HIP_TRY(launch_init_scalars(c.scal, d->cfl, 0.0, 0.0, st));
  if (dt > 0.0) {
    HIP_TRY(launch_set_dt(c.scal, dt, st));
  } else {
    HIP_TRY(launch_cfl(reduce_launch(&c), st));
  }
  HIP_TRY(enqueue_step_kernels(&c, parity, st));
  if (out) HIP_TRY(launch_step_results(c.scal, out, st));
  return HYDRO_OK;
}

int hydro_sweep(hydro_ctx* c, int axis, double dt, int fold_cfl) {
  if (!c) return fail(HYDRO_EINVAL, "null context");
  if (!items_current(c)) return fail(HYDRO_ESTATE, "batch work lists out of date");
  if (axis < 0 || axis > 2) return fail(HYDRO_EINVAL, "axis must be 0, 1 or 2");
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(HYDRO_EINVAL, "dt must be >= 0 and finite");
  if (dt > 0.0 || !c->dt_valid) HIP_TRY(set_step_dt(c, dt, c->stream));
  if (c->active[axis] && (!c->batch || c->nitems[axis] > 0)) {
    HIP_TRY(launch_sweep(sweep_launch(c, axis, fold_cfl ? 1 : 0), c->stream));
  }
  if (c->batch) HIP_TRY(launch_reset_tickets(c->scal, c->stream));
  c->totals_valid = false;
  if (fold_cfl) {
    // the device dt becomes the CFL dt of the swept state (t is left alone)
    if (c->pp_live)
      HIP_TRY(launch_patch_dt(c->pt, c->pdt, c->psmax, c->npatch, c->scal, 0, c->stream));
    else
      HIP_TRY(launch_finish_cfl(c->scal, c->stream));
    c->dt_valid = true;
  } else {
    c->dt_valid = false;
  }
  return HYDRO_OK;
}

int hydro_cfl_dt(hydro_ctx* c, double* dt) {
  if (!c || !dt) return fail(HYDRO_EINVAL, "null argument");
  *dt = 0.0;
  HIP_TRY(set_step_dt(c, HYDRO_DT_CFL, c->stream));
  DevScalars s;
  int rc = read_scalars(c, &s);
  if (rc) return rc;
  c->dt_valid = true;
  if (s.error) return fail(HYDRO_ENUMERIC, "state holds rho <= 0, p <= 0 or a non-finite value");
  if (c->pp_live) {  // the smallest patch dt
    std::vector<double> d(size_t(c->npatch));
    HIP_TRY(hipMemcpyAsync(d.data(), c->pdt, d.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *dt = *std::min_element(d.begin(), d.end());
    return HYDRO_OK;
  }
  *dt = s.dt;
  return HYDRO_OK;
}

int hydro_totals(hydro_ctx* c, double out[6]) {
  if (!c || !out) return fail(HYDRO_EINVAL, "null argument");
  if (!items_current(c)) return fail(HYDRO_ESTATE, "batch work lists out of date");
  if (!c->totals_valid) {
    // the last sweep of the step before the current one (odd order, ending
    // with x, before the first step), replayed with dt = 0 and no stores:
    // its partition of the sums, hence the bits a step folds
    std::vector<StepOp> ops = step_ops(c, int((c->step + 1) & 1));
    if (ops.empty()) {
      HIP_TRY(launch_totals(reduce_launch(c), c->stream));
    } else {
      LaunchSweep L = ops.back().L;
      L.do_cfl = 0;
      L.totals_only = 1;
      // the state itself (a fused step's last launch reads the second buffer)
      L.pool = c->pool;
      if (L.dst) L.dst = c->pool;
      HIP_TRY(launch_sweep(L, c->stream));
      HIP_TRY(launch_totals_finish(c->partials, sweep_parts(L), c->tslice, c->scal, 0,
                                   c->stream));
    }
    c->totals_valid = true;
  }
  DevScalars s;
  int rc = read_scalars(c, &s);
  if (rc) return rc;
  for (int v = 0; v < 6; ++v) out[v] = s.totals[v];
  return HYDRO_OK;
}

int hydro_diag_pdf(hydro_ctx* c, int quantity, double lo, double hi, int32_t nbins,
                   int64_t* counts) {
  if (!c || !counts) return fail(HYDRO_EINVAL, "null argument");
  if (reinterpret_cast<uintptr_t>(counts) & 7)
    return fail(HYDRO_EINVAL, "counts must be 8-byte aligned");
  if (quantity < HYDRO_Q_RHO || quantity > HYDRO_Q_MACH) return fail(HYDRO_EINVAL, "unknown quantity");
  if (nbins < 1 || nbins > kPdfMaxBins) return fail(HYDRO_EINVAL, "nbins out of range");
  if (!std::isfinite(lo) || !std::isfinite(hi) || !(hi > lo))
    return fail(HYDRO_EINVAL, "the range must be finite with hi > lo");
  const double w = double(nbins) / (hi - lo);
  if (!std::isfinite(w)) return fail(HYDRO_EINVAL, "range too narrow");
  LaunchDiag L{};
  L.pool = c->pool;
  L.patches = c->batch ? c->d_patches : nullptr;
  L.single = c->single;
  L.npatch = c->batch ? c->npatch : 1;
  L.fp64 = c->fp64;
  L.gamma = c->desc.gamma;
  L.quantity = quantity;
  L.nbins = nbins;
  L.lo = lo;
  L.w = w;
  L.counts = reinterpret_cast<unsigned long long*>(counts);
  HIP_TRY(launch_diag_pdf(L, c->stream));
  return HYDRO_OK;
}

int hydro_diag_profile(hydro_ctx* c, int axis, double rho_lo, double rho_hi, double* out) {
  if (!c || !out) return fail(HYDRO_EINVAL, "null argument");
  if (c->batch) return fail(HYDRO_ESTATE, "slab profiles are defined for single grids");
  if (reinterpret_cast<uintptr_t>(out) & 7) return fail(HYDRO_EINVAL, "out must be 8-byte aligned");
  if (axis < 0 || axis > 2) return fail(HYDRO_EINVAL, "axis must be 0, 1 or 2");
  if (!std::isfinite(rho_lo) || !std::isfinite(rho_hi) || !(rho_hi > rho_lo))
    return fail(HYDRO_EINVAL, "the density range must be finite with rho_hi > rho_lo");
  const PatchDev& P = c->single;
  LaunchDiag L{};
  L.pool = c->pool;
  L.single = P;
  L.fp64 = c->fp64;
  L.gamma = c->desc.gamma;
  L.axis = axis;
  if (axis == 0) {
    L.chunks = int32_t(std::min<int64_t>(kProfileChunksX, int64_t(P.n[1]) * P.n[2]));
  } else {
    const int64_t slab = int64_t(P.n[0]) * P.n[axis == 2 ? 1 : 2];
    L.chunks = int32_t(std::max<int64_t>(
        1, std::min<int64_t>(kProfileChunksYZ, (slab + 255) / 256)));
  }
  L.rho_lo = rho_lo;
  L.drho = rho_hi - rho_lo;
  L.dx_axis = P.dx[axis];
  L.partials = c->profile_partials;
  L.out = out;
  HIP_TRY(launch_diag_profile(L, c->stream));
  return HYDRO_OK;
}

int hydro_diag_spectrum(hydro_ctx* c, double* out) {
  if (!c || !out) return fail(HYDRO_EINVAL, "null argument");
  if (c->batch) return fail(HYDRO_ESTATE, "the spectrum is defined for single grids");
  if (reinterpret_cast<uintptr_t>(out) & 7) return fail(HYDRO_EINVAL, "out must be 8-byte aligned");
  const PatchDev& P = c->single;
  int m = P.n[0];
  while (m > 1 && m % 2 == 0) m /= 2;
  while (m > 1 && m % 3 == 0) m /= 3;
  if (P.n[0] < 2 || P.n[0] > kSpecMaxLen || m != 1)
    return fail(HYDRO_EINVAL, "the x extent must be 2^a 3^b, from 2 to 1024");
  LaunchDiag L{};
  L.pool = c->pool;
  L.single = P;
  L.fp64 = c->fp64;
  L.gamma = c->desc.gamma;
  const int64_t lines = int64_t(P.n[1]) * P.n[2];
  L.chunks = int32_t(std::min<int64_t>(kSpecBlocks, lines));
  // the partial spectra share the profile partials' region
  const int64_t nmax = std::max(P.n[0], std::max(P.n[1], P.n[2]));
  if (int64_t(L.chunks) * (P.n[0] / 2 + 1) > nmax * kProfileChunksX * 5)
    return fail(HYDRO_EINVAL, "spectrum partials exceed the workspace");
  L.partials = c->profile_partials;
  L.out = out;
  HIP_TRY(launch_diag_spectrum(L, c->stream));
  return HYDRO_OK;
}

int hydro_diag_spectrum3d_workspace_bytes(hydro_ctx* c, size_t* bytes, int32_t* nshells) {
  if (!c || !bytes) return fail(HYDRO_EINVAL, "null argument");
  if (c->batch) return fail(HYDRO_ESTATE, "the shell spectrum is defined for single grids");
  if (!spec3_shape_ok(c->single))
    return fail(HYDRO_EINVAL, "every extent must be 2^a 3^b, from 1 to 1024");
  int nb = 0;
  *bytes = spec3_workspace_bytes(c->single, &nb);
  if (nshells) *nshells = nb;
  return HYDRO_OK;
}

int hydro_diag_spectrum3d(hydro_ctx* c, void* work, size_t work_bytes, double* out) {
  if (!c || !work || !out) return fail(HYDRO_EINVAL, "null argument");
  if (c->batch) return fail(HYDRO_ESTATE, "the shell spectrum is defined for single grids");
  if (!spec3_shape_ok(c->single))
    return fail(HYDRO_EINVAL, "every extent must be 2^a 3^b, from 1 to 1024");
  if (reinterpret_cast<uintptr_t>(out) & 7) return fail(HYDRO_EINVAL, "out must be 8-byte aligned");
  if (reinterpret_cast<uintptr_t>(work) & 255)
    return fail(HYDRO_EINVAL, "the workspace must be 256-byte aligned");
  if (work_bytes < spec3_workspace_bytes(c->single, nullptr))
    return fail(HYDRO_EINVAL, "workspace too small (hydro_diag_spectrum3d_workspace_bytes)");
  LaunchSpec3 L{};
  L.pool = c->pool;
  L.single = c->single;
  L.fp64 = c->fp64;
  L.cu_count = c->cu_count;
  L.work = work;
  L.out = out;
  HIP_TRY(launch_diag_spectrum3d(L, c->stream));
  return HYDRO_OK;
}

int hydro_burn(hydro_ctx* c, void* X, size_t x_bytes, const hydro_network* net, double dt,
               int32_t nsub) {
  if (!c || !X || !net) return fail(HYDRO_EINVAL, "null argument");
  if (c->batch) return fail(HYDRO_ESTATE, "the reactive source is defined for single grids");
  const int m = net->nspec;
  if (m < 2 || m > HYDRO_MAX_SPECIES) return fail(HYDRO_EINVAL, "nspec must be in [2, 20]");
  if (!std::isfinite(dt) || dt < 0.0) return fail(HYDRO_EINVAL, "dt must be finite and >= 0");
  if (nsub < 1 || nsub > 1000000) return fail(HYDRO_EINVAL, "nsub must be in [1, 1e6]");
  for (int i = 0; i < m - 1; ++i)
    if (!std::isfinite(net->A[i]) || net->A[i] < 0.0 || !std::isfinite(net->Ta[i]) ||
        !std::isfinite(net->q[i]))
      return fail(HYDRO_EINVAL, "network rates and energies must be finite (A >= 0)");
  const size_t esz = c->fp64 ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(X) % esz) return fail(HYDRO_EINVAL, "X is misaligned");
  if (x_bytes < size_t(m) * size_t(c->single.plane) * esz)
    return fail(HYDRO_EINVAL, "X holds fewer than nspec planes");
  static_assert(HYDRO_MAX_SPECIES == kBurnMaxSpecies, "species limit");
  LaunchBurn L{};
  L.pool = c->pool;
  L.X = X;
  L.single = c->single;
  L.fp64 = c->fp64;
  L.nspec = m;
  L.nsub = nsub;
  L.gamma = c->desc.gamma;
  L.h = dt / double(nsub);
  double b = 0.0;
  for (int s = 0; s < m; ++s) {
    L.B[s] = b;
    if (s < m - 1) {
      L.A[s] = net->A[s];
      L.Ta[s] = net->Ta[s];
      b += net->q[s];
    }
  }
  HIP_TRY(launch_burn(L, c->stream));
  c->totals_valid = false;
  c->dt_valid = false;
  return HYDRO_OK;
}

int hydro_fill_ghosts(hydro_ctx* c) {
  if (!c) return fail(HYDRO_EINVAL, "null context");
  LaunchAmr L{};
  L.op = kAmrFill;
  L.fp64 = c->fp64;
  L.pool = c->pool;
  L.patches = c->batch ? c->d_patches : nullptr;
  L.single = c->single;
  L.npatch = c->batch ? c->npatch : 1;
  L.ng = c->batch ? 0 : c->desc.ng;
  for (int i = 0; i < 6; ++i) L.bc[i] = c->desc.bc[i];
  int64_t most = 0;
  int maxg = 0;
  for (const PatchDev& P : c->batch ? c->patches : std::vector<PatchDev>{c->single}) {
    const int64_t g = P.ng;
    most = std::max(most, (P.n[0] + 2 * g) * (P.n[1] + 2 * g) * (P.n[2] + 2 * g));
    maxg = std::max(maxg, P.ng);
  }
  if (maxg == 0) return HYDRO_OK;  // no stored ghosts
  L.cells = most;
  HIP_TRY(launch_amr(L, c->stream));
  return HYDRO_OK;
}

namespace {

// Checks one link of a restriction (prolong = false) or prolongation.
int check_link(const hydro_ctx* c, const hydro_amr_link& k, bool prolong, bool ghosts_only) {
  if (k.fine < 0 || k.fine >= c->npatch || k.coarse < 0 || k.coarse >= c->npatch ||
      k.fine == k.coarse)
    return fail(HYDRO_EINVAL, "link patch indices out of range");
  const PatchDev& F = c->patches[size_t(k.fine)];
  const PatchDev& C = c->patches[size_t(k.coarse)];
  const int o[3] = {k.ox, k.oy, k.oz};
  for (int a = 0; a < 3; ++a) {
    if (F.n[a] % 2) return fail(HYDRO_EINVAL, "fine patch extents must be even");
    if (!prolong) {
      if (o[a] < 0 || o[a] + F.n[a] / 2 > C.n[a])
        return fail(HYDRO_EINVAL, "the fine patch must lie inside the coarse interior");
    } else {
      const int g = ghosts_only ? F.ng : 0;
      const int64_t lo = int64_t(o[a]) + ((-g) >> 1) - 1;
      const int64_t hi = int64_t(o[a]) + ((F.n[a] + g - 1) >> 1) + 1;
      if (lo < -C.ng || hi > int64_t(C.n[a]) + C.ng - 1)
        return fail(HYDRO_EINVAL, "the coarse patch (with its ghosts) must cover the parents "
                                  "and their neighbours");
    }
  }
  return HYDRO_OK;
}

// Coarse parents of a prolongation for a fine patch of interior extents n
// and g ghost layers written (0: the interior): the box of every parent of a
// written cell, and the shell of those outside the block [0, (n + 1) / 2)
// along some axis (the parents with a ghost child).
void prolong_parents(const int64_t n[3], int64_t g, int64_t* box, int64_t* shell) {
  const int64_t lo = (-g) >> 1;
  int64_t b = 1, inner = 1;
  for (int a = 0; a < 3; ++a) {
    b *= ((n[a] + g - 1) >> 1) - lo + 1;
    inner *= (n[a] + 1) >> 1;
  }
  *box = b;
  *shell = g > 0 ? b - inner : 0;
}

// A ghost prolongation walks only the shell's parents where they are at
// most 40 % of the box (2 ghost layers on 32^3 patches: 30 %, faster; 4
// layers: 49 %, slower than the whole box).
bool prolong_shell(int64_t box, int64_t shell) { return shell > 0 && 10 * shell <= 4 * box; }

int amr_links(hydro_ctx* c, const hydro_amr_link* links, int32_t n, int op, int ghosts_only) {
  if (!c || (!links && n > 0) || n < 0) return fail(HYDRO_EINVAL, "bad arguments");
  if (!c->batch) return fail(HYDRO_ESTATE, "AMR links join patches of a batch");
  for (int32_t i = 0; i < n; ++i) {
    int rc = check_link(c, links[i], op == kAmrProlong, ghosts_only != 0);
    if (rc) return rc;
  }
  for (int32_t b = 0; b < n; b += kAmrLinksPerLaunch) {
    LaunchAmr L{};
    L.op = op;
    L.fp64 = c->fp64;
    L.pool = c->pool;
    L.patches = c->d_patches;
    L.npatch = c->npatch;
    L.ghosts_only = ghosts_only;
    L.nlinks = std::min<int32_t>(kAmrLinksPerLaunch, n - b);
    int64_t most = 0, box = 0, shell = 0;
    for (int32_t i = 0; i < L.nlinks; ++i) {
      const hydro_amr_link& k = links[b + i];
      L.links[i] = AmrLink{k.fine, k.coarse, k.ox, k.oy, k.oz, 0};
      const PatchDev& F = c->patches[size_t(k.fine)];
      // restriction: coarse cells; prolongation: parents of the written cells
      if (op == kAmrRestrict) {
        most = std::max(most, int64_t(F.n[0] / 2) * (F.n[1] / 2) * (F.n[2] / 2));
      } else {
        const int64_t nf[3] = {F.n[0], F.n[1], F.n[2]};
        int64_t pb, ps;
        prolong_parents(nf, ghosts_only ? F.ng : 0, &pb, &ps);
        box = std::max(box, pb);
        shell = std::max(shell, ps);
      }
    }
    if (op == kAmrProlong) {
      L.shell = ghosts_only && prolong_shell(box, shell) ? 1 : 0;
      most = L.shell ? shell : box;
    }
    L.cells = most;
    HIP_TRY(launch_amr(L, c->stream));
  }
  c->totals_valid = false;
  c->dt_valid = false;
  return HYDRO_OK;
}

}  // namespace

int hydro_amr_restrict(hydro_ctx* c, const hydro_amr_link* links, int32_t n) {
  return amr_links(c, links, n, kAmrRestrict, 0);
}

int hydro_amr_prolong(hydro_ctx* c, const hydro_amr_link* links, int32_t n, int ghosts_only) {
  return amr_links(c, links, n, kAmrProlong, ghosts_only ? 1 : 0);
}

namespace {

// Largest number of coarse faces on one side of a fine patch of `fine`
// (stored boxes with `g` ghost layers).
int64_t level_maxface(const hydro_ctx* fine, int g) {
  int64_t m = 1;
  for (const PatchDev& P : fine->patches) {
    const int64_t n[3] = {(P.n[0] - 2 * g) / 2, (P.n[1] - 2 * g) / 2, (P.n[2] - 2 * g) / 2};
    m = std::max({m, n[1] * n[2], n[0] * n[2], n[0] * n[1]});
  }
  return m;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Checks the two levels of hydro_amr_step and their links.
int check_level(const hydro_ctx* coarse, const hydro_ctx* fine, const hydro_amr_link* links,
                int32_t n, int g) {
  if (!coarse || !fine || coarse == fine) return fail(HYDRO_EINVAL, "two distinct contexts needed");
  if (!coarse->batch || !fine->batch) return fail(HYDRO_ESTATE, "both levels must be batches");
  if (coarse->per_patch || fine->per_patch)
    return fail(HYDRO_EINVAL, "the level step takes one dt per level (no HYDRO_BATCH_PER_PATCH_DT)");
  if (coarse->fp64 != fine->fp64) return fail(HYDRO_EINVAL, "the levels differ in precision");
  if (coarse->stream != fine->stream) return fail(HYDRO_EINVAL, "the levels must share a stream");
  if (coarse->desc.gamma != fine->desc.gamma) return fail(HYDRO_EINVAL, "the levels differ in gamma");
  for (int a = 0; a < 3; ++a)
    if (coarse->desc.grav[a] != fine->desc.grav[a])
      return fail(HYDRO_EINVAL, "the levels differ in gravity");
  if (!items_current(coarse) || !items_current(fine))
    return fail(HYDRO_ESTATE, "batch work lists out of date");
  if (g < 2) return fail(HYDRO_EINVAL, "fine patches need at least 2 ghost layers");
  if (!links || n != fine->npatch) return fail(HYDRO_EINVAL, "one link per fine patch needed");
  if (n > 65535) return fail(HYDRO_EINVAL, "at most 65535 fine patches");
  const int m = (g + 1) / 2 + 1;  // coarse cells between a patch and the coarse edge
  std::vector<int> seen(size_t(fine->npatch), 0);
  for (int32_t i = 0; i < n; ++i) {
    const hydro_amr_link& k = links[i];
    if (k.fine < 0 || k.fine >= fine->npatch || k.coarse < 0 || k.coarse >= coarse->npatch)
      return fail(HYDRO_EINVAL, "link patch indices out of range");
    if (seen[size_t(k.fine)]++) return fail(HYDRO_EINVAL, "a fine patch is linked twice");
    const PatchDev& F = fine->patches[size_t(k.fine)];
    const PatchDev& C = coarse->patches[size_t(k.coarse)];
    const int o[3] = {k.ox, k.oy, k.oz};
    for (int a = 0; a < 3; ++a) {
      const int nf = F.n[a] - 2 * g;
      if (C.n[a] < 2 || nf < 2 || nf % 2)
        return fail(HYDRO_EINVAL, "every axis needs > 1 coarse cell and even fine extents");
      if (F.dx[a] * 2.0 != C.dx[a]) return fail(HYDRO_EINVAL, "fine cells must be half as wide");
      if (o[a] < m || int64_t(o[a]) + nf / 2 + m > C.n[a])
        return fail(HYDRO_EINVAL, "fine patch too close to the coarse edge");
    }
  }
  // separation: sort by (coarse patch, x offset) and compare each link only
  // with the later ones whose x range can still touch its own
  std::vector<int32_t> ord(static_cast<size_t>(n));
  for (int32_t i = 0; i < n; ++i) ord[size_t(i)] = i;
  std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
    return links[a].coarse != links[b].coarse ? links[a].coarse < links[b].coarse
                                              : links[a].ox < links[b].ox;
  });
  auto hi = [&](const hydro_amr_link& k, int a) {  // one past the covered coarse cells
    const PatchDev& F = fine->patches[size_t(k.fine)];
    const int o[3] = {k.ox, k.oy, k.oz};
    return o[a] + (F.n[a] - 2 * g) / 2;
  };
  for (int32_t u = 0; u < n; ++u) {
    const hydro_amr_link& k = links[ord[size_t(u)]];
    const int ok[3] = {k.ox, k.oy, k.oz};
    for (int32_t v = u + 1; v < n; ++v) {
      const hydro_amr_link& q = links[ord[size_t(v)]];
      if (q.coarse != k.coarse || q.ox >= hi(k, 0) + 1) break;  // apart along x, as all later
      const int oq[3] = {q.ox, q.oy, q.oz};
      bool apart = false;
      for (int a = 0; a < 3; ++a)
        apart = apart || oq[a] >= hi(k, a) + 1 || ok[a] >= hi(q, a) + 1;
      if (!apart) return fail(HYDRO_EINVAL, "fine patches must be a coarse cell apart");
    }
  }
  return HYDRO_OK;
}

// Launches one AMR operator over every link: one launch reading the device
// link table `dlinks` (the same links, uploaded).
int level_launch(const hydro_ctx* coarse, const hydro_ctx* fine, const hydro_amr_link* links,
                 int32_t n, int g, int op, const AmrLink* dlinks,
                 const std::function<void(LaunchAmr&)>& fill) {
  LaunchAmr L{};
  L.op = op;
  L.fp64 = coarse->fp64;
  L.pool = coarse->pool;
  L.patches = coarse->d_patches;
  L.npatch = coarse->npatch;
  L.fpool = fine->pool;
  L.fpatches = fine->d_patches;
  L.finset = g;
  L.nlinks = n;
  L.dlinks = dlinks;
  int64_t most = 0;  // most work items of one link (grid sizing)
  int64_t pbox = 0, pshell = 0;
  for (int32_t i = 0; i < n; ++i) {
    const PatchDev& F = fine->patches[size_t(links[i].fine)];
    const int64_t nf[3] = {F.n[0] - 2 * g, F.n[1] - 2 * g, F.n[2] - 2 * g};
    int64_t cells = 0;
    const int64_t mg = (g + 1) / 2 + 1;  // snapshot margin
    if (op == kAmrRestrict) {
      cells = (nf[0] / 2) * (nf[1] / 2) * (nf[2] / 2);
    } else if (op == kAmrSnapshot) {
      cells = (nf[0] / 2 + 2 * mg) * (nf[1] / 2 + 2 * mg) * (nf[2] / 2 + 2 * mg);
    } else if (op == kAmrProlong) {
      int64_t pb, ps;
      prolong_parents(nf, g, &pb, &ps);
      pbox = std::max(pbox, pb);
      pshell = std::max(pshell, ps);
    } else {
      cells = std::max({nf[1] * nf[2], nf[0] * nf[2], nf[0] * nf[1]}) / 4;
    }
    most = std::max(most, cells);
  }
  if (op == kAmrProlong) {
    L.shell = prolong_shell(pbox, pshell) ? 1 : 0;  // the level step fills ghosts only
    most = L.shell ? pshell : pbox;
  }
  L.cells = most;
  fill(L);
  HIP_TRY(launch_amr(L, coarse->stream));
  return HYDRO_OK;
}

// The sweeps of one step of a level (no fused plane launch), each preceded
// by the flux registers of its axis; then the step bookkeeping.
int level_sweeps(hydro_ctx* c, const hydro_ctx* coarse, const hydro_ctx* fine,
                 const hydro_amr_link* links, int32_t n, int g, bool fine_side, double dt,
                 double* reg, int64_t nreg, int64_t maxface, const AmrLink* dlinks) {
  static const int even[3] = {0, 1, 2}, odd[3] = {2, 1, 0};
  const int* order = (c->step & 1) ? odd : even;
  HIP_TRY(launch_set_dt(c->scal, dt, c->stream));
  for (int i = 0; i < 3; ++i) {
    const int ax = order[i];
    int rc = level_launch(coarse, fine, links, n, g, kAmrFlux, dlinks, [&](LaunchAmr& L) {
      L.reg = reg;
      L.nreg = nreg;
      L.maxface = int32_t(maxface);
      L.axis = ax;
      L.fine = fine_side ? 1 : 0;
      if (fine_side) L.cells *= ax == 0 ? 16 : 4;  // lanes per coarse face
      L.dt = dt;
      L.weight = dt;
      L.gamma = c->desc.gamma;
      L.grav = c->desc.grav[ax];
    });
    if (rc) return rc;
    if (c->nitems[ax] > 0) HIP_TRY(launch_sweep(sweep_launch(c, ax, i == 2 ? 1 : 0), c->stream));
  }
  HIP_TRY(launch_finish_step(c->scal, c->stream));
  c->step += 1;
  c->dt_valid = false;
  c->totals_valid = false;
  return HYDRO_OK;
}

}  // namespace

int hydro_amr_cfl_dt(hydro_ctx* coarse, hydro_ctx* fine, double* dt) {
  if (!coarse || !fine || !dt) return fail(HYDRO_EINVAL, "null argument");
  *dt = 0.0;
  if (!coarse->batch || !fine->batch) return fail(HYDRO_ESTATE, "both levels must be batches");
  double dc = 0.0, df = 0.0;
  int rc = hydro_cfl_dt(coarse, &dc);
  if (rc) return rc;
  rc = hydro_cfl_dt(fine, &df);
  if (rc) return rc;
  *dt = std::min(dc, 2.0 * df);  // two fine substeps of dt/2 per coarse step
  return HYDRO_OK;
}

int hydro_amr_step_workspace_bytes(const hydro_ctx* coarse, const hydro_ctx* fine,
                                   int32_t fine_ng, size_t* bytes) {
  if (!coarse || !fine || !bytes) return fail(HYDRO_EINVAL, "null argument");
  if (!coarse->batch || !fine->batch) return fail(HYDRO_ESTATE, "both levels must be batches");
  if (fine_ng < 2) return fail(HYDRO_EINVAL, "fine patches need at least 2 ghost layers");
  const int64_t nreg = int64_t(fine->npatch) * 30 * level_maxface(fine, fine_ng);
  *bytes = align256(coarse->pool_bytes) + align256(size_t(2 * nreg) * sizeof(double)) +
           size_t(fine->npatch) * sizeof(AmrLink);
  return HYDRO_OK;
}

int hydro_amr_step(hydro_ctx* coarse, hydro_ctx* fine, const hydro_amr_link* links, int32_t n,
                   int32_t fine_ng, double dt, uint32_t flags, void* workspace,
                   size_t ws_bytes) {
  int rc = check_level(coarse, fine, links, n, fine_ng);
  if (rc) return rc;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(HYDRO_EINVAL, "dt must be > 0 and finite");
  if (flags & ~uint32_t(HYDRO_AMR_NO_REFLUX)) return fail(HYDRO_EINVAL, "unknown flags");
  size_t need = 0;
  rc = hydro_amr_step_workspace_bytes(coarse, fine, fine_ng, &need);
  if (rc) return rc;
  if (!workspace || ws_bytes < need) return fail(HYDRO_EINVAL, "workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(HYDRO_EINVAL, "workspace misaligned");
  const int g = fine_ng;
  const int64_t maxface = level_maxface(fine, g);
  const int64_t nreg = int64_t(n) * 30 * maxface;
  char* ws = static_cast<char*>(workspace);
  void* cold = ws;
  double* reg = reinterpret_cast<double*>(ws + align256(coarse->pool_bytes));
  AmrLink* dlinks = reinterpret_cast<AmrLink*>(ws + align256(coarse->pool_bytes) +
                                               align256(size_t(2 * nreg) * sizeof(double)));
  hipStream_t st = coarse->stream;
  std::vector<AmrLink> hl(static_cast<size_t>(n));
  for (int32_t i = 0; i < n; ++i)
    hl[size_t(i)] = AmrLink{links[i].fine, links[i].coarse, links[i].ox, links[i].oy, links[i].oz, 0};
  HIP_TRY(launch_amr_upload(dlinks, hl.data(), n, st));
  // the start-of-step coarse cells that ghost prolongation reads: every
  // cell within ceil(g/2) + 1 of a covered box (the parents of the ghost
  // shell and their neighbours), at their pool offsets
  rc = level_launch(coarse, fine, links, n, g, kAmrSnapshot, dlinks, [&](LaunchAmr& L) {
    L.cold = cold;
    L.margin = (g + 1) / 2 + 1;
  });
  if (rc) return rc;
  HIP_TRY(hipMemsetAsync(reg, 0, size_t(2 * nreg) * sizeof(double), st));
  // 1. the coarse step, registering its fluxes through the coarse-fine faces
  rc = level_sweeps(coarse, coarse, fine, links, n, g, false, dt, reg, nreg, maxface, dlinks);
  if (rc) return rc;
  // 2. two fine substeps, ghosts from the coarse data interpolated in time
  for (int s = 0; s < 2; ++s) {
    rc = level_launch(coarse, fine, links, n, g, kAmrProlong, dlinks, [&](LaunchAmr& L) {
      L.ghosts_only = 1;
      if (s == 0) {
        L.pool = cold;  // theta = 0: the start-of-step cells themselves
      } else {
        L.cold = cold;
        L.theta = 0.5 * s;
      }
    });
    if (rc) return rc;
    rc = level_sweeps(fine, coarse, fine, links, n, g, true, 0.5 * dt, reg, nreg, maxface,
                      dlinks);
    if (rc) return rc;
  }
  // 3. restriction, 4. refluxing
  rc = level_launch(coarse, fine, links, n, g, kAmrRestrict, dlinks, [](LaunchAmr&) {});
  if (rc) return rc;
  if (!(flags & HYDRO_AMR_NO_REFLUX)) {
    for (int ax = 0; ax < 3; ++ax)
      for (int side = 0; side < 2; ++side) {
        rc = level_launch(coarse, fine, links, n, g, kAmrReflux, dlinks, [&](LaunchAmr& L) {
          L.reg = reg;
          L.nreg = nreg;
          L.maxface = int32_t(maxface);
          L.axis = ax;
          L.side = side;
        });
        if (rc) return rc;
      }
  }
  return HYDRO_OK;
}

int hydro_get_time(hydro_ctx* c, double* t, int64_t* step) {
  if (!c) return fail(HYDRO_EINVAL, "null context");
  DevScalars s;
  int rc = read_scalars(c, &s);
  if (rc) return rc;
  double tt = s.t;
  if (c->pp_live) {  // the earliest patch time
    std::vector<double> pt(size_t(c->npatch));
    HIP_TRY(hipMemcpyAsync(pt.data(), c->pt, pt.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    tt = *std::min_element(pt.begin(), pt.end());
  }
  c->t_host = tt;
  if (t) *t = tt;
  if (step) *step = c->step;
  return HYDRO_OK;
}

int hydro_batch_times(hydro_ctx* c, double* t, double* dt) {
  if (!c || !t || !dt) return fail(HYDRO_EINVAL, "null argument");
  if (!c->batch) return fail(HYDRO_ESTATE, "not a batch context");
  const size_t n = size_t(c->npatch);
  if (c->pp_live) {
    HIP_TRY(hipMemcpyAsync(t, c->pt, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(dt, c->pdt, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return HYDRO_OK;
  }
  DevScalars s;
  int rc = read_scalars(c, &s);
  if (rc) return rc;
  for (size_t i = 0; i < n; ++i) {
    t[i] = s.t;
    dt[i] = s.dt;
  }
  return HYDRO_OK;
}

int hydro_set_time(hydro_ctx* c, double t, int64_t step) {
  if (!c) return fail(HYDRO_EINVAL, "null context");
  if (!std::isfinite(t) || step < 0) return fail(HYDRO_EINVAL, "bad time or step");
  HIP_TRY(launch_set_time(c->scal, t, c->t_end, c->stream));
  if (c->pp_live) HIP_TRY(launch_fill(c->pt, c->npatch, t, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->t_host = t;
  c->step = step;
  c->dt_valid = false;
  c->totals_valid = false;
  return HYDRO_OK;
}

int hydro_set_t_end(hydro_ctx* c, double t_end) {
  if (!c) return fail(HYDRO_EINVAL, "null context");
  if (!std::isfinite(t_end)) return fail(HYDRO_EINVAL, "t_end must be finite");
  double t = 0.0;
  int rc = hydro_get_time(c, &t, nullptr);
  if (rc) return rc;
  c->t_end = t_end > 0.0 ? t_end : 0.0;
  HIP_TRY(launch_set_time(c->scal, t, c->t_end, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->dt_valid = false;
  return HYDRO_OK;
}

int hydro_state_changed(hydro_ctx* c) {
  if (!c) return fail(HYDRO_EINVAL, "null context");
  c->dt_valid = false;
  c->totals_valid = false;
  return HYDRO_OK;
}

int hydro_get_error(hydro_ctx* c) {
  if (!c) return fail(HYDRO_EINVAL, "null context");
  DevScalars s;
  int rc = read_scalars(c, &s);
  if (rc) return rc;
  return s.error ? fail(HYDRO_ENUMERIC, "sticky numeric error flag is set") : HYDRO_OK;
}

int hydro_clear_error(hydro_ctx* c) {
  if (!c) return fail(HYDRO_EINVAL, "null context");
  HIP_TRY(launch_clear_error(c->scal, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return HYDRO_OK;
}

int hydro_get_config(hydro_ctx* c, char* buf, size_t len) {
  if (!c || !buf || len == 0) return fail(HYDRO_EINVAL, "bad argument");
  std::string s = cfg_text(c->cfg);
  if (s.size() + 1 > len) return fail(HYDRO_EINVAL, "buffer too small");
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return HYDRO_OK;
}

int hydro_set_config(hydro_ctx* c, const char* text) {
  if (!c || !text) return fail(HYDRO_EINVAL, "bad argument");
  Config cf = c->cfg;
  if (!parse_cfg(text, cf)) return fail(HYDRO_EINVAL, "cannot parse configuration");
  if (c->active[0] &&
      !x_cfg_ok_all(cf.ax[0], c->batch ? c->patches : std::vector<PatchDev>{c->single},
                    c->fp64))
    return fail(HYDRO_EINVAL, "invalid x config");
  for (int a = 1; a < 3; ++a)
    if (c->active[a] && !col_cfg_ok(cf.ax[a])) return fail(HYDRO_EINVAL, "invalid column config");
  if (c->batch && (cf.batch_blocks < 1 || cf.batch_blocks > 65536))
    return fail(HYDRO_EINVAL, "invalid persistent grid size");
  if (cf.batch_fuse && c->batch && !plane_ok(c, cf))
    return fail(HYDRO_EINVAL, "fused plane sweeps do not apply to these patches");
  if (cf.batch_zplane && !zplane_ok(c, cf))
    return fail(HYDRO_EINVAL, "the x-z plane z sweep does not apply to these patches");
  if (cf.batch_fuse && !c->batch && !win_ok(c, cf))
    return fail(HYDRO_EINVAL, "the fused x+y step does not apply (HYDRO_FLAG_FUSE_XY, even x "
                              "and y extents >= 64 and 64 (FP32) or 32 (FP64), active z; "
                              "w:v=1 or 2)");
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->cfg = cf;
  if (c->batch) {
    int rc = rebuild_items(c);
    if (rc) return rc;
  }
  return capture_graphs(c);
}

int hydro_time_sweeps(hydro_ctx* c, int reps, double ms[3]) {
  if (!c || !ms || reps < 1) return fail(HYDRO_EINVAL, "bad argument");
  HIP_TRY(launch_timing_begin(c->scal, c->stream));
  const bool pp = c->pp_live;
  c->pp_live = false;  // the timing runs take the one dt = 0 (state unchanged)
  int rc = HYDRO_OK;
  for (int a = 0; a < 3; ++a) {
    ms[a] = 0.0;
    if (!c->active[a] || (c->batch && c->nitems[a] == 0)) continue;
    rc = time_sweep(c, a, reps, &ms[a]);
    if (rc) break;
  }
  c->pp_live = pp;
  HIP_TRY(launch_timing_end(c->scal, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return rc;
}

int hydro_profile_step(hydro_ctx* c, double dt, double ms[4]) {
  if (!c || !ms) return fail(HYDRO_EINVAL, "bad argument");
  if (!items_current(c)) return fail(HYDRO_ESTATE, "batch work lists out of date");
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(HYDRO_EINVAL, "dt must be >= 0 and finite");
  for (int i = 0; i < 4; ++i) ms[i] = 0.0;
  if (dt > 0.0 || !c->dt_valid) HIP_TRY(set_step_dt(c, dt, c->stream));
  const std::vector<StepOp> ops = step_ops(c, int(c->step & 1));
  hipEvent_t ev[2];
  for (int i = 0; i < 2; ++i) HIP_TRY(hipEventCreate(&ev[i]));
  int rc = HYDRO_OK;
  for (const StepOp& op : ops) {
    float t = 0.f;
    if (hipEventRecord(ev[0], c->stream) != hipSuccess ||
        launch_sweep(op.L, c->stream) != hipSuccess ||
        hipEventRecord(ev[1], c->stream) != hipSuccess ||
        hipEventSynchronize(ev[1]) != hipSuccess ||
        hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess) {
      rc = fail(HYDRO_EDEVICE, "profiled sweep failed");
      break;
    }
    ms[op.slot] = double(t);
  }
  if (rc == HYDRO_OK && finish_step_launches(c, ops, c->stream) != hipSuccess)
    rc = fail(HYDRO_EDEVICE, "step bookkeeping launch failed");
  for (int i = 0; i < 2; ++i) (void)hipEventDestroy(ev[i]);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  ms[3] = ms[0] + ms[1] + ms[2];
  c->step += 1;
  c->dt_valid = true;
  c->totals_valid = true;
  return HYDRO_OK;
}

int hydro_stream_ceiling(hydro_ctx* c, int reps, double* ms) {
  if (!c || !ms || reps < 1) return fail(HYDRO_EINVAL, "bad argument");
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  int rc = HYDRO_OK;
  const int64_t bytes = int64_t(c->pool_bytes) & ~int64_t(15);
  if (launch_stream(c->pool, bytes, c->stream) != hipSuccess ||
      hipEventRecord(a, c->stream) != hipSuccess)
    rc = fail(HYDRO_EDEVICE, "stream launch failed");
  for (int i = 0; i < reps && rc == HYDRO_OK; ++i)
    if (launch_stream(c->pool, bytes, c->stream) != hipSuccess)
      rc = fail(HYDRO_EDEVICE, "stream launch failed");
  float t = 0.f;
  if (rc == HYDRO_OK && (hipEventRecord(b, c->stream) != hipSuccess ||
                         hipEventSynchronize(b) != hipSuccess ||
                         hipEventElapsedTime(&t, a, b) != hipSuccess))
    rc = fail(HYDRO_EDEVICE, "stream timing failed");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc == HYDRO_OK) *ms = double(t) / reps;
  return rc;
}

int hydro_destroy(hydro_ctx* c) {
  if (!c) return HYDRO_OK;
  (void)hipStreamSynchronize(c->stream);
  destroy_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
  return HYDRO_OK;
}

}  // extern "C"
