// Host side of the libbgk C interface (include/bgk.h): argument checks,
// workspace layout, and the order of kernel launches of one time step.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "bgk_internal.h"
#include "adjoint_plan.h"

namespace bgk {

// Device scratch of bgk_objective_static (the per-particle terms of the
// objective): a fixed array in every GPU's copy of the code object, held
// until the process ends.  Host code never uses its name as an address: the
// address of each GPU's copy is looked up once per device, with that device
// current, and kept here.
static __device__ __align__(256) double scratch[BGK_STATIC_SCRATCH_PARTICLES];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch;   // per device ordinal, null until looked up
}  // namespace

// Looks up this device's copy of the scratch (the device must be current).
hipError_t static_scratch_setup(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0) return hipErrorInvalidDevice;
  if (static_cast<size_t>(device) >= g_scratch.size()) g_scratch.resize(device + 1, nullptr);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* static_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device >= 0 && static_cast<size_t>(device) < g_scratch.size() ? g_scratch[device]
                                                                        : nullptr;
}

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Cells per axis: as many as possible with cell size 1/nca >= h (with a
// margin against rounding), and no more than about one particle per cell.
int cells_per_axis(const bgk_config& cfg) {
  int nca = static_cast<int>(std::floor(1.0 / cfg.h));
  const int cap_n = std::max(1, static_cast<int>(std::floor(
                                    std::pow(static_cast<double>(cfg.n_particles), 1.0 / cfg.dim))));
  nca = std::max(1, std::min(nca, cap_n));
  while (nca > 1 && 1.0 / nca < cfg.h * (1.0 + 1e-9)) --nca;
  return nca;
}

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

const char* status_text(int code) {
  switch (code) {
    case BGK_OK: return "ok";
    case BGK_EINVAL: return "invalid argument or configuration";
    case BGK_ENOMEM: return "workspace too small";
    case BGK_ENBR_OVERFLOW: return "neighbour count exceeds max_neighbors";
    case BGK_ESINGULAR: return "singular least-squares system (too few neighbours or pivot <= 0)";
    case BGK_ENONPHYS: return "non-physical moments (rho <= 0, T <= 0 or NaN)";
    case BGK_EDEVICE: return "HIP runtime error";
    case BGK_ENOTSUP: return "not supported";
    default: return "unknown error";
  }
}

int fail(Ctx* c, int code, const char* what) {
  if (c) {
    c->last_error = std::string(status_text(code)) + ": " + what;
  }
  return code;
}

int hip_fail(Ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return BGK_OK;
  if (c) c->last_error = std::string(what) + ": " + hipGetErrorString(e);
  return BGK_EDEVICE;
}

bool config_ok(const bgk_config& g) {
  return (g.dim == 2 || g.dim == 3) && g.n_particles > 0 && g.nv >= 2 && g.nv <= 1024 && g.nv % 2 == 0 &&
         g.wls_degree >= 0 && g.wls_degree <= 2 && g.max_neighbors >= g.dim + 2 &&
         g.max_neighbors <= 255 && (g.move == 0 || g.move == 1) && g.precision >= BGK_FP64 &&
         g.precision <= BGK_BF16 && (g.flags & ~(BGK_FLAG_GENERIC | BGK_FLAG_ADJOINT | BGK_FLAG_PARTICLES)) == 0 &&
         (!(g.flags & BGK_FLAG_ADJOINT) || g.precision != BGK_BF16) && g.vmax > 0 && g.h > 0 && g.alpha > 0 &&
         g.kn > 0 && g.dt > 0 && g.wall_T > 0 && g.dx > 0 && std::isfinite(g.lid_velocity) &&
         ipow(g.nv, g.dim) <= INT32_MAX / 4 &&
         (!(g.flags & BGK_FLAG_PARTICLES) || ipow(lattice_nodes(g), g.dim) < INT32_MAX / 2) &&
         static_cast<int64_t>(g.n_particles) * g.max_neighbors * g.dim * g.dim < INT32_MAX;
}

}  // namespace

size_t workspace_layout(const bgk_config& cfg, char* base, Dev* d, Adj* adj, Pm* pm,
                        MoveAdj* madj) {
  const int64_t N = cfg.n_particles, cap = cfg.max_neighbors, D = cfg.dim, DD = D * D;
  const int64_t ncell = ipow(cells_per_axis(cfg), cfg.dim);
  // patch unions for any patch size (chosen at init): at most (N+1)/2
  // patches and (N+3)*cap entries
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  Dev t{};
  t.err = reinterpret_cast<int32_t*>(take(kErrWords * 4));
  t.wall_id = reinterpret_cast<int32_t*>(take(N * 4));
  t.wall_list = reinterpret_cast<int32_t*>(take(N * 4));
  t.key = reinterpret_cast<int32_t*>(take(N * 4));
  t.cstart = reinterpret_cast<int32_t*>(take((2 * ncell + 1) * 4));
  t.ccursor = reinterpret_cast<int32_t*>(take(2 * ncell * 4));
  t.cperm = reinterpret_cast<int32_t*>(take(N * 4));
  t.cperm2 = reinterpret_cast<int32_t*>(take(N * 4));
  t.xs = reinterpret_cast<double*>(take(N * D * 8));
  t.ncnt = reinterpret_cast<int32_t*>(take(N * 4));
  t.nidx = reinterpret_cast<int32_t*>(take(N * cap * 4));
  t.ops64 = cfg.precision == BGK_FP64 ? reinterpret_cast<double*>(take(N * cap * DD * 8)) : nullptr;
  t.ops32 = cfg.precision != BGK_FP64 ? reinterpret_cast<float*>(take(N * cap * DD * 4)) : nullptr;
  t.wcnt = reinterpret_cast<int32_t*>(take(N * 4));
  t.widx = reinterpret_cast<int32_t*>(take(N * cap * 4));
  t.wc0 = reinterpret_cast<double*>(take(N * cap * 8));
  t.whb = reinterpret_cast<double*>(take(N * 8));
  t.ucount = reinterpret_cast<int32_t*>(take((N + 1) / 2 * 4));
  t.uj = reinterpret_cast<int32_t*>(take((N + 3) * cap * 4));
  t.ue = reinterpret_cast<uint32_t*>(take((N + 3) * cap * 4));
  t.jpart = reinterpret_cast<double*>(take(N * 8));
  t.scheck = reinterpret_cast<double*>(take((N + 1) * kCheckTerms * 8));
  const int64_t npw = wall_patches_max(N, cfg.dim);
  t.wpl = reinterpret_cast<int32_t*>(take(npw * kWallPatch * 4));
  t.wucount = reinterpret_cast<int32_t*>(take(npw * 4));
  t.wuj = reinterpret_cast<int32_t*>(take(npw * kWallPatch * cap * 4));
  t.wue = reinterpret_cast<uint32_t*>(take(npw * kWallPatch * cap * 4));
  if (d) *d = t;
  if (cfg.flags & BGK_FLAG_ADJOINT) {
    // The reverse step reads the wall rows of f^{n+1} before it writes the
    // interior rows of lam_ft, and never reads a wall row of lam_ft: the two
    // share storage.
    const int64_t NC = D == 2 ? 2 : 1, F = NC * N * ipow(cfg.nv, cfg.dim);
    Adj a{};
    a.tidx = reinterpret_cast<int32_t*>(take(N * cap * 4));
    a.wtstart = reinterpret_cast<int32_t*>(take((N + 1) * 4));
    a.wtcursor = reinterpret_cast<int32_t*>(take(N * 4));
    a.wt = reinterpret_cast<int32_t*>(take(N * cap * 4));
    const int64_t fs = cfg.precision == BGK_FP64 ? 8 : 4;  // f storage
    a.ft = take(F * fs);
    a.lam_ft = take(F * fs);
    a.f1 = a.lam_ft;
    a.rho1 = reinterpret_cast<double*>(take(N * 8));
    a.U1 = reinterpret_cast<double*>(take(N * D * 8));
    a.T1 = reinterpret_cast<double*>(take(N * 8));
    a.larr = take(F * fs);
    a.lidpart = reinterpret_cast<double*>(take(N * 8));
    const AdjPlan ap = adj_plan(cfg);
    const size_t npa = (N + ap.P - 1) / ap.P;
    a.gpart = reinterpret_cast<double*>(
        take(static_cast<size_t>(std::max(ap.tiles, ap.tiles_w)) * D * N * 8));
    a.ucount = reinterpret_cast<int32_t*>(take(npa * 4));
    a.uj = reinterpret_cast<int32_t*>(take(npa * ap.P * cap * 4));
    a.ue = reinterpret_cast<uint32_t*>(take(npa * ap.P * cap * 4));
    if (adj) *adj = a;
    if (cfg.move) {
      MoveAdj v{};
      v.wpos = reinterpret_cast<int32_t*>(take(N * 4));
      v.lamU_eff = reinterpret_cast<double*>(take(D * N * 8));
      v.xpass = reinterpret_cast<double*>(take(D * N * 8));
      v.lam_a = reinterpret_cast<double*>(take(N * cap * DD * 8));
      v.lc0 = reinterpret_cast<double*>(take(N * cap * 8));
      v.xc = reinterpret_cast<double*>(take(N * cap * D * 8));
      v.xs = reinterpret_cast<double*>(take(N * D * 8));
      v.wxc = reinterpret_cast<double*>(take(N * cap * D * 8));
      v.wxs = reinterpret_cast<double*>(take(N * D * 8));
      if (madj) *madj = v;
    }
  }
  if (cfg.flags & BGK_FLAG_PARTICLES) {
    const int64_t nodes = ipow(lattice_nodes(cfg), cfg.dim);
    Pm p{};
    p.nn = reinterpret_cast<int32_t*>(take(N * 4));
    p.partner = reinterpret_cast<int32_t*>(take(N * 4));
    p.keep = reinterpret_cast<int32_t*>(take((N + 1) * 4));
    p.mid = reinterpret_cast<int32_t*>(take((N + 1) * 4));
    p.hole = reinterpret_cast<int32_t*>(take((nodes + 1) * 4));
    if (pm) *pm = p;
  }
  return off;
}

bool use_fused(const Ctx& c) {
  return !(c.cfg.flags & BGK_FLAG_GENERIC) && fused_supported(c);
}

hipEvent_t take_event(Ctx& c) {
  if (!c.event_pool.empty()) {
    hipEvent_t e = c.event_pool.back();
    c.event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// S1-S3 and the wall rows into the workspace, then the patch unions.
static int build_geometry(Ctx& c, const double* x) {
  hipError_t e = launch_cells(c, x);
  if (e == hipSuccess) e = launch_neighbors(c, x, c.d.ncnt, c.d.nidx);
  if (e == hipSuccess)
    e = launch_wls(c, x, c.d.ncnt, c.d.nidx, nullptr, c.d.ops64, c.d.ops32, nullptr);
  if (e == hipSuccess) e = launch_wall_stencil(c, x);
  if (e == hipSuccess) e = launch_patches(c);
  c.adj_valid = false;
  c.pm_valid = false;
  if (e != hipSuccess) return hip_fail(&c, e, "geometry launch");
  c.geom_valid = true;
  return BGK_OK;
}

}  // namespace bgk

using bgk::Ctx;

extern "C" {

int bgk_workspace_bytes(const bgk_config* cfg, size_t* bytes) {
  if (!cfg || !bytes || !bgk::config_ok(*cfg)) return BGK_EINVAL;
  *bytes = bgk::workspace_layout(*cfg, nullptr, nullptr, nullptr, nullptr);
  return BGK_OK;
}

int bgk_init(const bgk_config* cfg, const int32_t* wall_id, void* workspace, size_t ws_bytes,
             void* hip_stream, bgk_ctx** out) {
  if (!out) return BGK_EINVAL;
  *out = nullptr;
  if (!cfg || !wall_id || !workspace || !bgk::config_ok(*cfg)) return BGK_EINVAL;
  const size_t need = bgk::workspace_layout(*cfg, nullptr, nullptr, nullptr, nullptr);
  if (ws_bytes < need) return BGK_ENOMEM;
  bgk_ctx* h = new (std::nothrow) bgk_ctx;
  if (!h) return BGK_ENOMEM;
  Ctx& c = h->c;
  c.cfg = *cfg;
  c.stream = static_cast<hipStream_t>(hip_stream);
  c.N = cfg->n_particles;
  c.D = cfg->dim;
  c.NC = cfg->dim == 2 ? 2 : 1;
  c.NV = static_cast<int>(bgk::ipow(cfg->nv, cfg->dim));
  c.cap = cfg->max_neighbors;
  c.DD = c.D * c.D;
  c.nca = bgk::cells_per_axis(*cfg);
  c.ncell = static_cast<int>(bgk::ipow(c.nca, c.D));
  c.lid = cfg->lid_velocity;
  bgk::workspace_layout(*cfg, static_cast<char*>(workspace), &c.d, &c.adj, &c.pm, &c.madj);
  c.nl = bgk::lattice_nodes(*cfg);
  c.nodes = bgk::ipow(c.nl, c.D);
  hipError_t e = hipGetDevice(&c.device);
  if (e == hipSuccess) e = bgk::static_scratch_setup(c.device);
  // wall ids: read once to count and list the wall particles
  std::vector<int32_t> wid(c.N);
  if (e == hipSuccess)
    e = hipMemcpyAsync(wid.data(), wall_id, sizeof(int32_t) * c.N, hipMemcpyDeviceToHost, c.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  if (e != hipSuccess) {
    delete h;
    return BGK_EDEVICE;
  }
  // wall particles listed face by face (owner wall, then index): neighbours
  // in the list are neighbours on the face and share interpolation stencils
  std::vector<int32_t> wl;
  for (int i = 0; i < c.N; ++i) {
    if (wid[i] < 0 || wid[i] > 2 * c.D) {
      delete h;
      return BGK_EINVAL;
    }
  }
  for (int w = 1; w <= 2 * c.D; ++w)
    for (int i = 0; i < c.N; ++i)
      if (wid[i] == w) wl.push_back(i);
  c.Nw = static_cast<int>(wl.size());
  c.Ni = c.N - c.Nw;
  c.tp = bgk::choose_patch(c.D, cfg->precision, c.NV, c.Ni);
  c.npatch = (c.Ni + c.tp - 1) / c.tp;
  c.ucap = c.tp * c.cap;
  // 3D wall patches: runs of kWallPatch consecutive entries of one face
  std::vector<int32_t> wp;
  if (c.D == 3) {
    for (int s0 = 0; s0 < c.Nw;) {
      int s1 = s0;
      while (s1 < c.Nw && wid[wl[s1]] == wid[wl[s0]]) ++s1;
      for (int q = s0; q < s1; q += bgk::kWallPatch)
        for (int t = 0; t < bgk::kWallPatch; ++t) wp.push_back(q + t < s1 ? q + t : -1);
      s0 = s1;
    }
  }
  c.npw = static_cast<int>(wp.size()) / bgk::kWallPatch;
  c.wucap = bgk::kWallPatch * c.cap;
  int32_t zeros[bgk::kErrWords] = {0};
  e = hipMemcpyAsync(c.d.wall_id, wid.data(), sizeof(int32_t) * c.N, hipMemcpyHostToDevice,
                     c.stream);
  if (e == hipSuccess && c.Nw > 0)
    e = hipMemcpyAsync(c.d.wall_list, wl.data(), sizeof(int32_t) * c.Nw, hipMemcpyHostToDevice,
                       c.stream);
  if (e == hipSuccess && c.npw > 0)
    e = hipMemcpyAsync(c.d.wpl, wp.data(), sizeof(int32_t) * wp.size(), hipMemcpyHostToDevice,
                       c.stream);
  std::vector<int32_t> wpos;
  if (c.madj.wpos) {  // wall-list index of every wall particle (moving-cloud reverse step)
    wpos.assign(c.N, -1);
    for (int k = 0; k < c.Nw; ++k) wpos[wl[k]] = k;
    if (e == hipSuccess)
      e = hipMemcpyAsync(c.madj.wpos, wpos.data(), sizeof(int32_t) * c.N, hipMemcpyHostToDevice,
                         c.stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(c.d.err, zeros, sizeof(zeros), hipMemcpyHostToDevice, c.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  if (e != hipSuccess) {
    delete h;
    return BGK_EDEVICE;
  }
  *out = h;
  return BGK_OK;
}

void bgk_destroy(bgk_ctx* ctx) {
  if (!ctx) return;
  Ctx& c = ctx->c;
  if (!c.timed.empty()) hipStreamSynchronize(c.stream);
  for (auto& p : c.timed) {
    hipEventDestroy(p.first);
    hipEventDestroy(p.second);
  }
  for (hipEvent_t e : c.event_pool) hipEventDestroy(e);
  delete ctx;
}

int bgk_timing_enable(bgk_ctx* ctx, int enable) {
  if (!ctx) return BGK_EINVAL;
  ctx->c.timing = enable != 0;
  return BGK_OK;
}

int bgk_timing_read(bgk_ctx* ctx, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches) return BGK_EINVAL;
  Ctx& c = ctx->c;
  hipError_t e = hipStreamSynchronize(c.stream);
  double sum = 0.0;
  for (auto& p : c.timed) {
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.first, p.second);
    sum += ms;
    c.event_pool.push_back(p.first);
    c.event_pool.push_back(p.second);
  }
  *total_ms = sum;
  *launches = static_cast<int64_t>(c.timed.size());
  c.timed.clear();
  return bgk::hip_fail(&c, e, "bgk_timing_read");
}

int bgk_set_lid_velocity(bgk_ctx* ctx, double lid) {
  if (!ctx || !std::isfinite(lid)) return BGK_EINVAL;
  ctx->c.lid = lid;
  return BGK_OK;
}

int bgk_build_neighbors(bgk_ctx* ctx, const double* x, int32_t* nbr_cnt, int32_t* nbr_idx) {
  if (!ctx || !x || !nbr_cnt || !nbr_idx) return BGK_EINVAL;
  Ctx& c = ctx->c;
  hipError_t e = bgk::launch_cells(c, x);
  if (e == hipSuccess) e = bgk::launch_neighbors(c, x, nbr_cnt, nbr_idx);
  c.geom_valid = false;
  c.pm_valid = false;
  return bgk::hip_fail(&c, e, "bgk_build_neighbors");
}

int bgk_wls_operators(bgk_ctx* ctx, const double* x, const int32_t* nbr_cnt,
                      const int32_t* nbr_idx, double* grad, double* ops, int32_t* degree) {
  if (!ctx || !x || !nbr_cnt || !nbr_idx || !grad || !ops) return BGK_EINVAL;
  Ctx& c = ctx->c;
  const int64_t slots = static_cast<int64_t>(c.N) * c.cap;
  hipError_t e = bgk::launch_cells(c, x);
  if (e == hipSuccess) e = bgk::launch_fill_f64(c.stream, grad, slots * c.D, 0.0);
  if (e == hipSuccess) e = bgk::launch_fill_f64(c.stream, ops, slots * c.DD, 0.0);
  if (e == hipSuccess && degree) e = bgk::launch_fill_i32(c.stream, degree, c.N, 0);
  if (e == hipSuccess) e = bgk::launch_wls(c, x, nbr_cnt, nbr_idx, grad, ops, nullptr, degree);
  c.geom_valid = false;
  c.pm_valid = false;
  return bgk::hip_fail(&c, e, "bgk_wls_operators");
}

int bgk_wall_stencil(bgk_ctx* ctx, const double* x, int32_t* wall_cnt, int32_t* wall_idx,
                     double* wall_c0, double* wall_radius) {
  if (!ctx || !x || !wall_cnt || !wall_idx || !wall_c0) return BGK_EINVAL;
  Ctx& c = ctx->c;
  const int64_t slots = static_cast<int64_t>(c.N) * c.cap;
  hipError_t e = bgk::launch_cells(c, x);
  if (e == hipSuccess) e = bgk::launch_wall_stencil(c, x);
  if (e == hipSuccess) e = bgk::launch_fill_i32(c.stream, wall_cnt, c.N, 0);
  if (e == hipSuccess) e = bgk::launch_fill_i32(c.stream, wall_idx, slots, 0);
  if (e == hipSuccess) e = bgk::launch_fill_f64(c.stream, wall_c0, slots, 0.0);
  if (e == hipSuccess && wall_radius) e = bgk::launch_fill_f64(c.stream, wall_radius, c.N, 0.0);
  if (e == hipSuccess) e = bgk::launch_scatter_wall_rows(c, wall_cnt, wall_idx, wall_c0, wall_radius);
  c.geom_valid = false;
  c.pm_valid = false;
  return bgk::hip_fail(&c, e, "bgk_wall_stencil");
}

int bgk_geometry(bgk_ctx* ctx, const double* x) {
  if (!ctx || !x) return BGK_EINVAL;
  return bgk::build_geometry(ctx->c, x);
}

int bgk_transport(bgk_ctx* ctx, const void* f_in, void* f_tilde, const double* U) {
  if (!ctx || !f_in || !f_tilde || !U || f_in == f_tilde) return BGK_EINVAL;
  Ctx& c = ctx->c;
  if (!c.geom_valid) return bgk::fail(&c, BGK_EINVAL, "bgk_transport before bgk_geometry");
  hipError_t e = bgk::use_fused(c)
                     ? bgk::launch_fused(c, f_in, f_tilde, U, nullptr, nullptr, nullptr, false)
                     : bgk::launch_transport(c, f_in, f_tilde, U);
  if (e == hipSuccess) e = bgk::launch_copy_wall_rows(c, f_in, f_tilde);
  return bgk::hip_fail(&c, e, "bgk_transport");
}

int bgk_collide(bgk_ctx* ctx, const void* f_tilde, void* f_out, double* rho, double* U,
                double* T) {
  if (!ctx || !f_tilde || !f_out || !rho || !U || !T) return BGK_EINVAL;
  Ctx& c = ctx->c;
  if (!c.geom_valid) return bgk::fail(&c, BGK_EINVAL, "bgk_collide before bgk_geometry");
  return bgk::hip_fail(&c, bgk::launch_collide(c, f_tilde, f_out, rho, U, T), "bgk_collide");
}

int bgk_wall_bc(bgk_ctx* ctx, void* f, double* rho, double* U, double* T) {
  if (!ctx || !f || !rho || !U || !T) return BGK_EINVAL;
  Ctx& c = ctx->c;
  if (!c.geom_valid) return bgk::fail(&c, BGK_EINVAL, "bgk_wall_bc before bgk_geometry");
  return bgk::hip_fail(&c, bgk::launch_wall_bc(c, f, rho, U, T), "bgk_wall_bc");
}

int bgk_move(bgk_ctx* ctx, double* x, const double* U) {
  if (!ctx || !x || !U) return BGK_EINVAL;
  Ctx& c = ctx->c;
  if (!c.geom_valid) return bgk::fail(&c, BGK_EINVAL, "bgk_move before bgk_geometry");
  const hipError_t e = bgk::launch_move(c, x, U);
  c.geom_valid = false;
  c.pm_valid = false;
  return bgk::hip_fail(&c, e, "bgk_move");
}

namespace {
// [a, a + na) and [b, b + nb) share a byte (null pointers share none)
bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b) return false;
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

// One full step; f_tilde (nullable) also receives the interior rows of the
// transported field.
int step_impl(Ctx& c, const void* f_in, void* f_out, double* x, double* U, double* rho,
              double* T, void* f_tilde) {
  if (c.cfg.move || !c.geom_valid) {
    const int rc = bgk::build_geometry(c, x);
    if (rc) return rc;
  }
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (c.timing) {
    ev0 = bgk::take_event(c);
    ev1 = bgk::take_event(c);
    if (!ev0 || !ev1) return bgk::fail(&c, BGK_EDEVICE, "event creation");
    hipEventRecord(ev0, c.stream);
  }
  const bool fused = bgk::use_fused(c);
  void* ft = f_tilde ? f_tilde : f_out;  // (the generic path's transport output)
  hipError_t e = fused ? bgk::launch_fused(c, f_in, f_out, U, rho, U, T, true, f_tilde)
                       : bgk::launch_transport(c, f_in, ft, U);
  if (c.timing) {
    hipEventRecord(ev1, c.stream);
    c.timed.emplace_back(ev0, ev1);
  }
  if (e == hipSuccess && !fused) e = bgk::launch_collide(c, ft, f_out, rho, U, T);
  if (e == hipSuccess) e = bgk::launch_wall_bc(c, f_out, rho, U, T);
  if (e == hipSuccess && c.cfg.move) {
    e = bgk::launch_move(c, x, U);
    c.geom_valid = false;
    c.pm_valid = false;
  }
  if (e != hipSuccess) return bgk::hip_fail(&c, e, "bgk_step");
  ++c.steps;
  return BGK_OK;
}
}  // namespace

int bgk_step(bgk_ctx* ctx, const void* f_in, void* f_out, double* x, double* U, double* rho,
             double* T) {
  if (!ctx || !f_in || !f_out || !x || !U || !rho || !T || f_in == f_out) return BGK_EINVAL;
  return step_impl(ctx->c, f_in, f_out, x, U, rho, T, nullptr);
}

int bgk_step_keep(bgk_ctx* ctx, const void* f_in, void* f_out, double* x, double* U, double* rho,
                  double* T, void* f_tilde) {
  if (!ctx || !f_in || !f_out || !x || !U || !rho || !T || !f_tilde || f_in == f_out)
    return BGK_EINVAL;
  Ctx& c = ctx->c;
  const size_t F = (c.cfg.precision == BGK_FP64 ? 8 : 4) * c.NC * static_cast<size_t>(c.N) * c.NV;
  const size_t DN = sizeof(double) * c.D * static_cast<size_t>(c.N), N8 = sizeof(double) * c.N;
  const void* other[] = {f_in, f_out, x, U, rho, T};
  const size_t nother[] = {F, F, DN, DN, N8, N8};
  for (int k = 0; k < 6; ++k)
    if (overlap(f_tilde, F, other[k], nother[k]))
      return bgk::fail(&c, BGK_EINVAL, "bgk_step_keep: f_tilde overlaps another argument");
  return step_impl(c, f_in, f_out, x, U, rho, T, f_tilde);
}

int bgk_pm_plan(bgk_ctx* ctx, const double* x, double merge_radius, double hole_radius,
                int32_t* n_pairs, int32_t* n_holes) {
  if (!ctx || !x || !n_pairs || !n_holes) return BGK_EINVAL;
  Ctx& c = ctx->c;
  if (!(c.cfg.flags & BGK_FLAG_PARTICLES))
    return bgk::fail(&c, BGK_ENOTSUP, "bgk_pm_plan needs a context with BGK_FLAG_PARTICLES");
  if (!(merge_radius > 0.0) || !(hole_radius > 0.0) || !(merge_radius + hole_radius <= c.cfg.h))
    return bgk::fail(&c, BGK_EINVAL, "bgk_pm_plan: radii must be > 0 with merge + hole <= h");
  // the plan rebuilds the cell list of x: the geometry of a frozen cloud is
  // rebuilt by the next step
  c.geom_valid = false;
  c.adj_valid = false;
  c.pm_valid = false;
  hipError_t e = bgk::launch_pm_plan(c, x, merge_radius, hole_radius);
  int32_t tot[3] = {0, 0, 0};
  if (e == hipSuccess)
    e = hipMemcpyAsync(&tot[0], c.pm.keep + c.N, 4, hipMemcpyDeviceToHost, c.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&tot[1], c.pm.mid + c.N, 4, hipMemcpyDeviceToHost, c.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&tot[2], c.pm.hole + c.nodes, 4, hipMemcpyDeviceToHost, c.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  if (e != hipSuccess) return bgk::hip_fail(&c, e, "bgk_pm_plan");
  for (int k = 0; k < 3; ++k) c.pm_tot[k] = tot[k];
  c.pm_valid = true;
  *n_pairs = tot[1];
  *n_holes = tot[2];
  return BGK_OK;
}

int bgk_pm_apply(bgk_ctx* ctx, const double* x, const void* f, const double* rho,
                 const double* U, const double* T, double* x_new, int32_t* wall_id_new,
                 void* f_new, double* rho_new, double* U_new, double* T_new) {
  if (!ctx || !x || !f || !rho || !U || !T || !x_new || !wall_id_new || !f_new || !rho_new ||
      !U_new || !T_new || f == f_new || x == x_new)
    return BGK_EINVAL;
  Ctx& c = ctx->c;
  if (!(c.cfg.flags & BGK_FLAG_PARTICLES))
    return bgk::fail(&c, BGK_ENOTSUP, "bgk_pm_apply needs a context with BGK_FLAG_PARTICLES");
  if (!c.pm_valid) return bgk::fail(&c, BGK_EINVAL, "bgk_pm_apply without a current bgk_pm_plan");
  const int n_keep = c.pm_tot[0], n_new = c.pm_tot[1] + c.pm_tot[2];
  const int Nn = n_keep + n_new;
  return bgk::hip_fail(&c, bgk::launch_pm_apply(c, x, f, rho, U, T, Nn, n_keep, n_new, x_new,
                                                wall_id_new, f_new, rho_new, U_new, T_new),
                       "bgk_pm_apply");
}

int bgk_moments(bgk_ctx* ctx, const void* f, double* rho, double* U, double* T) {
  if (!ctx || !f || !rho || !U || !T) return BGK_EINVAL;
  return bgk::hip_fail(&ctx->c, bgk::launch_moments(ctx->c, f, rho, U, T), "bgk_moments");
}

int bgk_state_check(bgk_ctx* ctx, const void* f, const double* rho, const double* U,
                    const double* T, double* out) {
  if (!ctx || !f || !rho || !U || !T || !out) return BGK_EINVAL;
  Ctx& c = ctx->c;
  double* dev = c.d.scheck + static_cast<size_t>(c.N) * bgk::kCheckTerms;  // the sums
  hipError_t e = bgk::launch_state_check(c, f, rho, U, T, dev);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, dev, bgk::kCheckTerms * sizeof(double), hipMemcpyDeviceToHost, c.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  return bgk::hip_fail(&c, e, "bgk_state_check");
}

int bgk_maxwellian(bgk_ctx* ctx, const double* rho, const double* U, const double* T,
                   void* f_out) {
  if (!ctx || !rho || !U || !T || !f_out) return BGK_EINVAL;
  return bgk::hip_fail(&ctx->c, bgk::launch_maxwellian(ctx->c, rho, U, T, f_out),
                       "bgk_maxwellian");
}

int bgk_objective(bgk_ctx* ctx, const void* f, const double* rho, const double* U,
                  double ke_weight, double* J, void* dJ_df, double* dJ_drho, double* dJ_dU) {
  if (!ctx || !f || !rho || !U || !J || !std::isfinite(ke_weight)) return BGK_EINVAL;
  Ctx& c = ctx->c;
  if (c.cfg.precision == BGK_BF16)
    return bgk::fail(&c, BGK_ENOTSUP, "bgk_objective needs FP64 or FP32");
  return bgk::hip_fail(&c, bgk::launch_objective(c, f, rho, U, ke_weight, J, dJ_df, dJ_drho, dJ_dU,
                                                c.d.jpart),
                       "bgk_objective");
}

int bgk_objective_static(bgk_ctx* ctx, const void* f, const double* rho, const double* U,
                         double ke_weight, double* J, void* dJ_df, double* dJ_drho,
                         double* dJ_dU) {
  if (!ctx || !f || !rho || !U || !J || !std::isfinite(ke_weight)) return BGK_EINVAL;
  Ctx& c = ctx->c;
  if (c.cfg.precision == BGK_BF16)
    return bgk::fail(&c, BGK_ENOTSUP, "bgk_objective_static needs FP64 or FP32");
  if (static_cast<int64_t>(c.N) > BGK_STATIC_SCRATCH_PARTICLES)
    return bgk::fail(&c, BGK_EINVAL,
                     "bgk_objective_static: more particles than its static scratch holds "
                     "(BGK_STATIC_SCRATCH_PARTICLES)");
  double* part = bgk::static_scratch(c.device);
  if (!part)
    return bgk::fail(&c, BGK_EDEVICE, "bgk_objective_static: no static scratch on this device");
  return bgk::hip_fail(&c, bgk::launch_objective(c, f, rho, U, ke_weight, J, dJ_df, dJ_drho, dJ_dU,
                                                part),
                       "bgk_objective_static");
}

int bgk_adjoint_step(bgk_ctx* ctx, const void* f_n, const double* U_n, const double* x,
                     const void* lam_f1, const double* lam_U1, const double* lam_rho1,
                     const double* lam_T1, void* lam_f, double* lam_U, double* dJ_dlid) {
  if (!ctx || !f_n || !U_n || !x || !lam_f1 || !lam_f || !lam_U) return BGK_EINVAL;
  Ctx& c = ctx->c;
  if (!(c.cfg.flags & BGK_FLAG_ADJOINT))
    return bgk::fail(&c, BGK_ENOTSUP, "bgk_adjoint_step needs a context with BGK_FLAG_ADJOINT");
  if (c.cfg.move)
    return bgk::fail(&c, BGK_ENOTSUP,
                     "bgk_adjoint_step is the frozen-cloud reverse step (move = 0); the moving "
                     "cloud's is bgk_adjoint_step_move");
  const size_t F = (c.cfg.precision == BGK_FP64 ? 8 : 4) * c.NC * static_cast<size_t>(c.N) * c.NV;
  const size_t DN = sizeof(double) * c.D * static_cast<size_t>(c.N), N8 = sizeof(double) * c.N;
  // outputs against every input; lam_f == lam_f1 and lam_U == lam_U1 are allowed
  const void* in[] = {f_n, U_n, x, lam_f1, lam_U1, lam_rho1, lam_T1, dJ_dlid};
  const size_t nin[] = {F, DN, DN, F, DN, N8, N8, sizeof(double)};
  for (int k = 0; k < 8; ++k) {
    if (overlap(lam_f, F, in[k], nin[k]) && !(k == 3 && in[k] == lam_f))
      return bgk::fail(&c, BGK_EINVAL, "bgk_adjoint_step: lam_f overlaps an input");
    if (overlap(lam_U, DN, in[k], nin[k]) && !(k == 4 && in[k] == lam_U))
      return bgk::fail(&c, BGK_EINVAL, "bgk_adjoint_step: lam_U overlaps an input");
  }
  if (overlap(lam_f, F, lam_U, DN))
    return bgk::fail(&c, BGK_EINVAL, "bgk_adjoint_step: lam_f overlaps lam_U");
  if (!c.geom_valid) {
    const int rc = bgk::build_geometry(c, x);
    if (rc) return rc;
  }
  hipError_t e = hipSuccess;
  if (!c.adj_valid) {
    e = bgk::launch_adjoint_transposes(c);
    if (e != hipSuccess) return bgk::hip_fail(&c, e, "bgk_adjoint_step transposes");
    c.adj_valid = true;
  }
  // recompute S4-S7 from (f_n, U_n), keeping f-tilde and the new moments
  const bgk::Adj& a = c.adj;
  // the fused kernel relaxes and keeps a copy of f-tilde (the generic path
  // transports, then relaxes)
  if (bgk::use_fused(c)) {
    e = bgk::launch_fused(c, f_n, a.f1, U_n, a.rho1, a.U1, a.T1, true, a.ft);
  } else {
    e = bgk::launch_transport(c, f_n, a.ft, U_n);
    if (e == hipSuccess) e = bgk::launch_collide(c, a.ft, a.f1, a.rho1, a.U1, a.T1);
  }
  if (e == hipSuccess) e = bgk::launch_wall_bc(c, a.f1, a.rho1, a.U1, a.T1);
  if (e == hipSuccess)
    e = bgk::launch_adjoint_step(c, f_n, U_n, lam_f1, lam_U1, lam_rho1, lam_T1, lam_f, lam_U,
                                 dJ_dlid);
  return bgk::hip_fail(&c, e, "bgk_adjoint_step");
}

int bgk_adjoint_step_kept(bgk_ctx* ctx, const void* f_n, const double* U_n, const double* x,
                          const void* f_tilde, const void* f_n1, const double* rho_n1,
                          const double* U_n1, const double* T_n1, const void* lam_f1,
                          const double* lam_U1, const double* lam_rho1, const double* lam_T1,
                          void* lam_f, double* lam_U, double* dJ_dlid) {
  if (!ctx || !f_n || !U_n || !x || !f_tilde || !f_n1 || !rho_n1 || !U_n1 || !T_n1 || !lam_f1 ||
      !lam_f || !lam_U)
    return BGK_EINVAL;
  Ctx& c = ctx->c;
  if (!(c.cfg.flags & BGK_FLAG_ADJOINT))
    return bgk::fail(&c, BGK_ENOTSUP, "bgk_adjoint_step_kept needs a context with BGK_FLAG_ADJOINT");
  if (c.cfg.move)
    return bgk::fail(&c, BGK_ENOTSUP,
                     "bgk_adjoint_step_kept is the frozen-cloud reverse step (move = 0)");
  const size_t F = (c.cfg.precision == BGK_FP64 ? 8 : 4) * c.NC * static_cast<size_t>(c.N) * c.NV;
  const size_t DN = sizeof(double) * c.D * static_cast<size_t>(c.N), N8 = sizeof(double) * c.N;
  // outputs against every input; lam_f == lam_f1 and lam_U == lam_U1 are allowed
  const void* in[] = {f_n, U_n, x, lam_f1, lam_U1, lam_rho1, lam_T1, dJ_dlid,
                      f_tilde, f_n1, rho_n1, U_n1, T_n1};
  const size_t nin[] = {F, DN, DN, F, DN, N8, N8, sizeof(double), F, F, N8, DN, N8};
  for (int k = 0; k < 13; ++k) {
    if (overlap(lam_f, F, in[k], nin[k]) && !(k == 3 && in[k] == lam_f))
      return bgk::fail(&c, BGK_EINVAL, "bgk_adjoint_step_kept: lam_f overlaps an input");
    if (overlap(lam_U, DN, in[k], nin[k]) && !(k == 4 && in[k] == lam_U))
      return bgk::fail(&c, BGK_EINVAL, "bgk_adjoint_step_kept: lam_U overlaps an input");
  }
  if (overlap(lam_f, F, lam_U, DN))
    return bgk::fail(&c, BGK_EINVAL, "bgk_adjoint_step_kept: lam_f overlaps lam_U");
  if (!c.geom_valid) {
    const int rc = bgk::build_geometry(c, x);
    if (rc) return rc;
  }
  hipError_t e = hipSuccess;
  if (!c.adj_valid) {
    e = bgk::launch_adjoint_transposes(c);
    if (e != hipSuccess) return bgk::hip_fail(&c, e, "bgk_adjoint_step_kept transposes");
    c.adj_valid = true;
  }
  const bgk::AdjState st{f_tilde, f_n1, rho_n1, U_n1, T_n1};
  e = bgk::launch_adjoint_step_kept(c, f_n, U_n, st, lam_f1, lam_U1, lam_rho1, lam_T1, lam_f,
                                    lam_U, dJ_dlid);
  return bgk::hip_fail(&c, e, "bgk_adjoint_step_kept");
}

int bgk_adjoint_step_move(bgk_ctx* ctx, const void* f_n, const double* U_n, const double* x_n,
                          const void* lam_f1, const double* lam_U1, const double* lam_x1,
                          const double* lam_rho1, const double* lam_T1, void* lam_f,
                          double* lam_U, double* lam_x, double* dJ_dlid) {
  if (!ctx || !f_n || !U_n || !x_n || !lam_f1 || !lam_f || !lam_U || !lam_x) return BGK_EINVAL;
  Ctx& c = ctx->c;
  if (!(c.cfg.flags & BGK_FLAG_ADJOINT) || !c.cfg.move)
    return bgk::fail(&c, BGK_ENOTSUP,
                     "bgk_adjoint_step_move needs a context with BGK_FLAG_ADJOINT and move = 1");
  const size_t F = (c.cfg.precision == BGK_FP64 ? 8 : 4) * c.NC * static_cast<size_t>(c.N) * c.NV;
  const size_t DN = sizeof(double) * c.D * static_cast<size_t>(c.N), N8 = sizeof(double) * c.N;
  // outputs against every input; lam_f == lam_f1, lam_U == lam_U1 and
  // lam_x == lam_x1 are allowed
  const void* in[] = {f_n, U_n, x_n, lam_f1, lam_U1, lam_x1, lam_rho1, lam_T1, dJ_dlid};
  const size_t nin[] = {F, DN, DN, F, DN, DN, N8, N8, sizeof(double)};
  for (int k = 0; k < 9; ++k) {
    if (overlap(lam_f, F, in[k], nin[k]) && !(k == 3 && in[k] == lam_f))
      return bgk::fail(&c, BGK_EINVAL, "bgk_adjoint_step_move: lam_f overlaps an input");
    if (overlap(lam_U, DN, in[k], nin[k]) && !(k == 4 && in[k] == lam_U))
      return bgk::fail(&c, BGK_EINVAL, "bgk_adjoint_step_move: lam_U overlaps an input");
    if (overlap(lam_x, DN, in[k], nin[k]) && !(k == 5 && in[k] == lam_x))
      return bgk::fail(&c, BGK_EINVAL, "bgk_adjoint_step_move: lam_x overlaps an input");
  }
  if (overlap(lam_f, F, lam_U, DN) || overlap(lam_f, F, lam_x, DN) ||
      overlap(lam_U, DN, lam_x, DN))
    return bgk::fail(&c, BGK_EINVAL, "bgk_adjoint_step_move: the outputs overlap");
  // the geometry of x^n, its transposed stencils, then the step recomputed
  int rc = bgk::build_geometry(c, x_n);
  if (rc) return rc;
  hipError_t e = bgk::launch_adjoint_transposes(c);
  if (e != hipSuccess) return bgk::hip_fail(&c, e, "bgk_adjoint_step_move transposes");
  c.adj_valid = false;
  const bgk::Adj& a = c.adj;
  if (bgk::use_fused(c)) {
    e = bgk::launch_fused(c, f_n, a.f1, U_n, a.rho1, a.U1, a.T1, true, a.ft);
  } else {
    e = bgk::launch_transport(c, f_n, a.ft, U_n);
    if (e == hipSuccess) e = bgk::launch_collide(c, a.ft, a.f1, a.rho1, a.U1, a.T1);
  }
  if (e == hipSuccess) e = bgk::launch_wall_bc(c, a.f1, a.rho1, a.U1, a.T1);
  // S8 reverse, then the frozen-operator reverse with the position update's
  // share of lam_U^{n+1}, then the reverse through the operators and rows
  if (e == hipSuccess) e = bgk::launch_adjoint_move_prep(c, x_n, lam_U1, lam_x1);
  if (e == hipSuccess)
    e = bgk::launch_adjoint_step(c, f_n, U_n, lam_f1, c.madj.lamU_eff, lam_rho1, lam_T1, lam_f,
                                 lam_U, dJ_dlid, true);
  if (e == hipSuccess) e = bgk::launch_adjoint_move_geometry(c, f_n, U_n, x_n, lam_x);
  return bgk::hip_fail(&c, e, "bgk_adjoint_step_move");
}

int bgk_moments_adjoint(bgk_ctx* ctx, const double* rho, const double* U, const double* T,
                        const double* lam_rho, const double* lam_U, const double* lam_T,
                        void* lam_f) {
  if (!ctx || !rho || !U || !T || !lam_f) return BGK_EINVAL;
  Ctx& c = ctx->c;
  if (c.cfg.precision == BGK_BF16)
    return bgk::fail(&c, BGK_ENOTSUP, "bgk_moments_adjoint needs FP64 or FP32");
  return bgk::hip_fail(&c, bgk::launch_moments_adjoint(c, rho, U, T, lam_rho, lam_U, lam_T, lam_f),
                       "bgk_moments_adjoint");
}

int bgk_check(bgk_ctx* ctx) {
  if (!ctx) return BGK_EINVAL;
  Ctx& c = ctx->c;
  int32_t w[bgk::kErrWords];
  hipError_t e = hipStreamSynchronize(c.stream);
  if (e == hipSuccess) e = hipMemcpy(w, c.d.err, sizeof(w), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bgk::hip_fail(&c, e, "bgk_check");
  if (w[0] == 0) return BGK_OK;
  int code = BGK_EDEVICE;
  for (int k = 1; k < 31; ++k)
    if (w[0] & bgk::err_bit(k)) {
      code = k;
      break;
    }
  const int32_t zero = 0;
  e = hipMemcpy(c.d.err, &zero, sizeof(zero), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bgk::hip_fail(&c, e, "bgk_check");
  return bgk::fail(&c, code, "reported by a kernel");
}

int bgk_diagnostics(bgk_ctx* ctx, int64_t* out4) {
  if (!ctx || !out4) return BGK_EINVAL;
  Ctx& c = ctx->c;
  int32_t w[bgk::kErrWords];
  hipError_t e = hipSuccess;
  if (c.geom_valid || c.steps > 0) {
    e = bgk::launch_max_i32(c.stream, c.d.ncnt, c.N, c.d.err + 2);
    if (e == hipSuccess) e = bgk::launch_max_i32(c.stream, c.d.ucount, c.npatch, c.d.err + 3);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  if (e == hipSuccess) e = hipMemcpy(w, c.d.err, sizeof(w), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bgk::hip_fail(&c, e, "bgk_diagnostics");
  out4[0] = w[1];
  out4[1] = c.steps;
  out4[2] = w[2];
  out4[3] = w[3];
  return BGK_OK;
}

const char* bgk_last_error(bgk_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->c.last_error.c_str();
}

}  // extern "C"
