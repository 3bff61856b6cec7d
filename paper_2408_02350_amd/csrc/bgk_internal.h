// Internal declarations of libbgk (HIP, gfx950).  Not part of the public
// interface: the public C ABI is include/bgk.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "bgk.h"

namespace bgk {

// Interior particles per transport patch (the union entries pack one byte
// per patch particle, so at most 4).  Four particles share each row load.
// FP64 in 2D has the registers for 4 particles only at 2 velocities per
// lane (512-lane blocks); it takes them when half the velocity grid fills
// whole waves and the patches fill the chip (at least 1024 of them), and
// otherwise runs 2-particle patches with 4 velocities per lane (256-lane
// blocks), which fill ragged grids and small clouds better.
constexpr int kPatchMax = 4;
// Wall particles per wall patch: consecutive wall-list entries of one face
// whose interpolation rows share most interior particles (3D).
constexpr int kWallPatch = 4;
inline int64_t wall_patches_max(int64_t N, int dim) { return N / kWallPatch + 2 * dim + 1; }
inline int choose_patch(int dim, int precision, int NV, int Ni) {
  if (dim != 2 || precision != BGK_FP64) return 4;
  const int lanes = NV / 2;
  return (lanes % 64 == 0 && lanes <= 512 && (Ni + 3) / 4 >= 1024) ? 4 : 2;
}
constexpr int kThreads = 256;   // threads per block of the per-particle kernels

// bit of the device error word for each status code
__host__ __device__ constexpr int err_bit(int code) { return 1 << code; }

// Device error word layout (int32): [0] error bits, [1] clamped coordinates,
// [2] largest neighbour count, [3] largest patch union (these two are filled
// on demand by bgk_diagnostics from the current geometry).
constexpr int kErrWords = 8;

// Device views of the workspace for one context.
struct Dev {
  int32_t* err;          // [kErrWords]
  int32_t* wall_id;      // [N]
  int32_t* wall_list;    // [Nw]  wall particles by owner wall, then ascending
  int32_t* key;          // [N]   cell key of each particle
  int32_t* cstart;       // [2*ncell + 1] start of each (cell, interior|wall) range
  int32_t* ccursor;      // [2*ncell]
  int32_t* cperm;        // [N]   particles sorted by key; first Ni are interior
  int32_t* cperm2;       // [N]   the same, unordered inside each key (scatter output)
  double* xs;            // [d][N] positions in cperm order
  int32_t* ncnt;         // [N]
  int32_t* nidx;         // [N][cap]
  double* ops64;         // [N][cap][d*d]
  float* ops32;          // [N][cap][d*d] (precision != FP64)
  int32_t* wcnt;         // [Nw]
  int32_t* widx;         // [Nw][cap]
  double* wc0;           // [Nw][cap]
  double* whb;           // [Nw]
  int32_t* ucount;       // [npatch]
  int32_t* uj;           // [npatch][ucap]
  uint32_t* ue;          // [npatch][ucap] packed 8-bit slot of each patch particle
  int32_t* wpl;          // [npw][kWallPatch] wall-list slots of each wall patch (-1: empty)
  int32_t* wucount;      // [npw]
  int32_t* wuj;          // [npw][kWallPatch*cap] union of the patch's wall rows
  uint32_t* wue;         // [npw][kWallPatch*cap] packed 8-bit slot in each wall row
  double* jpart;         // [N]   per-particle terms of the objective
  double* scheck;        // [N][kCheckTerms] per-particle terms of bgk_state_check, then its sums
};

// Workspace of the reverse step (BGK_FLAG_ADJOINT; FP64, frozen cloud).
struct Adj {
  int32_t* tidx;      // [N][cap]  slot of j in the row of nidx[j][e] (-1: not transported)
  int32_t* wtstart;   // [N+1]     start of particle j's wall-stencil uses
  int32_t* wtcursor;  // [N]
  int32_t* wt;        // [Nw*cap]  uses of j as (wall list index << 8 | slot), sorted
  void* ft;           // [n_c][N][N_v] recomputed f-tilde (f storage type)
  void* f1;           // [n_c][N][N_v] recomputed f^{n+1}; storage shared with lam_ft
  void* lam_ft;       // [n_c][N][N_v] adjoint of f-tilde (interior rows)
  double* rho1;       // [N]
  double* U1;         // [d][N]
  double* T1;         // [N]
  void* larr;         // [Nw][n_c][N_v] adjoint reaching the interpolated wall values
  double* lidpart;    // [max(Nw,1)]
  double* gpart;      // [tiles][d][N] per-tile parts of lam_U (reverse transport)
  int32_t* ucount;    // [(N+1)/2]   unions of the reverse transport's 2-particle patches
  int32_t* uj;        // [(N+1)/2][2*cap]
  uint32_t* ue;       // [(N+1)/2][2*cap]
};

// Workspace of the reverse step with the moving cloud (BGK_FLAG_ADJOINT with
// move = 1): the adjoint through the positions.
struct MoveAdj {
  int32_t* wpos;      // [N]        wall-list index of each wall particle (-1: interior)
  double* lamU_eff;   // [d][N]     adjoint of U^{n+1} with the position update's share
  double* xpass;      // [d][N]     adjoint of x^{n+1} passed to x^n by the position update
  double* lam_a;      // [N][cap][d*d] adjoint of the upwind vectors of every edge
  double* lc0;        // [N][cap]   adjoint of the wall value rows (wall-list order)
  double* xc;         // [N][cap][d] contribution of row i's slot e to the adjoint of x_j
  double* xs;         // [N][d]      contribution of row i to the adjoint of x_i
  double* wxc;        // [N][cap][d] the same for the wall rows
  double* wxs;        // [N][d]
};

// Workspace of the particle management (BGK_FLAG_PARTICLES).
struct Pm {
  int32_t* nn;        // [N]         nearest interior neighbour within h (-1: none)
  int32_t* partner;   // [N]         other particle of a merged pair (-1: none)
  int32_t* keep;      // [N+1]       exclusive scan of the kept particles
  int32_t* mid;       // [N+1]       exclusive scan of the lower pair members
  int32_t* hole;      // [nodes+1]   exclusive scan of the hole nodes
};

// Quadrature weight of every velocity node, (2 vmax/(nv-1))^d.
inline double omega_of(const bgk_config& cfg) {
  const double dv = 2.0 * cfg.vmax / static_cast<double>(cfg.nv - 1);
  double w = 1.0;
  for (int a = 0; a < cfg.dim; ++a) w = w * dv;
  return w;
}

// Lattice nodes per axis of the initial cloud (spacing dx on [0, 1]).
inline int lattice_nodes(const bgk_config& cfg) {
  return static_cast<int>(std::lround(1.0 / cfg.dx)) + 1;
}

struct Ctx {
  bgk_config cfg;
  hipStream_t stream = nullptr;
  int device = 0;
  int N = 0, D = 0, NC = 0, NV = 0, cap = 0, DD = 0;
  int Ni = 0, Nw = 0, npatch = 0, ucap = 0, tp = 4;  // tp: particles per patch
  int npw = 0, wucap = 0;   // wall patches (0: the wall condition runs per wall particle)
  int nca = 0, ncell = 0;
  double lid = 0.0;
  Dev d{};
  Adj adj{};
  MoveAdj madj{};
  Pm pm{};
  int nl = 0;               // lattice nodes per axis (particle management)
  int64_t nodes = 0;        // nl^d
  bool pm_valid = false;    // a particle-management plan of the current cloud is held
  int32_t pm_tot[3] = {0, 0, 0};  // kept, midpoints, holes of that plan
  bool adj_valid = false;   // transposed stencils match the current geometry
  bool geom_valid = false;  // geometry of the current (frozen) cloud is built
  int64_t steps = 0;
  std::string last_error;
  bool timing = false;                                 // event pairs around S4
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timed;
  std::vector<hipEvent_t> event_pool;
};

// Per-device address of the static scratch of bgk_objective_static
// (looked up by bgk_init with the device current; null before).
hipError_t static_scratch_setup(int device);
double* static_scratch(int device);

// Workspace layout: returns total bytes; fills d when base != nullptr.
size_t workspace_layout(const bgk_config& cfg, char* base, Dev* d, Adj* adj, Pm* pm,
                        MoveAdj* madj = nullptr);

// ---- launchers (enqueue on c.stream; return hipError_t of the launch) ----
hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v);
hipError_t launch_fill_f64(hipStream_t s, double* p, int64_t n, double v);
hipError_t launch_copy_i32(hipStream_t s, const int32_t* src, int32_t* dst, int64_t n);
hipError_t launch_max_i32(hipStream_t s, const int32_t* a, int n, int32_t* out);
hipError_t launch_scan(hipStream_t s, int32_t* a, int n);  // exclusive, a[n] = total
hipError_t launch_scatter_wall_rows(const Ctx& c, int32_t* cnt_out, int32_t* idx_out,
                                    double* c0_out, double* hb_out);

hipError_t launch_cells(const Ctx& c, const double* x);              // key, cstart, cperm
hipError_t launch_neighbors(const Ctx& c, const double* x, int32_t* cnt, int32_t* idx);
hipError_t launch_wls(const Ctx& c, const double* x, const int32_t* cnt, const int32_t* idx,
                      double* grad, double* ops, float* ops32, int32_t* degree);
hipError_t launch_wall_stencil(const Ctx& c, const double* x);
hipError_t launch_patches(const Ctx& c);
hipError_t launch_wall_unions(const Ctx& c);
// sorted unions of the rows of patches of P entries of plist (n entries,
// -1 = empty); one wavefront per patch
hipError_t launch_unions(const Ctx& c, int P, int n, const int32_t* plist, const int32_t* cnt,
                         const int32_t* idx, int drop_self, int ucap, int32_t* ucount,
                         int32_t* uj, uint32_t* ue);

hipError_t launch_transport(const Ctx& c, const void* f_in, void* f_out, const double* U);
hipError_t launch_copy_wall_rows(const Ctx& c, const void* f_in, void* f_out);
// Fused S4-S6 (or S4 alone with fuse = false) over patches x all velocities.
// With fuse and f_tilde non-null, f-tilde's interior rows are also stored
// there (the reverse step's recompute).
bool fused_supported(const Ctx& c);
bool use_fused(const Ctx& c);
hipError_t launch_fused(const Ctx& c, const void* f_in, void* f_out, const double* U_in,
                        double* rho, double* U_out, double* T, bool fuse,
                        void* f_tilde = nullptr);
hipError_t launch_collide(const Ctx& c, const void* ft, void* fout, double* rho, double* U,
                          double* T);
hipError_t launch_wall_bc(const Ctx& c, void* f, double* rho, double* U, double* T);
hipError_t launch_move(const Ctx& c, double* x, const double* U);
hipError_t launch_moments(const Ctx& c, const void* f, double* rho, double* U, double* T);
constexpr int kCheckTerms = 12;  // per-particle slots of the state check (and its outputs)
hipError_t launch_state_check(const Ctx& c, const void* f, const double* rho, const double* U,
                              const double* T, double* out_dev);
hipError_t launch_maxwellian(const Ctx& c, const double* rho, const double* U, const double* T,
                             void* f);

// Reverse mode (FP64, frozen cloud).
hipError_t launch_pm_plan(Ctx& c, const double* x, double rm, double rh);
hipError_t launch_pm_apply(const Ctx& c, const double* x, const void* f, const double* rho,
                           const double* U, const double* T, int Nn, int n_keep, int n_new,
                           double* x_new, int32_t* wall_id_new, void* f_new, double* rho_new,
                           double* U_new, double* T_new);
hipError_t launch_adjoint_transposes(const Ctx& c);
// f-sized arguments (f_n, lam_f1, lam_f, dJ_df) are in the f storage type.
// wall_rows: also the adjoint of the wall value rows (moving cloud), taken
// between the wall and the relaxation kernels (f^{n+1}'s interior rows
// share storage with the adjoint of f-tilde)
hipError_t launch_adjoint_step(const Ctx& c, const void* f_n, const double* U_n,
                               const void* lam_f1, const double* lam_U1, const double* lam_rho1,
                               const double* lam_T1, void* lam_f, double* lam_U,
                               double* dJ_dlid, bool wall_rows = false);
// Reverse through the positions (k_adjoint_move.hip): the position update's
// share (before launch_adjoint_step), the wall-row adjoints (inside it),
// then the operators, frames and wall rows (after it).
hipError_t launch_adjoint_move_prep(const Ctx& c, const double* x, const double* lam_U1,
                                    const double* lam_x1);
hipError_t launch_adjoint_wallrow(const Ctx& c);
hipError_t launch_adjoint_move_geometry(const Ctx& c, const void* f_n, const double* U_n,
                                        const double* x, double* lam_x);
// part: N doubles of device scratch for the per-particle terms (the
// context's workspace, or the static scratch of bgk_objective_static)
hipError_t launch_objective(const Ctx& c, const void* f, const double* rho, const double* U,
                            double ke, double* J, void* dJ_df, double* dJ_drho, double* dJ_dU,
                            double* part);
hipError_t launch_moments_adjoint(const Ctx& c, const double* rho, const double* U,
                                  const double* T, const double* lr, const double* lU,
                                  const double* lT, void* lam_f);

}  // namespace bgk

struct bgk_ctx {
  bgk::Ctx c;
};
