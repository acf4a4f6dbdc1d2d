// crkdg_api.hip -- host side of the cRKDG library: the C ABI declared in
// include/crkdg.h.  Argument checking, tableau handling, buffer layout and
// the launch sequence of one step (Section 2.2, equation (crkdg)).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "crkdg_internal.hpp"
#include "dg_core.hpp"

using namespace crk;

struct crkdg_state {
  crkdg_mesh mesh;
  int k, flux, eq, nc, nb;
  Geo geo;
  PhysDev ph;
  BCDev bc;
  // tableau (Section 2.1, equation (butcher))
  int s;
  double A[MAXS][MAXS], b[MAXS], c[MAXS];
  int ws;        // stages the workspace layout holds (>= s; fixed once bound)
  bool subdiag;  // a_ij = 0 unless j == i - 1: inner stages need one accumulator
  // bound memory
  bool bound;
  // time-dependent boundary data with dt in device memory: the step's time
  // lives on the device (t_dev_ptr) and st->t is stale while this is set
  bool t_dev_valid;
  char* dofs;
  char* work;
  hipStream_t stream;
  int cur;  // 0: the current state is in dofs, 1: in the work buffer's first slot
  double t;
  size_t S;       // bytes of one state (device layout lay)
  size_t S_stage; // bytes of one stored stage state (layout lay_stage)
  int lay, lay_stage;
  int prec;  // Prec: P64, PBULK, PINNER or PINC
  int sched; // CRKDG_SCHED_SPLIT or CRKDG_SCHED_FUSED (when the step allows it)
  // per-launch timing (measurement only)
  bool prof;
  int prof_max;
  std::vector<hipEvent_t> ev;   // 2 per launch
  std::vector<int> ev_cls;
  int prof_n;
};

namespace {

constexpr size_t ALIGN = 256;
constexpr size_t SCRATCH = (size_t)RED_BLOCKS * 3 * sizeof(double) + 1024;

size_t round_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

size_t slot_bytes(const crkdg_state* st) {
  return round_up(st->S > st->S_stage ? st->S : st->S_stage);
}
char* slot_ptr(const crkdg_state* st, int slot) {
  // work layout: [state B][stage 1..ws-1][L 0..ws-2][scratch]
  return st->work + (size_t)slot * slot_bytes(st);
}
char* cur_ptr(const crkdg_state* st) { return st->cur ? slot_ptr(st, 0) : st->dofs; }
char* nxt_ptr(const crkdg_state* st) { return st->cur ? st->dofs : slot_ptr(st, 0); }
char* stage_ptr(const crkdg_state* st, int i) { return slot_ptr(st, i); }         // i = 1..ws-1
char* lbuf_ptr(const crkdg_state* st, int j) { return slot_ptr(st, st->ws + j); } // j = 0..ws-2
char* scratch_ptr(const crkdg_state* st) { return slot_ptr(st, 2 * st->ws - 1); }
// per-block wave-speed maxima written by the limiter (one double per 256 cells)
int wave_blocks(const crkdg_state* st) { return (int)((st->geo.N + 255) / 256); }
size_t wave_partial_bytes(const crkdg_state* st) {
  return round_up((size_t)wave_blocks(st) * sizeof(double));
}
// the device copy of the time (one double in the scratch area's free tail)
double* t_dev_ptr(const crkdg_state* st) { return (double*)(scratch_ptr(st) + SCRATCH - 128); }
double* wave_partial_ptr(const crkdg_state* st) {
  return (double*)(scratch_ptr(st) + round_up(SCRATCH));
}

void set_tableau_internal(crkdg_state* st, int s, const double* c, const double* A,
                          const double* b) {
  st->s = s;
  if (s > st->ws) st->ws = s;
  memset(st->A, 0, sizeof st->A);
  for (int i = 0; i < s; ++i) {
    st->b[i] = b[i];
    st->c[i] = c[i];
    for (int j = 0; j < s; ++j) st->A[i][j] = A[i * s + j];
  }
  bool sub = true;
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < i - 1; ++j)
      if (st->A[i][j] != 0.0) sub = false;
  st->subdiag = sub;
}

int hip_rc(hipError_t e) { return e == hipSuccess ? CRKDG_OK : CRKDG_EHIP; }

enum { KC_INNER = 0, KC_FINAL = 1, KC_LOC = 2, KC_COMBINE = 3, KC_DT = 4, KC_LIMIT = 5, KC_OTHER = 6,
       KC_FUSED = 7 };

// event pair around one launch when profiling is on
struct ProfScope {
  crkdg_state* st;
  int idx;
  ProfScope(crkdg_state* s, int cls) : st(s), idx(-1) {
    if (st->prof && st->prof_n < st->prof_max) {
      idx = st->prof_n++;
      st->ev_cls[idx] = cls;
      (void)hipEventRecord(st->ev[2 * idx], st->stream);
    }
  }
  ~ProfScope() {
    if (idx >= 0) (void)hipEventRecord(st->ev[2 * idx + 1], st->stream);
  }
};

}  // namespace

extern "C" {

const char* crkdg_strerror(int code) {
  switch (code) {
    case CRKDG_OK: return "ok";
    case CRKDG_EINVAL: return "invalid argument";
    case CRKDG_EUNSUPPORTED: return "unsupported configuration";
    case CRKDG_ENONPHYSICAL: return "non-physical cell average (rho <= 0, p <= 0 or NaN)";
    case CRKDG_EHIP: return "HIP runtime or kernel launch failure";
    case CRKDG_EUNBOUND: return "state has no device memory bound";
    default: return "unknown error";
  }
}

int crkdg_gauss_rule(int n, double* x, double* w) {
  if (n < 1 || n > 8 || !x || !w) return CRKDG_EINVAL;
  for (int a = 0; a < n; ++a) {
    x[a] = crk::gl_x(n, a);
    w[a] = crk::gl_w(n, a);
  }
  return CRKDG_OK;
}

// Double Mach reflection data (CRKDG_IC_DMR): the Mach 10 shock into gas at
// rest (rho, p) = (1.4, 1) through (1/6, 0) at 60 degrees.  Post-shock state
// from the normal-shock relations: pressure ratio (2 gamma M^2 - (gamma - 1))
// / (gamma + 1), density ratio from the Rankine--Hugoniot (Hugoniot curve)
// relation between the two, gas speed behind the shock S (1 - rho1 / rho2)
// along the shock normal.  Layout as in DMR_NPARAM (crkdg_internal.hpp).
static void dmr_params(double gamma, double* P) {
  const double rho1 = 1.4, p1 = 1.0, mach = 10.0;
  const double S = mach * sqrt(gamma * p1 / rho1);
  const double pr = (2.0 * gamma * mach * mach - (gamma - 1.0)) / (gamma + 1.0);
  const double dr = ((gamma + 1.0) * pr + (gamma - 1.0)) / ((gamma - 1.0) * pr + (gamma + 1.0));
  const double rho2 = rho1 * dr, p2 = p1 * pr;
  const double w = S * (1.0 - 1.0 / dr);
  const double nx = 0.5 * sqrt(3.0), ny = -0.5;  // normal at 60 degrees, into the gas at rest
  const double u2 = w * nx, v2 = w * ny;
  for (int e = 0; e < NPARAM; ++e) P[e] = 0.0;
  P[0] = 1.0 / 6.0;
  P[1] = nx;
  P[2] = ny;
  P[3] = S;
  P[4] = rho2;
  P[5] = rho2 * u2;
  P[6] = rho2 * v2;
  P[7] = p2 / (gamma - 1.0) + 0.5 * rho2 * (u2 * u2 + v2 * v2);
  P[8] = rho1;
  P[9] = 0.0;
  P[10] = 0.0;
  P[11] = p1 / (gamma - 1.0);
}

int crkdg_create(const crkdg_mesh* mesh, int k, int flux, int rk_stages, crkdg_state** out) {
  if (!mesh || !out) return CRKDG_EINVAL;
  if (k < 0 || k > 4) return CRKDG_EINVAL;
  if (mesh->dim != 1 && mesh->dim != 2) return CRKDG_EINVAL;
  if (mesh->nx < 1 || mesh->ny < 1 || (mesh->dim == 1 && mesh->ny != 1)) return CRKDG_EINVAL;
  // device addressing uses 32-bit byte offsets within each component slab of
  // a state (and within the block of FP64 cell averages): cap the mesh so
  // that 8 bytes x max(modes, components) x cells stays below 4 GiB
  {
    const long long ncell = (long long)mesh->nx * mesh->ny;
    const long long nbm = mesh->dim == 2 ? (long long)(k + 1) * (k + 1) : (long long)(k + 1);
    const long long span = nbm > 4 ? nbm : 4;
    if (ncell * span * 8 >= (1LL << 32)) return CRKDG_EINVAL;
  }
  if (!(mesh->x1 > mesh->x0) || (mesh->dim == 2 && !(mesh->y1 > mesh->y0))) return CRKDG_EINVAL;
  if (rk_stages < 1 || rk_stages > 5) return CRKDG_EINVAL;
  if (flux != CRKDG_FLUX_UPWIND && flux != CRKDG_FLUX_LLF && flux != CRKDG_FLUX_GODUNOV)
    return CRKDG_EINVAL;
  if (mesh->precision != CRKDG_FP64 && mesh->precision != CRKDG_FP32_MIXED &&
      mesh->precision != CRKDG_FP32_INNER && mesh->precision != CRKDG_FP32_INCREMENTS)
    return CRKDG_EINVAL;
  for (int sd = 0; sd < 4; ++sd)
    if (mesh->bc[sd] < CRKDG_BC_PERIODIC || mesh->bc[sd] > CRKDG_BC_DIRICHLET) return CRKDG_EINVAL;
  int eq;
  if (mesh->equation == CRKDG_EQ_ADVECTION) {
    if (flux == CRKDG_FLUX_GODUNOV) return CRKDG_EUNSUPPORTED;
    eq = mesh->dim == 1 ? EQ_ADV1 : EQ_ADV2;
  } else if (mesh->equation == CRKDG_EQ_EULER) {
    if (mesh->dim != 2) return CRKDG_EUNSUPPORTED;
    if (flux != CRKDG_FLUX_LLF) return CRKDG_EUNSUPPORTED;
    if (!(mesh->gamma > 1.0)) return CRKDG_EINVAL;
    if (k > 3) return CRKDG_EUNSUPPORTED;  // k = 4 is built for the scalar equations
    eq = EQ_EULER2;
  } else if (mesh->equation == CRKDG_EQ_BURGERS) {
    if (mesh->dim != 1 || flux != CRKDG_FLUX_GODUNOV) return CRKDG_EUNSUPPORTED;
    eq = EQ_BURGERS1;
  } else {
    return CRKDG_EINVAL;
  }
  if (mesh->bc_exact != 0 && mesh->bc_exact != CRKDG_IC_ADV_SIN && mesh->bc_exact != CRKDG_IC_DMR)
    return CRKDG_EUNSUPPORTED;
  if (mesh->bc_exact == CRKDG_IC_ADV_SIN && eq != EQ_ADV1 && eq != EQ_ADV2)
    return CRKDG_EUNSUPPORTED;
  if (mesh->bc_exact == CRKDG_IC_DMR &&
      (eq != EQ_EULER2 || mesh->bc[0] != CRKDG_BC_DIRICHLET ||
       mesh->bc[1] != CRKDG_BC_TRANSMISSIVE || mesh->bc[2] != CRKDG_BC_DIRICHLET ||
       mesh->bc[3] != CRKDG_BC_DIRICHLET))
    return CRKDG_EUNSUPPORTED;
  // the FP32 forms are built for 2D Euler, k = 1..3
  if (mesh->precision != CRKDG_FP64 && (eq != EQ_EULER2 || k < 1)) return CRKDG_EUNSUPPORTED;
  crkdg_state* st = new (std::nothrow) crkdg_state();
  if (!st) return CRKDG_EINVAL;
  st->mesh = *mesh;
  st->k = k;
  st->flux = flux;
  st->eq = eq;
  st->nc = mesh->equation == CRKDG_EQ_EULER ? 4 : 1;
  st->nb = mesh->dim == 2 ? (k + 1) * (k + 1) : k + 1;
  Geo& g = st->geo;
  g.nx = mesh->nx;
  g.ny = mesh->dim == 2 ? mesh->ny : 1;
  g.N = (long long)g.nx * g.ny;
  g.x0 = mesh->x0;
  g.y0 = mesh->dim == 2 ? mesh->y0 : 0.0;
  g.dx = (mesh->x1 - mesh->x0) / mesh->nx;
  g.dy = mesh->dim == 2 ? (mesh->y1 - mesh->y0) / mesh->ny : 1.0;
  g.inv_dx = 1.0 / g.dx;
  g.inv_dy = 1.0 / g.dy;
  st->ph.gamma = mesh->gamma;
  st->ph.ax = mesh->adv[0];
  st->ph.ay = mesh->adv[1];
  st->ph.upwind = flux == CRKDG_FLUX_UPWIND;
  for (int sd = 0; sd < 4; ++sd) {
    st->bc.type[sd] = mesh->bc[sd];
    for (int cc = 0; cc < 4; ++cc) st->bc.state[sd][cc] = mesh->bc_state[sd][cc];
  }
  if (mesh->dim == 1) st->bc.type[2] = st->bc.type[3] = CRKDG_BC_PERIODIC;
  st->bc.exact = mesh->bc_exact;
  memset(st->bc.params, 0, sizeof st->bc.params);
  st->bc.t = 0.0;
  if (mesh->bc_exact == CRKDG_IC_DMR) dmr_params(mesh->gamma, st->bc.params);
  // tableaus named by the paper: forward Euler, (eq:2), (eq:3), classical RK4,
  // and Fehlberg's six-stage method advanced with its fifth-order weights
  // (E. Fehlberg, NASA TR R-315, 1969)
  static const double FE_A[1] = {0}, FE_b[1] = {1}, FE_c[1] = {0};
  static const double E2_A[4] = {0, 0, 0.5, 0}, E2_b[2] = {0, 1}, E2_c[2] = {0, 0.5};
  static const double E3_A[9] = {0, 0, 0, 1.0 / 3.0, 0, 0, 0, 2.0 / 3.0, 0},
                      E3_b[3] = {0.25, 0, 0.75}, E3_c[3] = {0, 1.0 / 3.0, 2.0 / 3.0};
  static const double R4_A[16] = {0, 0, 0, 0, 0.5, 0, 0, 0, 0, 0.5, 0, 0, 0, 0, 1, 0},
                      R4_b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0},
                      R4_c[4] = {0, 0.5, 0.5, 1};
  static const double F5_A[36] = {
      0, 0, 0, 0, 0, 0,
      1.0 / 4, 0, 0, 0, 0, 0,
      3.0 / 32, 9.0 / 32, 0, 0, 0, 0,
      1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197, 0, 0, 0,
      439.0 / 216, -8.0, 3680.0 / 513, -845.0 / 4104, 0, 0,
      -8.0 / 27, 2.0, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40, 0};
  static const double F5_b[6] = {16.0 / 135, 0, 6656.0 / 12825, 28561.0 / 56430, -9.0 / 50,
                                 2.0 / 55},
                      F5_c[6] = {0, 1.0 / 4, 3.0 / 8, 12.0 / 13, 1, 1.0 / 2};
  st->ws = 4;
  switch (rk_stages) {
    case 1: set_tableau_internal(st, 1, FE_c, FE_A, FE_b); break;
    case 2: set_tableau_internal(st, 2, E2_c, E2_A, E2_b); break;
    case 3: set_tableau_internal(st, 3, E3_c, E3_A, E3_b); break;
    case 4: set_tableau_internal(st, 4, R4_c, R4_A, R4_b); break;
    default: set_tableau_internal(st, 6, F5_c, F5_A, F5_b); break;
  }
  st->prec = mesh->precision == CRKDG_FP32_MIXED        ? PBULK
             : mesh->precision == CRKDG_FP32_INNER      ? PINNER
             : mesh->precision == CRKDG_FP32_INCREMENTS ? PINC
                                                        : P64;
  // stored stages use the state's layout
  if (st->prec == PBULK) {
    st->lay = LMIX;
    st->S = (size_t)st->nc * g.N * sizeof(double) + (size_t)st->nc * (st->nb - 1) * g.N * sizeof(float);
  } else {
    st->lay = L64;
    st->S = (size_t)st->nc * st->nb * g.N * sizeof(double);
  }
  st->lay_stage = st->lay;
  st->S_stage = st->S;
  st->sched = CRKDG_SCHED_FUSED;  // taken wherever the one-pass step applies
  st->bound = false;
  st->cur = 0;
  st->t = 0.0;
  *out = st;
  return CRKDG_OK;
}

int crkdg_set_tableau(crkdg_state* st, int s, const double* c, const double* A, const double* b) {
  if (!st || !c || !A || !b || s < 1 || s > MAXS) return CRKDG_EINVAL;
  if (st->bound && s > st->ws) return CRKDG_EINVAL;  // the bound workspace holds ws stages
  for (int i = 0; i < s; ++i) {
    if (!isfinite(b[i]) || !isfinite(c[i])) return CRKDG_EINVAL;
    for (int j = 0; j < s; ++j) {
      const double a = A[i * s + j];
      if (!isfinite(a)) return CRKDG_EINVAL;
      if (j >= i && a != 0.0) return CRKDG_EINVAL;  // explicit: strictly lower triangular
    }
  }
  set_tableau_internal(st, s, c, A, b);
  return CRKDG_OK;
}

size_t crkdg_state_bytes(const crkdg_state* st) { return st ? st->S : 0; }

size_t crkdg_workspace_bytes(const crkdg_state* st) {
  if (!st) return 0;
  return (size_t)(2 * st->ws - 1) * slot_bytes(st) + round_up(SCRATCH) + wave_partial_bytes(st);
}

int crkdg_bind(crkdg_state* st, void* dofs_dev, void* work_dev, void* stream) {
  if (!st || !dofs_dev || !work_dev) return CRKDG_EINVAL;
  if (((uintptr_t)dofs_dev % ALIGN) || ((uintptr_t)work_dev % ALIGN)) return CRKDG_EINVAL;
  st->dofs = (char*)dofs_dev;
  st->work = (char*)work_dev;
  st->stream = (hipStream_t)stream;
  st->bound = true;
  st->cur = 0;
  st->t_dev_valid = false;
  return CRKDG_OK;
}

void* crkdg_current_dofs(const crkdg_state* st) {
  if (!st || !st->bound) return nullptr;
  return cur_ptr(st);
}

// host conversion between the canonical FP64 layout and the device layout
static void to_device_layout(const crkdg_state* st, const double* in, char* out) {
  const long long N = st->geo.N;
  const int nc = st->nc, nb = st->nb;
  double* avg = (double*)out;
  float* hi = (float*)(out + (size_t)nc * N * sizeof(double));
  for (int c = 0; c < nc; ++c) {
    for (long long e = 0; e < N; ++e) avg[c * N + e] = in[(long long)(c * nb) * N + e];
    for (int b = 1; b < nb; ++b)
      for (long long e = 0; e < N; ++e)
        hi[(long long)(c * (nb - 1) + b - 1) * N + e] = (float)in[(long long)(c * nb + b) * N + e];
  }
}
static void from_device_layout(const crkdg_state* st, const char* in, double* out) {
  const long long N = st->geo.N;
  const int nc = st->nc, nb = st->nb;
  const double* avg = (const double*)in;
  const float* hi = (const float*)(in + (size_t)nc * N * sizeof(double));
  for (int c = 0; c < nc; ++c) {
    for (long long e = 0; e < N; ++e) out[(long long)(c * nb) * N + e] = avg[c * N + e];
    for (int b = 1; b < nb; ++b)
      for (long long e = 0; e < N; ++e)
        out[(long long)(c * nb + b) * N + e] = (double)hi[(long long)(c * (nb - 1) + b - 1) * N + e];
  }
}

int crkdg_set_state(crkdg_state* st, const double* host) {
  if (!st || !host) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  hipError_t e;
  if (st->lay != LMIX) {
    e = hipMemcpyAsync(cur_ptr(st), host, st->S, hipMemcpyHostToDevice, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  } else {
    char* tmp = (char*)malloc(st->S);
    if (!tmp) return CRKDG_EINVAL;
    to_device_layout(st, host, tmp);
    e = hipMemcpyAsync(cur_ptr(st), tmp, st->S, hipMemcpyHostToDevice, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
    free(tmp);
  }
  return hip_rc(e);
}

int crkdg_get_state(const crkdg_state* st, double* host) {
  if (!st || !host) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  hipError_t e;
  if (st->lay != LMIX) {
    e = hipMemcpyAsync(host, cur_ptr(st), st->S, hipMemcpyDeviceToHost, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  } else {
    char* tmp = (char*)malloc(st->S);
    if (!tmp) return CRKDG_EINVAL;
    e = hipMemcpyAsync(tmp, cur_ptr(st), st->S, hipMemcpyDeviceToHost, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
    if (e == hipSuccess) from_device_layout(st, tmp, host);
    free(tmp);
  }
  return hip_rc(e);
}

int crkdg_set_time(crkdg_state* st, double t) {
  if (!st || !isfinite(t)) return CRKDG_EINVAL;
  st->t = t;
  st->t_dev_valid = false;
  return CRKDG_OK;
}

// bring the host time up to date with the device copy (syncs the stream)
static int sync_time(crkdg_state* st) {
  if (!st->t_dev_valid) return CRKDG_OK;
  double t = 0.0;
  hipError_t e = hipMemcpyAsync(&t, t_dev_ptr(st), sizeof t, hipMemcpyDeviceToHost, st->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  if (e != hipSuccess) return CRKDG_EHIP;
  st->t = t;
  st->t_dev_valid = false;
  return CRKDG_OK;
}

double crkdg_get_time(const crkdg_state* st) {
  if (!st) return NAN;
  crkdg_state* w = const_cast<crkdg_state*>(st);
  return sync_time(w) == CRKDG_OK ? w->t : NAN;
}

static int copy_params(crkdg_state* st, const double* params, int nparams, double* dst) {
  memset(dst, 0, sizeof(double) * NPARAM);
  if (nparams < 0 || nparams > NPARAM || (nparams > 0 && !params)) return CRKDG_EINVAL;
  for (int e = 0; e < nparams; ++e) dst[e] = params[e];
  (void)st;
  return CRKDG_OK;
}

// small parameter blocks travel through the scratch area (stream-ordered)
static int upload_params(crkdg_state* st, const double* P, double** dev) {
  double* d = (double*)(scratch_ptr(st) + (size_t)RED_BLOCKS * 3 * sizeof(double));
  hipError_t e = hipMemcpyAsync(d, P, sizeof(double) * NPARAM, hipMemcpyHostToDevice, st->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);  // P lives on the host stack
  *dev = d;
  return hip_rc(e);
}

int crkdg_project(crkdg_state* st, int ic, const double* params, int nparams,
                  const double* aux_dev) {
  if (!st) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  if (ic < CRKDG_IC_CONST || ic > CRKDG_IC_BURGERS_SIN) return CRKDG_EINVAL;
  if (ic == CRKDG_IC_BURGERS_SIN && st->eq != EQ_BURGERS1) return CRKDG_EINVAL;
  if (ic == CRKDG_IC_SHOCK && !aux_dev) return CRKDG_EINVAL;
  if ((ic == CRKDG_IC_EULER_WAVE || ic == CRKDG_IC_VORTEX || ic == CRKDG_IC_QUADRANT ||
       ic == CRKDG_IC_SHOCK || ic == CRKDG_IC_DMR) && st->eq != EQ_EULER2)
    return CRKDG_EINVAL;
  double P[NPARAM];
  int rc = copy_params(st, params, nparams, P);
  if (rc) return rc;
  if (ic == CRKDG_IC_DMR) {
    if (nparams != 0) return CRKDG_EINVAL;
    dmr_params(st->ph.gamma, P);
  }
  double* Pd;
  rc = upload_params(st, P, &Pd);
  if (rc) return rc;
  if (int rs = sync_time(st)) return rs;
  hipError_t e = launch_project(st->eq, st->k, st->lay, st->ph, st->geo, ic, Pd, aux_dev, st->t,
                                cur_ptr(st), st->stream);
  return hip_rc(e);
}

// whether this step can run as one fused pass: 2D, a kernel for the
// equation/degree/precision/boundary data, and a subdiagonal tableau whose
// weights are nonzero only on the first and the last stage
static bool fusable(const crkdg_state* st) {
  if (st->mesh.dim != 2 || !fused_supported(st->eq, st->k, st->prec, st->bc)) return false;
  if (st->s > 1 && !st->subdiag) return false;
  for (int i = 1; i + 1 < st->s; ++i)
    if (st->b[i] != 0.0) return false;
  return true;
}

// one step with dt from the host (dt_dev == NULL) or from device memory
static int step_impl(crkdg_state* st, double dt, const double* dt_dev,
                     const double* t_dev = nullptr) {
  const void* un = cur_ptr(st);
  void* unew = nxt_ptr(st);
  hipError_t e = hipSuccess;
  const int s = st->s;
  if (st->sched == CRKDG_SCHED_FUSED && fusable(st)) {
    FusedArgs fa{};
    fa.un = un;
    fa.out = unew;
    fa.s = s;
    for (int i = 1; i < s; ++i) fa.a_sub[i] = st->A[i][i - 1];
    fa.w_first = st->b[0];
    fa.w_last = s > 1 ? st->b[s - 1] : 0.0;
    fa.dt = dt;
    fa.dt_ptr = dt_dev;
    {
      ProfScope ps(st, KC_FUSED);
      e = launch_fused(st->eq, st->k, st->prec, st->ph, st->geo, st->bc, fa, st->stream);
    }
    if (e != hipSuccess) return CRKDG_EHIP;
    st->cur ^= 1;
    return CRKDG_OK;
  }
  FinalArgs fa{};
  fa.base = un;
  fa.lay_base = st->lay;
  fa.out = unew;
  fa.dt = dt;
  fa.dt_ptr = dt_dev;
  const void* stages[MAXS];
  int lays[MAXS];
  stages[0] = un;
  lays[0] = st->lay;
  if (s > 1 && st->subdiag) {
    // all inner stages in one element-local pass
    InnerArgs ia{};
    ia.un = un;
    ia.lay_in = st->lay;
    ia.lay_stage = st->lay_stage;
    ia.s = s;
    ia.dt = dt;
    ia.dt_ptr = dt_dev;
    ia.store_mask = 0;
    for (int i = 1; i < s; ++i) {
      ia.a_sub[i] = st->A[i][i - 1];
      ia.stage[i] = stage_ptr(st, i);
      stages[i] = ia.stage[i];
      lays[i] = st->lay_stage;
      if (st->b[i] != 0.0) ia.store_mask |= 1 << i;
    }
    // a stage with b_i == 0 is still needed by later stages only through the
    // register chain, so it is not stored
    ProfScope ps(st, KC_INNER);
    e = launch_inner(st->eq, st->k, st->prec, st->ph, st->geo, ia, st->stream);
  } else if (s > 1) {
    if (st->prec != P64) return CRKDG_EUNSUPPORTED;  // materialised path: FP64 only
    // general tableau: one pass per inner stage computes L_{i-1} =
    // loc(u^(i-1)), keeps it in the workspace if a later stage uses it, and
    // forms u^(i) = u^n - dt sum_j a_ij L_j
    for (int i = 1; i < s && e == hipSuccess; ++i) {
      LocCombineArgs la{};
      la.in = (const double*)stages[i - 1];
      la.un = (const double*)un;
      bool later = false;
      for (int m = i + 1; m < s; ++m) later = later || st->A[m][i - 1] != 0.0;
      la.L_out = later ? (double*)lbuf_ptr(st, i - 1) : nullptr;
      for (int j = 0; j < i - 1; ++j) {
        if (st->A[i][j] == 0.0) continue;
        la.coef[la.nx] = dt_dev ? -st->A[i][j] : -dt * st->A[i][j];
        la.X[la.nx] = (const double*)lbuf_ptr(st, j);
        ++la.nx;
      }
      la.use_last = st->A[i][i - 1] != 0.0;
      la.coef_last = dt_dev ? -st->A[i][i - 1] : -dt * st->A[i][i - 1];
      la.dt_ptr = dt_dev;
      double* ui = (double*)stage_ptr(st, i);
      la.out = ui;
      ProfScope ps(st, KC_INNER);
      e = launch_loc_combine(st->eq, st->k, st->ph, st->geo, la, st->stream);
      stages[i] = ui;
      lays[i] = L64;
    }
  }
  if (e != hipSuccess) return CRKDG_EHIP;
  int ns = 0;
  for (int i = 0; i < s; ++i) {
    if (st->b[i] == 0.0) continue;
    fa.st[ns] = stages[i];
    fa.lay[ns] = lays[i];
    fa.w[ns] = st->b[i];
    fa.tst[ns] = st->t + st->c[i] * (dt_dev ? 0.0 : dt);
    fa.cst[ns] = st->c[i];
    ++ns;
  }
  fa.ns = ns;
  fa.t_ptr = t_dev;
  {
    ProfScope ps(st, KC_FINAL);
    e = launch_final(st->eq, st->k, st->prec, st->ph, st->geo, st->bc, fa, st->stream);
  }
  if (e != hipSuccess) return CRKDG_EHIP;
  st->cur ^= 1;
  return CRKDG_OK;
}

int crkdg_set_schedule(crkdg_state* st, int sched) {
  if (!st || (sched != CRKDG_SCHED_SPLIT && sched != CRKDG_SCHED_FUSED)) return CRKDG_EINVAL;
  if (sched == CRKDG_SCHED_FUSED && !fusable(st)) return CRKDG_EUNSUPPORTED;
  st->sched = sched;
  return CRKDG_OK;
}

int crkdg_get_schedule(const crkdg_state* st) {
  if (!st) return CRKDG_EINVAL;
  return st->sched == CRKDG_SCHED_FUSED && fusable(st) ? CRKDG_SCHED_FUSED : CRKDG_SCHED_SPLIT;
}

int crkdg_step(crkdg_state* st, double dt) {
  if (!st) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  if (!isfinite(dt) || !(dt > 0.0)) return CRKDG_EINVAL;
  int rc = sync_time(st);
  if (rc) return rc;
  rc = step_impl(st, dt, nullptr);
  if (rc == CRKDG_OK) st->t += dt;
  return rc;
}

int crkdg_step_dev(crkdg_state* st, const double* dt_dev) {
  if (!st || !dt_dev) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  if (st->bc.exact <= 0) return step_impl(st, 0.0, dt_dev);
  // time-dependent boundary data: the stage times come from a device copy
  // of the time, which then advances by *dt_dev on the device
  double* td = t_dev_ptr(st);
  if (!st->t_dev_valid) {
    if (launch_time_set(td, st->t, st->stream) != hipSuccess) return CRKDG_EHIP;
    st->t_dev_valid = true;
  }
  int rc = step_impl(st, 0.0, dt_dev, td);
  if (rc) return rc;
  return launch_time_add(td, dt_dev, st->stream) == hipSuccess ? CRKDG_OK : CRKDG_EHIP;
}

// forward declaration (defined with the limiter entry points below)
static int limit_impl(crkdg_state* st, double M, const float* params, float tau_lo, float tau_hi,
                      uint8_t* flags_dev, int64_t* counts, int ncounts, double cfl,
                      double* dt_dev, void* target, double t_ghost, const double* ghost_dt,
                      double ghost_fac);

// The original RKDG in the Shu--Osher SSP form (Section 2.1; the comparison
// scheme of Section 4): every stage applies the DG operator with face fluxes
// and, when M >= 0, the limiter.  Each stage is one final-stage launch whose
// update starts from bw1 u^n + bw2 u^(i-1) (FinalArgs::base2), so no separate
// combination pass.  Buffers: u^(1) in stage slot 1, u^(2) (order 3) or
// u^{n+1} (order 2) in the second state buffer; the order-3 result is
// written over u^n (each cell reads its own u^n before writing it, and the
// neighbour data come from u^(2) only).
int crkdg_step_rkdg(crkdg_state* st, int order, double M, double dt, const double* dt_dev) {
  if (!st) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  if ((order != 0 && order != 2 && order != 3) || isnan(M)) return CRKDG_EINVAL;
  if (order == 0 && M >= 0.0) return CRKDG_EINVAL;  // the Butcher form runs unlimited
  if (!dt_dev && (!isfinite(dt) || !(dt > 0.0))) return CRKDG_EINVAL;
  if (st->prec != P64) return CRKDG_EUNSUPPORTED;
  // time-dependent boundary data with dt on the device: the time lives in
  // device memory (as in crkdg_step_dev); otherwise on the host
  const bool tdev = dt_dev && st->bc.exact > 0;
  double* td = t_dev_ptr(st);
  if (tdev && !st->t_dev_valid) {
    if (launch_time_set(td, st->t, st->stream) != hipSuccess) return CRKDG_EHIP;
    st->t_dev_valid = true;
  }
  if (!tdev)
    if (int rs = sync_time(st)) return rs;
  char* u0 = cur_ptr(st);
  char* un = nxt_ptr(st);
  char* s1 = stage_ptr(st, 1);
  const double h = dt_dev ? 0.0 : dt;  // stage times of boundary data
  auto pass = [&](const void* base2, double bw1, double bw2, const void* stage, double w,
                  double t_bc, double c, void* out) {
    FinalArgs fa{};
    fa.t_ptr = tdev ? td : nullptr;
    fa.cst[0] = c;
    fa.base = u0;
    fa.lay_base = st->lay;
    fa.base2 = base2;
    fa.bw1 = bw1;
    fa.bw2 = bw2;
    fa.out = out;
    fa.dt = dt;
    fa.dt_ptr = dt_dev;
    fa.ns = 1;
    fa.st[0] = stage;
    fa.lay[0] = st->lay;
    fa.w[0] = w;
    fa.tst[0] = t_bc;
    ProfScope ps(st, KC_FINAL);
    return launch_final(st->eq, st->k, st->prec, st->ph, st->geo, st->bc, fa, st->stream) ==
                   hipSuccess
               ? CRKDG_OK
               : CRKDG_EHIP;
  };
  // each stage is limited with ghost data at the time it approximates, t + f dt
  auto limit = [&](void* u, double f) {
    if (M < 0.0) return (int)CRKDG_OK;
    return tdev ? limit_impl(st, M, nullptr, 0.f, 0.f, nullptr, nullptr, 1, 0.0, nullptr, u, NAN,
                             dt_dev, f)
                : limit_impl(st, M, nullptr, 0.f, 0.f, nullptr, nullptr, 1, 0.0, nullptr, u,
                             st->t + f * h, nullptr, 0.0);
  };
  const double t = st->t;
  if (order == 0) {
    // Butcher form with the state's tableau: E_i = -dt DG(u^(i)) at the
    // stage time t + c_i dt (a final-stage pass from a zero base), u^(i) =
    // u^n + sum_{j<i} a_ij E_j and u^{n+1} = u^n + sum_i b_i E_i (combination
    // passes); E_j lives in the j-th operator slot, the last one in the
    // second stage slot, u^(i) (i >= 1) in the first stage slot
    const int s = st->s;
    const long long n = (long long)(st->S / sizeof(double));
    auto E = [&](int j) { return (double*)(j < st->ws - 1 ? lbuf_ptr(st, j) : stage_ptr(st, 2)); };
    int rc = CRKDG_OK;
    for (int i = 0; i < s && !rc; ++i) {
      const void* ui = u0;
      if (i > 0) {
        double coef[MAXS];
        const double* X[MAXS];
        int nx = 0;
        for (int j = 0; j < i; ++j) {
          if (st->A[i][j] == 0.0) continue;
          coef[nx] = st->A[i][j];
          X[nx++] = E(j);
        }
        ProfScope ps(st, KC_COMBINE);
        if (launch_combine(n, (double*)s1, (const double*)u0, nx, coef, X, nullptr, st->stream) !=
            hipSuccess)
          rc = CRKDG_EHIP;
        ui = s1;
      }
      if (!rc) {
        FinalArgs fa{};
        fa.t_ptr = tdev ? td : nullptr;
        fa.cst[0] = st->c[i];
        fa.base = nullptr;
        fa.lay_base = st->lay;
        fa.out = E(i);
        fa.dt = dt;
        fa.dt_ptr = dt_dev;
        fa.ns = 1;
        fa.st[0] = ui;
        fa.lay[0] = st->lay;
        fa.w[0] = 1.0;
        fa.tst[0] = t + st->c[i] * h;
        ProfScope ps(st, KC_FINAL);
        if (launch_final(st->eq, st->k, st->prec, st->ph, st->geo, st->bc, fa, st->stream) !=
            hipSuccess)
          rc = CRKDG_EHIP;
      }
    }
    if (!rc) {
      double coef[MAXS];
      const double* X[MAXS];
      int nx = 0;
      for (int i = 0; i < s; ++i) {
        if (st->b[i] == 0.0) continue;
        coef[nx] = st->b[i];
        X[nx++] = E(i);
      }
      ProfScope ps(st, KC_COMBINE);
      if (launch_combine(n, (double*)un, (const double*)u0, nx, coef, X, nullptr, st->stream) !=
          hipSuccess)
        rc = CRKDG_EHIP;
    }
    if (!rc) st->cur ^= 1;
    if (!rc && tdev) rc = launch_time_add(td, dt_dev, st->stream) == hipSuccess ? CRKDG_OK : CRKDG_EHIP;
    if (!rc && !dt_dev) st->t += dt;
    return rc;
  }
  int rc = pass(nullptr, 1.0, 0.0, u0, 1.0, t, 0.0, s1);  // u^(1) = u^n - dt DG(u^n)
  if (!rc) rc = limit(s1, 1.0);
  if (order == 2) {  // u^{n+1} = u^n / 2 + (u^(1) - dt DG(u^(1))) / 2
    if (!rc) rc = pass(s1, 0.5, 0.5, s1, 0.5, t + h, 1.0, un);
    if (!rc) rc = limit(un, 1.0);
    if (!rc) st->cur ^= 1;
  } else {  // u^(2) = 3/4 u^n + 1/4 (u^(1) - dt DG(u^(1))), then the third stage
    if (!rc) rc = pass(s1, 0.75, 0.25, s1, 0.25, t + h, 1.0, un);
    if (!rc) rc = limit(un, 0.5);
    if (!rc) rc = pass(un, 1.0 / 3.0, 2.0 / 3.0, un, 2.0 / 3.0, t + 0.5 * h, 0.5, u0);
    if (!rc) rc = limit(u0, 1.0);
  }
  if (!rc && tdev) rc = launch_time_add(td, dt_dev, st->stream) == hipSuccess ? CRKDG_OK : CRKDG_EHIP;
  if (!rc && !dt_dev) st->t += dt;
  return rc;
}

int crkdg_compute_dt(crkdg_state* st, double cfl, double* dt_dev) {
  if (!st || !dt_dev || !isfinite(cfl) || !(cfl > 0.0)) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  double* partial = (double*)scratch_ptr(st);
  ProfScope ps(st, KC_DT);
  hipError_t e = launch_wavespeed(st->eq, st->k, st->lay, st->ph, st->geo, cur_ptr(st), partial,
                                  RED_BLOCKS, cfl, nullptr, dt_dev, st->stream);
  return hip_rc(e);
}

int crkdg_max_wavespeed(crkdg_state* st, double* smax) {
  if (!st || !smax) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  double* partial = (double*)scratch_ptr(st);
  double* res = partial + RED_BLOCKS * 2;
  hipError_t e = launch_wavespeed(st->eq, st->k, st->lay, st->ph, st->geo, cur_ptr(st), partial,
                                  RED_BLOCKS, 1.0, res, nullptr, st->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(smax, res, sizeof(double), hipMemcpyDeviceToHost, st->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  return hip_rc(e);
}

static int limit_impl(crkdg_state* st, double M, const float* params, float tau_lo, float tau_hi,
                      uint8_t* flags_dev, int64_t* counts, int ncounts, double cfl = 0.0,
                      double* dt_dev = nullptr, void* target = nullptr, double t_ghost = NAN,
                      const double* ghost_dt = nullptr, double ghost_fac = 0.0) {
  unsigned long long* counters =
      counts ? (unsigned long long*)(scratch_ptr(st) + SCRATCH - 64) : nullptr;
  hipError_t e;
  BCDev bc = st->bc;  // time-dependent ghost averages at the state's time
  bc.t = isnan(t_ghost) ? st->t : t_ghost;
  // with the time on the device: *t (+ ghost_fac * *ghost_dt within a step)
  bc.t_ptr = isnan(t_ghost) && st->t_dev_valid ? t_dev_ptr(st) : nullptr;
  bc.dt_ptr = bc.t_ptr ? ghost_dt : nullptr;
  bc.dt_fac = ghost_fac;
  {
    ProfScope ps(st, KC_LIMIT);
    e = launch_limit(st->eq, st->k, st->lay, st->ph, st->geo, bc, M, params, tau_lo, tau_hi,
                     target ? target : cur_ptr(st), flags_dev, counters,
                     dt_dev ? wave_partial_ptr(st) : nullptr,
                     st->stream);
  }
  if (e == hipSuccess && dt_dev) {
    ProfScope ps(st, KC_DT);
    e = launch_wave_final(wave_partial_ptr(st), wave_blocks(st), cfl, nullptr, dt_dev, st->stream);
  }
  if (e != hipSuccess) return CRKDG_EHIP;
  if (counts) {
    unsigned long long h[3] = {0, 0, 0};
    e = hipMemcpyAsync(h, counters, sizeof h, hipMemcpyDeviceToHost, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
    if (e != hipSuccess) return CRKDG_EHIP;
    counts[0] = (int64_t)h[0];
    if (ncounts > 1) counts[1] = (int64_t)h[2];
    if (h[1]) return CRKDG_ENONPHYSICAL;
  }
  return CRKDG_OK;
}

int crkdg_limit(crkdg_state* st, double M, uint8_t* flags_dev, int64_t* n_flagged) {
  if (!st || !isfinite(M) || M < 0.0) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  return limit_impl(st, M, nullptr, 0.f, 0.f, flags_dev, n_flagged, 1);
}

int crkdg_limit_mlp(crkdg_state* st, double M, const float* params_dev, float tau_lo,
                    float tau_hi, uint8_t* flags_dev, int64_t* counts_host) {
  if (!st || !params_dev || !isfinite(M) || M < 0.0 || !(tau_lo <= tau_hi)) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  if (st->eq != EQ_EULER2 || st->k < 1 || st->bc.exact == CRKDG_IC_DMR) return CRKDG_EUNSUPPORTED;
  return limit_impl(st, M, params_dev, tau_lo, tau_hi, flags_dev, counts_host, 2);
}

int crkdg_limit_dt(crkdg_state* st, double M, const float* params_dev, float tau_lo,
                   float tau_hi, uint8_t* flags_dev, double cfl, double* dt_dev) {
  if (!st || !dt_dev || !isfinite(M) || M < 0.0 || !isfinite(cfl) || !(cfl > 0.0))
    return CRKDG_EINVAL;
  if (params_dev && !(tau_lo <= tau_hi)) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  if (params_dev && (st->eq != EQ_EULER2 || st->k < 1 || st->bc.exact == CRKDG_IC_DMR))
    return CRKDG_EUNSUPPORTED;
  return limit_impl(st, M, params_dev, tau_lo, tau_hi, flags_dev, nullptr, 0, cfl, dt_dev);
}

int crkdg_mlp_features(crkdg_state* st, double M, float* X_dev) {
  if (!st || !X_dev || !isfinite(M) || M < 0.0) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  if (st->eq != EQ_EULER2 || st->k < 1 || st->bc.exact == CRKDG_IC_DMR) return CRKDG_EUNSUPPORTED;
  BCDev bc = st->bc;  // the limiter's ghost rules at the state's time
  bc.t = st->t;
  bc.t_ptr = st->t_dev_valid ? t_dev_ptr(st) : nullptr;
  return hip_rc(launch_mlp_features(st->k, st->lay, st->geo, bc, M, cur_ptr(st), X_dev,
                                    st->stream));
}

size_t crkdg_mlp_work_bytes(int B) { return B > 0 ? mlp_work_floats(B) * sizeof(float) : 0; }

int crkdg_mlp_forward(const float* params, const float* X, int B, float* logits, void* stream) {
  if (!params || !X || !logits || B < 1) return CRKDG_EINVAL;
  return hip_rc(launch_mlp_forward(params, X, B, logits, (hipStream_t)stream));
}

int crkdg_mlp_grad(const float* params, const float* X, const uint8_t* y, int B, float pos_weight,
                   float* grad, float* loss, void* work, size_t work_bytes, void* stream) {
  if (!params || !X || !y || !grad || !work || B < 1 || !isfinite(pos_weight) || pos_weight <= 0)
    return CRKDG_EINVAL;
  if (work_bytes < crkdg_mlp_work_bytes(B)) return CRKDG_EINVAL;
  return hip_rc(launch_mlp_grad(params, X, y, B, pos_weight, grad, loss, (float*)work,
                                (hipStream_t)stream));
}

int crkdg_mlp_grad_noalloc(const float* params, const float* X, const uint8_t* y, int B,
                           float pos_weight, float* grad, float* loss, void* stream) {
  if (!params || !X || !y || !grad || B < 1 || !isfinite(pos_weight) || pos_weight <= 0)
    return CRKDG_EINVAL;
  if (B > mlp_noalloc_max_batch()) return CRKDG_EINVAL;
  return hip_rc(launch_mlp_grad_noalloc(params, X, y, B, pos_weight, grad, loss,
                                        (hipStream_t)stream));
}

int crkdg_mlp_adam(float* params, float* m1, float* m2, const float* grad, int step, float lr,
                   float beta1, float beta2, float eps, void* stream) {
  if (!params || !m1 || !m2 || !grad || step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) ||
      !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return CRKDG_EINVAL;
  return hip_rc(launch_mlp_adam(params, m1, m2, grad, step, lr, beta1, beta2, eps,
                                (hipStream_t)stream));
}

int crkdg_error(crkdg_state* st, int ic, const double* params, int nparams, double t, int comp,
                double out[3]) {
  if (!st || !out || comp < 0 || comp >= st->nc) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  if (ic < CRKDG_IC_CONST || (ic > CRKDG_IC_QUADRANT && ic != CRKDG_IC_BURGERS_SIN))
    return CRKDG_EINVAL;
  if (ic == CRKDG_IC_BURGERS_SIN && st->eq != EQ_BURGERS1) return CRKDG_EINVAL;
  double P[NPARAM];
  int rc = copy_params(st, params, nparams, P);
  if (rc) return rc;
  double* Pd;
  rc = upload_params(st, P, &Pd);
  if (rc) return rc;
  double* partial = (double*)scratch_ptr(st);
  double* res = (double*)(scratch_ptr(st) + SCRATCH - 256);
  hipError_t e = launch_error(st->eq, st->k, st->lay, st->ph, st->geo, cur_ptr(st), ic, Pd,
                              nullptr, t, comp, partial, RED_BLOCKS, res, st->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, res, 3 * sizeof(double), hipMemcpyDeviceToHost, st->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  return hip_rc(e);
}

int crkdg_total(crkdg_state* st, int comp, double* out) {
  if (!st || !out || comp < 0 || comp >= st->nc) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  double* partial = (double*)scratch_ptr(st);
  double* res = (double*)(scratch_ptr(st) + SCRATCH - 256);
  hipError_t e = launch_total(st->eq, st->k, st->lay, st->geo, cur_ptr(st), comp, partial,
                              RED_BLOCKS, res, st->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, st->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  return hip_rc(e);
}

static const double* avg_base(const crkdg_state* st, int comp) {
  const double* u = (const double*)cur_ptr(st);
  const long long N = st->geo.N;
  return st->lay == LMIX ? u + (long long)comp * N : u + (long long)comp * st->nb * N;
}

int crkdg_error_ref(crkdg_state* st, crkdg_state* ref, int comp, double out[3]) {
  if (!st || !ref || !out || comp < 0 || comp >= st->nc) return CRKDG_EINVAL;
  if (!st->bound || !ref->bound) return CRKDG_EUNBOUND;
  if (ref->eq != st->eq || ref->nc != st->nc) return CRKDG_EINVAL;
  const Geo& g = st->geo;
  const Geo& f = ref->geo;
  const bool two_d = st->mesh.dim == 2;
  if (ref->mesh.dim != st->mesh.dim || f.nx % g.nx != 0 || (two_d && f.ny % g.ny != 0))
    return CRKDG_EINVAL;
  const int r = f.nx / g.nx, ry = two_d ? f.ny / g.ny : 1;
  // same domain: the fine cells must tile the coarse ones exactly
  const double tol = 1e-12;
  if (fabs(f.dx * r - g.dx) > tol * g.dx || fabs(f.x0 - g.x0) > tol * (g.dx + fabs(g.x0)) ||
      (two_d && (fabs(f.dy * ry - g.dy) > tol * g.dy || fabs(f.y0 - g.y0) > tol * (g.dy + fabs(g.y0)))))
    return CRKDG_EINVAL;
  if (ref->stream != st->stream) {
    hipError_t e = hipStreamSynchronize(ref->stream);
    if (e != hipSuccess) return hip_rc(e);
  }
  double* partial = (double*)scratch_ptr(st);
  double* res = (double*)(scratch_ptr(st) + SCRATCH - 256);
  const double area = g.dx * (two_d ? g.dy : 1.0);
  hipError_t e = launch_error_ref(g, avg_base(st, comp), avg_base(ref, comp), r, ry, f.nx, area,
                                  partial, RED_BLOCKS, res, st->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, res, 3 * sizeof(double), hipMemcpyDeviceToHost, st->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  return hip_rc(e);
}

int crkdg_apply_op(crkdg_state* st, int op, const void* in, void* out, double t_bc) {
  if (!st || !in || !out || (op != CRKDG_OP_LOC && op != CRKDG_OP_DG)) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  if (in == out) return CRKDG_EINVAL;
  if (st->lay != L64) return CRKDG_EUNSUPPORTED;
  hipError_t e;
  if (op == CRKDG_OP_LOC) {
    e = launch_loc(st->eq, st->k, st->ph, st->geo, (const double*)in, (double*)out, st->stream);
  } else {
    // out = 0 - (-1) * DG(in)
    FinalArgs fa{};
    fa.base = nullptr;
    fa.lay_base = L64;
    fa.out = out;
    fa.ns = 1;
    fa.st[0] = in;
    fa.lay[0] = L64;
    fa.w[0] = 1.0;
    fa.tst[0] = t_bc;
    fa.dt = -1.0;
    e = launch_final(st->eq, st->k, P64, st->ph, st->geo, st->bc, fa, st->stream);
  }
  return hip_rc(e);
}

int crkdg_combine(crkdg_state* st, void* out, const void* base, int n, const double* coef,
                  const void* const* X) {
  if (!st || !out || n < 0 || n > MAXS || (n > 0 && (!coef || !X))) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  if (st->lay != L64) return CRKDG_EUNSUPPORTED;
  for (int j = 0; j < n; ++j)
    if (!X[j] || !isfinite(coef[j])) return CRKDG_EINVAL;
  const long long len = (long long)(st->S / sizeof(double));
  const double* Xd[MAXS];
  for (int j = 0; j < n; ++j) Xd[j] = (const double*)X[j];
  return hip_rc(launch_combine(len, (double*)out, (const double*)base, n, coef, Xd, nullptr,
                               st->stream));
}

int crkdg_profile_begin(crkdg_state* st, int max_launches) {
  if (!st || max_launches < 1 || max_launches > (1 << 20)) return CRKDG_EINVAL;
  if (!st->bound) return CRKDG_EUNBOUND;
  if ((int)st->ev.size() < 2 * max_launches) {
    const size_t old = st->ev.size();
    st->ev.resize(2 * (size_t)max_launches);
    for (size_t e = old; e < st->ev.size(); ++e)
      // timing-only events: no system-scope fence (and cache writeback) at
      // each record; profile_end synchronises the stream before reading them
      if (hipEventCreateWithFlags(&st->ev[e], hipEventDisableSystemFence) != hipSuccess) {
        st->ev.resize(e);
        return CRKDG_EHIP;
      }
  }
  st->ev_cls.assign(max_launches, 0);
  st->prof_max = max_launches;
  st->prof_n = 0;
  st->prof = true;
  return CRKDG_OK;
}

int crkdg_profile_end(crkdg_state* st, double ms[8], int64_t counts[8]) {
  if (!st || !ms || !counts) return CRKDG_EINVAL;
  for (int c = 0; c < 8; ++c) {
    ms[c] = 0.0;
    counts[c] = 0;
  }
  if (!st->prof) return CRKDG_EINVAL;
  st->prof = false;
  if (hipStreamSynchronize(st->stream) != hipSuccess) return CRKDG_EHIP;
  for (int i = 0; i < st->prof_n; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, st->ev[2 * i], st->ev[2 * i + 1]) != hipSuccess) return CRKDG_EHIP;
    ms[st->ev_cls[i]] += t;
    counts[st->ev_cls[i]] += 1;
  }
  return CRKDG_OK;
}

void crkdg_destroy(crkdg_state* st) {
  if (!st) return;
  for (hipEvent_t e : st->ev) (void)hipEventDestroy(e);
  delete st;
}

}  // extern "C"
