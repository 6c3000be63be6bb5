// C ABI of librpywall.so: argument validation, workspace handling, launch
// shape table, instrumentation.  Validation runs on the host before any HIP
// call, so a rejected call touches no device state.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "rpyw_internal.h"

namespace rpyw {

namespace {

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }
bool valid_prec(int p) { return p == RPYW_FP64 || p == RPYW_FP32C; }
constexpr int64_t kMaxN = (int64_t)1 << 31;

// Scratch: the caller's workspace, or stream-ordered memory owned for the
// duration of one call.
struct Scratch {
    Arena ar{nullptr, 0, 0};
    void* owned = nullptr;
    hipStream_t st = nullptr;
    ~Scratch() {
        if (owned) (void)hipFreeAsync(owned, st);
    }
};

int acquire(void* ws, size_t ws_bytes, size_t need, hipStream_t st, Scratch& s) {
    s.st = st;
    if (ws) {
        if (((uintptr_t)ws % kAlign) != 0) return RPYW_EINVAL;
        if (ws_bytes < need) return RPYW_ENOMEM;
        s.ar = Arena{(char*)ws, ws_bytes, 0};
        return RPYW_OK;
    }
    if (hipMallocAsync(&s.owned, need, st) != hipSuccess) {
        s.owned = nullptr;
        return RPYW_ENOMEM;
    }
    s.ar = Arena{(char*)s.owned, need, 0};
    return RPYW_OK;
}

// ---------------------------------------------------------- fixed scratch
// Workspace of rpy_wall_matvec_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code uses its device address
// from hipGetSymbolAddress (taken once per device, with that device
// current), never the array's name.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, or nullptr.
void* scratch_address() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// ---------------------------------------------------------- shape table
std::mutex g_shape_mu;
std::map<std::tuple<int, int, int>, Shape> g_shapes;     // tuned (and persisted)
std::map<std::tuple<int, int, int>, Shape> g_overrides;  // rpy_wall_set_shape (not persisted)

int size_class(int64_t N) {
    int c = 0;
    while (((int64_t)1 << (c + 1)) <= N) ++c;
    return c;
}
int kclass(int k) {
    int p = 1;
    while (p < k && p < 16) p <<= 1;
    return p;
}

// ---------------------------------------------------------- profiling
struct ProfRec {
    hipEvent_t a, b;
    double pairs;
};
bool g_prof = false;
std::vector<ProfRec> g_prof_recs;
double g_prof_ms = 0.0, g_prof_pairs = 0.0;
int64_t g_prof_n = 0;

}  // namespace

// Defaults from measurements on MI355X: the symmetric kernel wins for one
// right-hand side from a few hundred blobs up (1.7x at 1e5, 2x at 1000,
// where its passes are also split into segments); groups of
// 64 blobs, one item per workgroup, are up to 3x faster than groups of 256
// below ten thousand blobs (which leave the GPU underfilled) and still 5% at
// 30000; wider RHS blocks are faster on the plain kernel, and FP32C blocks
// of 8 or more are contracted on the matrix cores.  For groups of 256
// ipw keeps the grid at roughly 16k workgroups or more.
Shape default_shape(int64_t N, int k, int prec) {
    Shape s;
    s.tpl = N >= 65536 ? 2 : 1;
    s.tile = 64;
    // FP64: blocks of up to 8 on the vector units; 9 to 16 right-hand sides
    // go to the matrix cores as one block of 16 (a block of 8 there would
    // leave half of every contraction empty).
    s.kblk = std::min(kclass(k), prec == RPYW_FP32C ? 16 : (kclass(k) > 8 ? 16 : 8));
    s.sym = (s.kblk == 1 && N >= 512) ? (N <= kSym64MaxN ? 2 : 1) : 0;
    const int64_t ng = (N + 255) / 256, hm = ng / 2 + 1;
    s.ipw = s.sym == 2 ? 1 : (int)std::max<int64_t>(1, std::min<int64_t>(4, hm * ng / 16384));
    s.mat = (s.kblk >= (prec == RPYW_FP32C ? 8 : 16)) ? 1 : 0;
    return s;
}

namespace {
// Persisted shapes: loaded once (under g_shape_mu) from RPYW_AUTOTUNE_CACHE;
// entries of other GPU architectures are kept for the rewrite.
bool g_cache_loaded = false;
std::vector<CachedShape> g_foreign;

void load_cache_locked() {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const char* path = autotune_cache_path();
    if (!path) return;
    std::vector<CachedShape> entries;
    if (read_shape_cache(path, entries) != 0) {
        log_line("autotune cache %s not read (missing or unparsable)", path);
        return;
    }
    const std::string arch = device_arch();
    int used = 0;
    for (const CachedShape& c : entries) {
        if (c.arch != arch) {
            g_foreign.push_back(c);
            continue;
        }
        const auto key = std::make_tuple(c.prec, c.size_class, c.kclass);
        if (!g_shapes.count(key)) {
            g_shapes[key] = c.s;
            ++used;
        }
    }
    log_line("autotune cache %s: %d shapes for %s", path, used, arch.c_str());
}

void save_cache_locked() {
    const char* path = autotune_cache_path();
    if (!path) return;
    std::vector<CachedShape> out = g_foreign;
    const std::string arch = device_arch();
    for (const auto& kv : g_shapes) {
        CachedShape c;
        c.arch = arch;
        c.prec = std::get<0>(kv.first);
        c.size_class = std::get<1>(kv.first);
        c.kclass = std::get<2>(kv.first);
        c.s = kv.second;
        out.push_back(c);
    }
    if (write_shape_cache(path, out) != 0) log_line("autotune cache %s not written", path);
}
}  // namespace

Shape tuned_shape(int64_t N, int k, int prec) {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    load_cache_locked();
    const std::tuple<int, int, int> key{prec, size_class(N), kclass(k)};
    auto ov = g_overrides.find(key);
    if (ov != g_overrides.end()) return apply_env_overrides(ov->second);
    auto it = g_shapes.find(key);
    return apply_env_overrides(it != g_shapes.end() ? it->second : default_shape(N, k, prec));
}

void set_tuned_shape(int64_t N, int k, int prec, Shape s) {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    load_cache_locked();
    g_shapes[{prec, size_class(N), kclass(k)}] = s;
}

void set_shape_override(int64_t N, int k, int prec, Shape s) {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_overrides[{prec, size_class(N), kclass(k)}] = s;
}

void clear_shape_override(int64_t N, int k, int prec) {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_overrides.erase({prec, size_class(N), kclass(k)});
}

bool profiling_enabled() { return g_prof; }

// One log line for a product-type call: sizes, precision, the launch shape
// its products use, and the status.
void log_shape(const char* fn, int64_t N, int k, int prec, int rc) {
    const Shape sh = tuned_shape(N, k, prec);
    log_line("%s N=%lld k=%d prec=%d shape tpl=%d tile=%d kblk=%d sym=%d ipw=%d mat=%d status=%d", fn, (long long)N, k,
             prec, sh.tpl, sh.tile, sh.kblk, sh.sym, sh.ipw, sh.mat, rc);
}

void profile_begin(hipStream_t st, hipEvent_t* ev) {
    *ev = nullptr;
    if (!g_prof) return;
    if (hipEventCreate(ev) != hipSuccess) {
        *ev = nullptr;
        return;
    }
    (void)hipEventRecord(*ev, st);
}

void profile_end(hipStream_t st, hipEvent_t ev0, double pairs) {
    if (!g_prof || !ev0) return;
    hipEvent_t ev1;
    if (hipEventCreate(&ev1) != hipSuccess) return;
    (void)hipEventRecord(ev1, st);
    g_prof_recs.push_back({ev0, ev1, pairs});
}

}  // namespace rpyw

using namespace rpyw;

extern "C" {

const char* rpyw_strerror(int status) {
    switch (status) {
        case RPYW_OK: return "ok";
        case RPYW_NOT_CONVERGED: return "iteration limit reached before the tolerance (best iterate written)";
        case RPYW_EINVAL: return "invalid argument";
        case RPYW_EHIP: return "HIP runtime error";
        case RPYW_ENOMEM: return "workspace too small or device allocation failed";
        case RPYW_ENOTSPD: return "preconditioner block not positive definite";
        default: return "unknown status";
    }
}

size_t rpy_wall_workspace_bytes(int op, int64_t N, int32_t k, int32_t max_iter, int32_t n_bodies, int precision) {
    if (N < 1 || N >= kMaxN || !valid_prec(precision)) return 0;
    switch (op) {
        case RPYW_OP_MATVEC: {
            if (k < 1) return 0;
            return product_ws_bytes(N, precision, std::min(kclass(k), 16));
        }
        case RPYW_OP_BATCHED:
            if (k < 1 || n_bodies < 1) return 0;
            return batched_ws_bytes(N, n_bodies, k, precision);
        case RPYW_OP_LANCZOS:
            if (max_iter < 1) return 0;
            return lanczos_ws_bytes(N, max_iter, n_bodies, precision);
        case RPYW_OP_VJP:
        case RPYW_OP_DIVERGENCE: return vjp_ws_bytes(N, precision);
        case RPYW_OP_RIGID:
            if (max_iter < 1 || n_bodies < 1) return 0;
            return rigid_ws_bytes(N, max_iter, n_bodies, precision);
        case RPYW_OP_TS:
            if (max_iter < 1 || n_bodies < 1) return 0;
            return ts_ws_bytes(N, max_iter, n_bodies, precision);
        default: return 0;
    }
}

int rpy_wall_matvec_multi(const double* pos, const double* F, double* U, int64_t N, int32_t k, double a,
                          double eta, int precision, void* ws, size_t ws_bytes, void* stream) {
    if (!pos || !F || !U || N < 1 || N >= kMaxN || k < 1 || k > 4096 || !finite_pos(a) || !finite_pos(eta) ||
        !valid_prec(precision))
        return RPYW_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Scratch s;
    int rc = acquire(ws, ws_bytes, product_ws_bytes(N, precision, std::min(kclass(k), 16)), st, s);
    if (rc == RPYW_OK) rc = products(pos, F, U, N, k, a, eta, precision, s.ar, st);
    if (log_enabled()) log_shape("rpy_wall_matvec_multi", N, k, precision, rc);
    return rc;
}

int rpy_wall_matvec_periodic(const double* pos, const double* F, double* U, int64_t N, int32_t k, double a,
                             double eta, double Lx, double Ly, int precision, void* ws, size_t ws_bytes,
                             void* stream) {
    if (!pos || !F || !U || N < 1 || N >= kMaxN || k < 1 || k > 4096 || !finite_pos(a) || !finite_pos(eta) ||
        !finite_pos(Lx) || !finite_pos(Ly) || !valid_prec(precision))
        return RPYW_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Scratch s;
    int rc = acquire(ws, ws_bytes, product_ws_bytes(N, precision, 1), st, s);
    if (rc == RPYW_OK) rc = products(pos, F, U, N, k, a, eta, precision, s.ar, st, Domain{Lx, Ly});
    if (log_enabled()) log_shape("rpy_wall_matvec_periodic", N, k, precision, rc);
    return rc;
}

int rpy_wall_matvec(const double* pos, const double* force, double* vel, int64_t N, double a, double eta,
                    int precision, void* ws, size_t ws_bytes, void* stream) {
    return rpy_wall_matvec_multi(pos, force, vel, N, 1, a, eta, precision, ws, ws_bytes, stream);
}

size_t rpy_wall_noalloc_scratch_bytes(void) { return kScratchBytes; }

int rpy_wall_matvec_noalloc(const double* pos, const double* force, double* vel, int64_t N, double a, double eta,
                            int precision, void* stream) {
    if (!pos || !force || !vel || N < 1 || N >= kMaxN || !finite_pos(a) || !finite_pos(eta) ||
        !valid_prec(precision))
        return RPYW_EINVAL;
    if (product_ws_bytes(N, precision, 1) > kScratchBytes) {
        log_line("rpy_wall_matvec_noalloc N=%lld: workspace %zu B exceeds the fixed scratch (%zu B)", (long long)N,
                 product_ws_bytes(N, precision, 1), kScratchBytes);
        return RPYW_ENOMEM;
    }
    void* p = scratch_address();
    if (!p) return RPYW_EHIP;
    Arena ar{(char*)p, kScratchBytes, 0};
    const int rc = products(pos, force, vel, N, 1, a, eta, precision, ar, (hipStream_t)stream);
    if (log_enabled()) log_shape("rpy_wall_matvec_noalloc", N, 1, precision, rc);
    return rc;
}

int rpy_wall_matvec_batched(const double* pos, const int64_t* sys_offsets, int32_t S, const double* F, double* U,
                            int32_t k, double a, double eta, int precision, void* ws, size_t ws_bytes,
                            void* stream) {
    if (!pos || !sys_offsets || !F || !U || S < 1 || k < 1 || k > 4096 || !finite_pos(a) || !finite_pos(eta) ||
        !valid_prec(precision))
        return RPYW_EINVAL;
    if (sys_offsets[0] != 0) return RPYW_EINVAL;
    for (int s = 0; s < S; ++s)
        if (sys_offsets[s + 1] <= sys_offsets[s]) return RPYW_EINVAL;
    const int64_t Ntot = sys_offsets[S];
    if (Ntot >= kMaxN) return RPYW_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Scratch s;
    int rc = acquire(ws, ws_bytes, batched_ws_bytes(Ntot, S, k, precision), st, s);
    if (rc == RPYW_OK) rc = batched_products(pos, sys_offsets, S, F, U, k, a, eta, precision, s.ar, st);
    log_line("rpy_wall_matvec_batched S=%d Ntot=%lld k=%d prec=%d status=%d", S, (long long)Ntot, k, precision, rc);
    return rc;
}

static int lanczos_api(const double* pos, const double* W, double* out, int64_t N, double a, double eta,
                       const int64_t* body_offsets, int32_t n_bodies, double tol, int32_t max_iter, int precision,
                       void* ws, size_t ws_bytes, int32_t* iters_out, double* err_est_out, void* stream,
                       const Domain& dom) {
    if (!pos || !W || !out || N < 1 || N >= kMaxN || !finite_pos(a) || !finite_pos(eta) || !valid_prec(precision) ||
        !finite_pos(tol) || max_iter < 1 || max_iter > 100000)
        return RPYW_EINVAL;
    if (body_offsets) {
        if (n_bodies < 1 || body_offsets[0] != 0 || body_offsets[n_bodies] != N) return RPYW_EINVAL;
        for (int p = 0; p < n_bodies; ++p) {
            const int64_t n = body_offsets[p + 1] - body_offsets[p];
            if (n < 1 || n > kMaxBodyBlobs) return RPYW_EINVAL;
        }
    } else {
        n_bodies = 0;
    }
    hipStream_t st = (hipStream_t)stream;
    Scratch s;
    int rc = acquire(ws, ws_bytes, lanczos_ws_bytes(N, max_iter, n_bodies, precision), st, s);
    if (rc != RPYW_OK) return rc;
    int it = 0;
    double err = 0.0;
    rc = lanczos_sqrt(pos, W, out, N, a, eta, body_offsets, n_bodies, tol, max_iter, precision, s.ar, &it, &err, st,
                      dom);
    if (iters_out) *iters_out = it;
    if (err_est_out) *err_est_out = err;
    log_line("rpy_wall_lanczos_sqrt%s N=%lld bodies=%d prec=%d tol=%g iterations=%d change=%.3e status=%d",
             dom.periodic() ? "_periodic" : "", (long long)N, n_bodies, precision, tol, it, err, rc);
    return rc;
}

int rpy_wall_lanczos_sqrt(const double* pos, const double* W, double* out, int64_t N, double a, double eta,
                          const int64_t* body_offsets, int32_t n_bodies, double tol, int32_t max_iter,
                          int precision, void* ws, size_t ws_bytes, int32_t* iters_out, double* err_est_out,
                          void* stream) {
    return lanczos_api(pos, W, out, N, a, eta, body_offsets, n_bodies, tol, max_iter, precision, ws, ws_bytes,
                       iters_out, err_est_out, stream, Domain{});
}

int rpy_wall_lanczos_sqrt_periodic(const double* pos, const double* W, double* out, int64_t N, double a, double eta,
                                   double Lx, double Ly, const int64_t* body_offsets, int32_t n_bodies, double tol,
                                   int32_t max_iter, int precision, void* ws, size_t ws_bytes, int32_t* iters_out,
                                   double* err_est_out, void* stream) {
    if (!finite_pos(Lx) || !finite_pos(Ly)) return RPYW_EINVAL;
    return lanczos_api(pos, W, out, N, a, eta, body_offsets, n_bodies, tol, max_iter, precision, ws, ws_bytes,
                       iters_out, err_est_out, stream, Domain{Lx, Ly});
}

static int rigid_api(const double* pos, const double* q, const int64_t* body_offsets, int32_t n_bodies,
                     const double* slip, const double* force_torque, double* lambda, double* U, int64_t N, double a,
                     double eta, double tol, int32_t max_iter, int precision, void* ws, size_t ws_bytes,
                     int32_t* iters_out, double* res_out, void* stream, const Domain& dom) {
    if (!pos || !q || !body_offsets || !lambda || !U || N < 1 || N >= kMaxN || n_bodies < 1 || !finite_pos(a) ||
        !finite_pos(eta) || !valid_prec(precision) || !finite_pos(tol) || max_iter < 1 || max_iter > 100000)
        return RPYW_EINVAL;
    if (body_offsets[0] != 0 || body_offsets[n_bodies] != N) return RPYW_EINVAL;
    for (int p = 0; p < n_bodies; ++p) {
        const int64_t n = body_offsets[p + 1] - body_offsets[p];
        if (n < 1 || n > kMaxBodyBlobs) return RPYW_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    Scratch s;
    int rc = acquire(ws, ws_bytes, rigid_ws_bytes(N, max_iter, n_bodies, precision), st, s);
    if (rc != RPYW_OK) return rc;
    int it = 0;
    double res = 0.0;
    rc = rigid_solve(pos, q, body_offsets, n_bodies, slip, force_torque, lambda, U, N, a, eta, tol, max_iter,
                     precision, s.ar, &it, &res, st, dom);
    if (iters_out) *iters_out = it;
    if (res_out) *res_out = res;
    log_line("rpy_wall_rigid_solve%s N=%lld bodies=%d prec=%d tol=%g iterations=%d residual=%.3e status=%d",
             dom.periodic() ? "_periodic" : "", (long long)N, n_bodies, precision, tol, it, res, rc);
    return rc;
}

int rpy_wall_rigid_solve(const double* pos, const double* q, const int64_t* body_offsets, int32_t n_bodies,
                         const double* slip, const double* force_torque, double* lambda, double* U, int64_t N,
                         double a, double eta, double tol, int32_t max_iter, int precision, void* ws,
                         size_t ws_bytes, int32_t* iters_out, double* res_out, void* stream) {
    return rigid_api(pos, q, body_offsets, n_bodies, slip, force_torque, lambda, U, N, a, eta, tol, max_iter,
                     precision, ws, ws_bytes, iters_out, res_out, stream, Domain{});
}

int rpy_wall_rigid_solve_periodic(const double* pos, const double* q, const int64_t* body_offsets, int32_t n_bodies,
                                  const double* slip, const double* force_torque, double* lambda, double* U,
                                  int64_t N, double a, double eta, double Lx, double Ly, double tol,
                                  int32_t max_iter, int precision, void* ws, size_t ws_bytes, int32_t* iters_out,
                                  double* res_out, void* stream) {
    if (!finite_pos(Lx) || !finite_pos(Ly)) return RPYW_EINVAL;
    return rigid_api(pos, q, body_offsets, n_bodies, slip, force_torque, lambda, U, N, a, eta, tol, max_iter,
                     precision, ws, ws_bytes, iters_out, res_out, stream, Domain{Lx, Ly});
}

static bool valid_bodies(const int64_t* offs, int32_t nb, int64_t N) {
    if (!offs || nb < 1 || offs[0] != 0 || offs[nb] != N) return false;
    for (int p = 0; p < nb; ++p) {
        const int64_t n = offs[p + 1] - offs[p];
        if (n < 1 || n > kMaxBodyBlobs) return false;
    }
    return true;
}

static bool valid_cell(double Lx, double Ly) {
    return (Lx == 0.0 && Ly == 0.0) || (finite_pos(Lx) && finite_pos(Ly));
}

int rpy_wall_body_blobs(const double* q, const double* theta, const double* ref, const int64_t* body_offsets,
                        int32_t n_bodies, double* pos, int64_t N, void* ws, size_t ws_bytes, void* stream) {
    if (!q || !theta || !ref || !pos || N < 1 || N >= kMaxN || !body_offsets || n_bodies < 1 ||
        body_offsets[0] != 0 || body_offsets[n_bodies] != N)
        return RPYW_EINVAL;
    for (int p = 0; p < n_bodies; ++p)
        if (body_offsets[p + 1] <= body_offsets[p]) return RPYW_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Scratch s;
    int rc = acquire(ws, ws_bytes, align_up((size_t)(n_bodies + 1) * sizeof(int)) + kAlign, st, s);
    if (rc != RPYW_OK) return rc;
    int* bofs = (int*)s.ar.take((size_t)(n_bodies + 1) * sizeof(int));
    if (!bofs) return RPYW_ENOMEM;
    std::vector<int> hb(n_bodies + 1);
    for (int p = 0; p <= n_bodies; ++p) hb[p] = (int)body_offsets[p];
    if ((rc = stage_upload(hb.data(), hb.size() * sizeof(int), bofs, st))) return rc;
    return body_blobs(q, theta, ref, bofs, n_bodies, pos, st);
}

int rpy_wall_body_move(const double* q, const double* theta, const double* U, double h, int32_t n_bodies,
                       double* q_out, double* theta_out, void* stream) {
    if (!q || !theta || !U || !q_out || !theta_out || n_bodies < 1 || !std::isfinite(h)) return RPYW_EINVAL;
    return body_move(q, theta, U, nullptr, h, n_bodies, q_out, theta_out, (hipStream_t)stream);
}

size_t rpy_wall_ts_state_bytes(int64_t N, int32_t n_bodies) {
    if (N < 1 || N >= kMaxN || n_bodies < 1) return 0;
    return ts_state_bytes(N, n_bodies);
}

int rpy_wall_ts_predict(const double* q, const double* theta, const double* ref, const int64_t* body_offsets,
                        int32_t n_bodies, int64_t N, const double* Lp, const double* force_torque, const double* Ws,
                        const double* Wn, double kT, double dt, double delta, double a, double eta, double Lx,
                        double Ly, double tol, int32_t max_iter, int precision, double* q_tilde, double* theta_tilde,
                        double* pos_tilde, void* state, size_t state_bytes, void* ws, size_t ws_bytes,
                        int32_t* iters_out, void* stream) {
    if (!q || !theta || !ref || !Lp || !force_torque || !Ws || !Wn || !q_tilde || !theta_tilde || !pos_tilde ||
        !state || N < 1 || N >= kMaxN || !valid_bodies(body_offsets, n_bodies, N) || !(kT >= 0.0) ||
        !std::isfinite(kT) || !finite_pos(dt) || !finite_pos(delta) || !finite_pos(a) || !finite_pos(eta) ||
        !valid_cell(Lx, Ly) || !finite_pos(tol) || max_iter < 1 || max_iter > 100000 || !valid_prec(precision) ||
        state_bytes < ts_state_bytes(N, n_bodies) || ((uintptr_t)state % 256) != 0)
        return RPYW_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Scratch s;
    int rc = acquire(ws, ws_bytes, ts_ws_bytes(N, max_iter, n_bodies, precision), st, s);
    if (rc != RPYW_OK) return rc;
    int it[3] = {0, 0, 0};
    rc = ts_predict(q, theta, ref, body_offsets, n_bodies, N, Lp, force_torque, Ws, Wn, kT, dt, delta, a, eta,
                    Domain{Lx, Ly}, tol, max_iter, precision, q_tilde, theta_tilde, pos_tilde, (double*)state, s.ar,
                    it, st);
    if (iters_out)
        for (int k = 0; k < 3; ++k) iters_out[k] = it[k];
    return rc;
}

int rpy_wall_ts_correct(const double* q, const double* theta, const double* q_tilde, const double* theta_tilde,
                        const double* ref, const int64_t* body_offsets, int32_t n_bodies, int64_t N,
                        const double* force_torque_tilde, const void* state, double dt, double a, double eta,
                        double Lx, double Ly, double tol, int32_t max_iter, int precision, double* q_next,
                        double* theta_next, void* ws, size_t ws_bytes, int32_t* iters_out, void* stream) {
    if (!q || !theta || !q_tilde || !theta_tilde || !ref || !force_torque_tilde || !state || !q_next ||
        !theta_next || N < 1 || N >= kMaxN || !valid_bodies(body_offsets, n_bodies, N) || !finite_pos(dt) ||
        !finite_pos(a) || !finite_pos(eta) || !valid_cell(Lx, Ly) || !finite_pos(tol) || max_iter < 1 ||
        max_iter > 100000 || !valid_prec(precision) || ((uintptr_t)state % 256) != 0)
        return RPYW_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Scratch s;
    int rc = acquire(ws, ws_bytes, ts_ws_bytes(N, max_iter, n_bodies, precision), st, s);
    if (rc != RPYW_OK) return rc;
    int it = 0;
    rc = ts_correct(q, theta, q_tilde, theta_tilde, ref, body_offsets, n_bodies, N, force_torque_tilde,
                    (const double*)state, dt, a, eta, Domain{Lx, Ly}, tol, max_iter, precision, q_next, theta_next,
                    s.ar, &it, st);
    if (iters_out) *iters_out = it;
    return rc;
}

int rpy_wall_emt_step(const double* q, const double* theta, const double* ref, const int64_t* body_offsets,
                      int32_t n_bodies, int64_t N, const double* Lp, const double* force_torque, const double* Wf,
                      const double* Wt, const double* Wn, double kT, double dt, double delta, double a, double eta,
                      double Lx, double Ly, double tol, int32_t max_iter, int precision, double* q_next,
                      double* theta_next, void* ws, size_t ws_bytes, int32_t* iters_out, void* stream) {
    if (!q || !theta || !ref || !Lp || !force_torque || !Wf || !Wt || !Wn || !q_next || !theta_next || N < 1 ||
        N >= kMaxN || !valid_bodies(body_offsets, n_bodies, N) || !(kT >= 0.0) || !std::isfinite(kT) ||
        !finite_pos(dt) || !finite_pos(delta) || !finite_pos(a) || !finite_pos(eta) || !valid_cell(Lx, Ly) ||
        !finite_pos(tol) || max_iter < 1 || max_iter > 100000 || !valid_prec(precision))
        return RPYW_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Scratch s;
    int rc = acquire(ws, ws_bytes, ts_ws_bytes(N, max_iter, n_bodies, precision), st, s);
    if (rc != RPYW_OK) return rc;
    int it[3] = {0, 0, 0};
    rc = emt_step(q, theta, ref, body_offsets, n_bodies, N, Lp, force_torque, Wf, Wt, Wn, kT, dt, delta, a, eta,
                  Domain{Lx, Ly}, tol, max_iter, precision, q_next, theta_next, s.ar, it, st);
    if (iters_out)
        for (int k = 0; k < 3; ++k) iters_out[k] = it[k];
    return rc;
}

int rpy_wall_emrfd_step(const double* q, const double* theta, const double* ref, const int64_t* body_offsets,
                        int32_t n_bodies, int64_t N, const double* Lp, const double* force_torque, const double* Wf,
                        const double* Wt, const double* Wn, double kT, double dt, double delta, double a, double eta,
                        double Lx, double Ly, double tol, int32_t max_iter, int precision, double* q_next,
                        double* theta_next, void* ws, size_t ws_bytes, int32_t* iters_out, void* stream) {
    if (!q || !theta || !ref || !Lp || !force_torque || !Wf || !Wt || !Wn || !q_next || !theta_next || N < 1 ||
        N >= kMaxN || !valid_bodies(body_offsets, n_bodies, N) || !(kT >= 0.0) || !std::isfinite(kT) ||
        !finite_pos(dt) || !finite_pos(delta) || !finite_pos(a) || !finite_pos(eta) || !valid_cell(Lx, Ly) ||
        !finite_pos(tol) || max_iter < 1 || max_iter > 100000 || !valid_prec(precision))
        return RPYW_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Scratch s;
    int rc = acquire(ws, ws_bytes, ts_ws_bytes(N, max_iter, n_bodies, precision), st, s);
    if (rc != RPYW_OK) return rc;
    int it[4] = {0, 0, 0, 0};
    rc = emrfd_step(q, theta, ref, body_offsets, n_bodies, N, Lp, force_torque, Wf, Wt, Wn, kT, dt, delta, a, eta,
                    Domain{Lx, Ly}, tol, max_iter, precision, q_next, theta_next, s.ar, it, st);
    if (iters_out)
        for (int k = 0; k < 4; ++k) iters_out[k] = it[k];
    return rc;
}

int rpy_wall_matvec_vjp(const double* pos, const double* force, const double* grad_vel, double* grad_pos,
                        double* grad_force, int64_t N, double a, double eta, int precision, void* ws,
                        size_t ws_bytes, void* stream) {
    if (!pos || !force || !grad_vel || (!grad_pos && !grad_force) || N < 1 || N >= kMaxN || !finite_pos(a) ||
        !finite_pos(eta) || !valid_prec(precision))
        return RPYW_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Scratch s;
    int rc = acquire(ws, ws_bytes, vjp_ws_bytes(N, precision), st, s);
    if (rc == RPYW_OK) rc = vjp(pos, force, grad_vel, grad_pos, grad_force, N, a, eta, precision, s.ar, st);
    if (log_enabled()) log_shape("rpy_wall_matvec_vjp", N, 1, precision, rc);
    return rc;
}

int rpy_wall_divergence(const double* pos, double* div, int64_t N, double a, double eta, int precision, void* ws,
                        size_t ws_bytes, void* stream) {
    if (!pos || !div || N < 1 || N >= kMaxN || !finite_pos(a) || !finite_pos(eta) || !valid_prec(precision))
        return RPYW_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Scratch s;
    int rc = acquire(ws, ws_bytes, vjp_ws_bytes(N, precision), st, s);
    if (rc == RPYW_OK) rc = divergence(pos, div, N, a, eta, precision, s.ar, st);
    log_line("rpy_wall_divergence N=%lld prec=%d status=%d", (long long)N, precision, rc);
    return rc;
}

int rpy_wall_autotune(const double* pos, const double* F, double* U, int64_t N, int32_t k, double a, double eta,
                      int precision, void* ws, size_t ws_bytes, void* stream) {
    if (!pos || !F || !U || N < 1 || N >= kMaxN || k < 1 || k > 4096 || !finite_pos(a) || !finite_pos(eta) ||
        !valid_prec(precision))
        return RPYW_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int kc = kclass(k);
    Scratch s;
    int rc = acquire(ws, ws_bytes, product_ws_bytes(N, precision, std::min(kc, 16)), st, s);
    if (rc != RPYW_OK) return rc;
    hipEvent_t e0, e1;
    RPYW_HIP(hipEventCreate(&e0));
    RPYW_HIP(hipEventCreate(&e1));
    const bool prof = g_prof;
    g_prof = false;
    // Candidates in order of preference (least partial-sum traffic first):
    // symmetric over groups of 256 with ipw 4, 2, 1, then (small problems)
    // over groups of 64 with ipw 4, 2, 1, then (FP32C blocks of 8 or more)
    // the matrix-core kernel, then plain (tpl, tile) in {1,2} x {64,256},
    // for every RHS block width.  Two timed rounds over all candidates (the
    // first also brings the clocks up); each candidate keeps its faster
    // round.  A later candidate must be faster by 1.5% to win, so near-ties
    // resolve the same way every time.
    std::vector<Shape> cands;
    for (int kb = 1; kb <= std::min(kc, 16); kb <<= 1) {
        for (int cand = 0; cand < 10; ++cand) {
            Shape sh{1, 256, kb, cand < 3 ? 1 : 2, 4 >> (cand % 3)};
            if (cand >= 6) sh = Shape{1 + ((cand - 6) & 1), ((cand - 6) & 2) ? 256 : 64, kb, 0, 4};
            if (cand >= 6 && kb >= 8 && sh.tpl == 2) continue;
            if (cand < 6 && kb > 4) continue;
            if (sh.sym == 2 && N > kSym64MaxN) continue;
            if (cand == 6 && kb >= 8) {
                Shape m{1, 64, kb, 0, 4};
                m.mat = 1;
                cands.push_back(m);
            }
            if (precision == RPYW_FP64 && kb > 8) continue;  // the vector units take FP64 blocks of up to 8
            cands.push_back(sh);
        }
    }
    std::vector<double> tbest(cands.size(), 1e300);
    for (int round = 0; round < 2; ++round) {
        for (size_t c = 0; c < cands.size(); ++c) {
            float ms = 0.f;
            for (int rep = 0; rep < 3; ++rep) {
                if (rep == 1) RPYW_HIP(hipEventRecord(e0, st));
                for (int k0 = 0; k0 < k; k0 += cands[c].kblk) {
                    const int n = std::min(cands[c].kblk, k - k0);
                    rc = product_pass(pos, F + (size_t)k0 * N * 3, U + (size_t)k0 * N * 3, N, n, a, eta, precision,
                                      cands[c], s.ar, st);
                    if (rc != RPYW_OK) {
                        g_prof = prof;
                        return rc;
                    }
                }
            }
            RPYW_HIP(hipEventRecord(e1, st));
            RPYW_HIP(hipEventSynchronize(e1));
            RPYW_HIP(hipEventElapsedTime(&ms, e0, e1));
            tbest[c] = std::min(tbest[c], (double)ms);
        }
    }
    Shape best = default_shape(N, k, precision);
    double best_t = 1e300;
    for (size_t c = 0; c < cands.size(); ++c)
        if (tbest[c] < 0.985 * best_t) {
            best_t = tbest[c];
            best = cands[c];
        }
    g_prof = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_tuned_shape(N, k, precision, best);
    {
        std::lock_guard<std::mutex> lk(g_shape_mu);
        save_cache_locked();
    }
    log_line("rpy_wall_autotune N=%lld k=%d prec=%d -> tpl=%d tile=%d kblk=%d sym=%d ipw=%d mat=%d (%.4f ms)",
             (long long)N, k, precision, best.tpl, best.tile, best.kblk, best.sym, best.ipw, best.mat, best_t / 2.0);
    return RPYW_OK;
}

int rpy_wall_set_shape(int precision, int64_t N, int32_t k, int32_t tpl, int32_t tile, int32_t kblk, int32_t sym,
                       int32_t ipw, int32_t mat) {
    if (tpl == 0 && valid_prec(precision) && N >= 1 && N < kMaxN && k >= 1) {
        clear_shape_override(N, k, precision);
        return RPYW_OK;
    }
    if (!valid_prec(precision) || N < 1 || N >= kMaxN || k < 1 || (tpl != 1 && tpl != 2) ||
        (tile != 64 && tile != 256) || kblk < 1 || kblk > (precision == RPYW_FP32C || mat ? 16 : 8) ||
        (kblk & (kblk - 1)) != 0 || sym < 0 || sym > 2 || (sym && kblk > 4) || ipw < 1 || mat < 0 || mat > 1 ||
        (mat && kblk < 8))
        return RPYW_EINVAL;
    Shape sh{tpl, tile, kblk, sym, ipw};
    sh.mat = mat;
    set_shape_override(N, k, precision, sh);
    return RPYW_OK;
}

int rpy_wall_get_shape(int precision, int64_t N, int32_t k, int32_t* out6) {
    if (!valid_prec(precision) || N < 1 || N >= kMaxN || k < 1 || !out6) return RPYW_EINVAL;
    Shape s = tuned_shape(N, k, precision);
    const int K = std::min(kclass(s.kblk), precision == RPYW_FP32C || s.mat ? 16 : 8);
    if (K >= 8) s.tpl = 1;
    if (K > 4) s.sym = 0;
    if (K < 8) s.mat = 0;
    out6[0] = s.tpl;
    out6[1] = s.tile;
    out6[2] = s.kblk;
    out6[3] = s.sym;
    out6[4] = s.ipw;
    out6[5] = s.mat;
    return RPYW_OK;
}

int rpyw_tridiag_sqrt_coeffs(const double* alpha, const double* beta, int32_t k, double beta0, double* c_out) {
    if (!alpha || !c_out || k < 1 || (k > 1 && !beta) || !std::isfinite(beta0)) return RPYW_EINVAL;
    for (int i = 0; i < k; ++i)
        if (!std::isfinite(alpha[i]) || (i + 1 < k && !std::isfinite(beta[i]))) return RPYW_EINVAL;
    return tridiag_sqrt_coeffs(alpha, beta, k, beta0, c_out);
}

int rpy_wall_profile_enable(int enable) {
    g_prof = enable != 0;
    return RPYW_OK;
}

int rpy_wall_profile_read(double* ms_total, int64_t* launches, double* pair_interactions, int reset) {
    for (auto& r : g_prof_recs) {
        float ms = 0.f;
        RPYW_HIP(hipEventSynchronize(r.b));
        RPYW_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        g_prof_ms += ms;
        g_prof_pairs += r.pairs;
        g_prof_n += 1;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof_recs.clear();
    if (ms_total) *ms_total = g_prof_ms;
    if (launches) *launches = g_prof_n;
    if (pair_interactions) *pair_interactions = g_prof_pairs;
    if (reset) {
        g_prof_ms = 0.0;
        g_prof_pairs = 0.0;
        g_prof_n = 0;
    }
    return RPYW_OK;
}

}  // extern "C"
