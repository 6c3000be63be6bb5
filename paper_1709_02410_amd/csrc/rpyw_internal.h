// Host-side internals shared by the translation units of librpywall.so.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rpywall.h"

namespace rpyw {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kMaxBodyBlobs = 42;    // largest body the preconditioner takes
constexpr size_t kAlign = 256;

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// Launch shape of the pair kernels.
struct Shape {
    int tpl;   // targets per lane: 1 or 2
    int tile;  // sources per LDS tile: 64 or 256
    int kblk;  // right-hand sides per pass: 1, 2, 4, 8 or 16
    int sym;   // symmetric pair evaluation (kblk <= 4): 0 off, 1 groups of 256 blobs, 2 groups of 64
    int ipw;   // symmetric path: source groups per workgroup
    int mat = 0;  // FP32C blocks of 8 or 16 right-hand sides: contraction on the matrix cores
};

// Domain along the wall: open (lx = ly = 0) or the pseudo-periodic cell
// lx x ly (physical units): every source at its minimum image plus the 8
// periodic images around it.
struct Domain {
    double lx = 0.0, ly = 0.0;
    bool periodic() const { return lx > 0.0; }
};

// Symmetric path geometry for N blobs, K right-hand sides.
struct SymPlan {
    int G;     // blobs per group: 256 or 64
    int ns;    // waves per item that split its passes (1, or 4 for groups of 64 when items are few)
    int nseg;  // workgroups per item that split its passes (1, 2 or 4: more workgroups for tiny problems)
    int ng, Hmax, C;
    size_t rec_bytes, tpart_bytes, spart_bytes;
    bool ok;
};
// Groups of 64 are for problems up to this size: their source partials grow
// as N^2 / 128 per quantity, four times those of groups of 256, and beyond
// a few ten thousand blobs both group sizes run at the same speed.
constexpr int64_t kSym64MaxN = 32768;
// Work items (group pairs) below which the symmetric passes are split into
// segments.
constexpr int64_t kSymItemsMin = 8192;
// Largest partial-sum array (source or target side) the symmetric path
// takes.  The partials grow as N^2 / G (3 N^2 / 512 values per side for one
// right-hand side and groups of 256), so this admits the symmetric kernel
// up to about 6e5 blobs in FP64 and 8.5e5 in FP32 (the "hundreds of
// thousands of blobs" up to which the paper finds direct products
// competitive); beyond it products use the plain kernel, whose workspace
// grows as N.
constexpr size_t kSymPartialMaxBytes = (size_t)16 << 30;
SymPlan sym_plan(int64_t N, int prec, int K, int ipw, int G = 256);
inline int sym_group(int sym) { return sym == 2 ? 64 : 256; }
// The three stages of a symmetric product pass, for callers that keep the
// records between passes (the Krylov solvers):
//   sym_pack   records (positions, wrapped into the cell when periodic, and
//              B f for kb right-hand sides; padded records are force-free
//              blobs far away) and B, for ng G blobs;
//   sym_launch the pair kernel over the records into the partial sums (with
//              ps, groups of 64 only: the kernel forms the records from
//              positions and right-hand sides itself; rec is unused);
//   sym_finish U = mu0 B (sum of the partials), fixed order (B null: B from
//              the positions, pos and 1 / a given).
int sym_pack(const double* pos, const double* F, int64_t N, int kb, int K, int prec, const SymPlan& sp, double a,
             const Domain& dom, void* rec, double* B, hipStream_t st);
struct PackSrc;
int sym_launch(const void* rec, const SymPlan& sp, int ipw, int K, int prec, double a, const Domain& dom,
               double* tpart, void* spart, hipStream_t st, const PackSrc* ps = nullptr);
int sym_finish(const double* tpart, const void* spart, const double* B, int64_t N, int kb, int K, int prec,
               const SymPlan& sp, double mu0, double* U, hipStream_t st, const double* pos = nullptr,
               double inv_a = 1.0);

// Bump allocator over a caller workspace.
struct Arena {
    char* base;
    size_t size;
    size_t used;
    void* take(size_t bytes) {
        size_t off = align_up(used);
        if (off + bytes > size) return nullptr;
        used = off + bytes;
        return base + off;
    }
};

// Record width (elements of the kernel precision) of one preprocessed blob.
inline int rec_width(int prec, int kblk) {
    if (prec == RPYW_FP32C) return (5 + 3 * kblk + 3) / 4 * 4;
    return (3 + 3 * kblk + 1) / 2 * 2;
}
inline size_t real_size(int prec) { return prec == RPYW_FP32C ? 4 : 8; }

// Number of source splits of the plain product and the chunk length.
void split_plan(int64_t N, int tpl, int* splits, int64_t* chunk);

// Workspace bytes of one product pass of width kblk (upper bound over the
// shapes the tuner may pick).
size_t product_ws_bytes(int64_t N, int prec, int kblk);

// u-block products: U[k0..k0+kb) = M F[k0..k0+kb); kb <= shape.kblk.
// pre: preprocessed records already hold positions; forces are (re)packed.
int product_pass(const double* pos, const double* F, double* U, int64_t N, int kb, double a, double eta, int prec,
                 Shape shape, Arena& ar, hipStream_t st);

// Full multi-RHS product with the tuned or default shape; in a periodic
// domain one right-hand side at a time through the symmetric kernel.
int products(const double* pos, const double* F, double* U, int64_t N, int k, double a, double eta, int prec,
             Arena& ar, hipStream_t st, const Domain& dom = Domain{});

// Batched independent systems (persistent kernel, LPT work list).
size_t batched_ws_bytes(int64_t Ntot, int S, int k, int prec);
int batched_products(const double* pos, const int64_t* sys_offsets, int S, const double* F, double* U, int k,
                     double a, double eta, int prec, Arena& ar, hipStream_t st);

// Shape selection.
Shape default_shape(int64_t N, int k, int prec);
// The launch shape products of N blobs and k right-hand sides use: the one
// fixed by rpy_wall_set_shape for this (precision, size class, RHS class) if
// any, else the tuned one, else the built-in default; then the RPYW_TILE /
// RPYW_RHS_WIDTH overrides.
Shape tuned_shape(int64_t N, int k, int prec);
void set_tuned_shape(int64_t N, int k, int prec, Shape s);
void set_shape_override(int64_t N, int k, int prec, Shape s);
void clear_shape_override(int64_t N, int k, int prec);

// Run-time settings (settings.hip): RPYW_LOG, RPYW_TILE, RPYW_RHS_WIDTH and
// the persisted shape cache RPYW_AUTOTUNE_CACHE.
struct CachedShape {
    std::string arch;
    int prec = 0, size_class = 0, kclass = 0;
    Shape s{};
};
bool log_enabled();
void log_line(const char* fmt, ...);
Shape apply_env_overrides(Shape s);
// RPYW_SYM_SPLIT: the split of item passes of the symmetric kernel with
// groups of 64 (false when not set).
bool sym_split_override(int* ns, int* nseg);
const char* autotune_cache_path();
std::string device_arch();
int read_shape_cache(const char* path, std::vector<CachedShape>& out);
int write_shape_cache(const char* path, const std::vector<CachedShape>& entries);

// Instrumentation around the O(N^2) launches.
bool profiling_enabled();
void profile_begin(hipStream_t st, hipEvent_t* ev);
void profile_end(hipStream_t st, hipEvent_t ev0, double pairs);

// v[e] - sum_{j < nc} c[j] V[j ld + e], the terms subtracted in order.
__device__ __forceinline__ double minus_comb(const double* __restrict__ v, const double* __restrict__ V, int64_t ld,
                                             const double* __restrict__ c, int nc, int64_t e) {
    double x = v[e];
    int j = 0;
    for (; j + 7 < nc; j += 8) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = V[(j + u) * ld + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) x -= c[j + u] * a[u];
    }
    for (; j < nc; ++j) x -= c[j] * V[j * ld + e];
    return x;
}

// Fused Lanczos steps (lanczos_step.hip): four launches per step when the
// product runs through the symmetric kernel and max_iter is at most
// kLanczosFusedMaxIter (the coefficient vectors live in LDS).
constexpr int kLanczosFusedMaxIter = 512;
constexpr int kLanczosGs2PerThread = 8;
constexpr int kLanczosOutEntries = 64;  // entries per workgroup of the gather (larger bodies alone)
// A gather group: units [g0, g1) (bodies, or runs of blobs), blobs [b0, b1),
// the offset loff of the first unit's factor block (L_p then L_p^-1 at
// 2 loff) and sq = sum of n_p^2 over its units (entries of each factor).
struct LanczosGroup {
    int g0, g1, b0, b1;
    int64_t loff;
    int sq, pad;
};
constexpr int kLanczosGroupUnits = kLanczosOutEntries / 3 + 1;  // units of a group, at most
struct BodyFactors;
bool lanczos_fused_applies(int64_t N, int prec, int max_iter, const Domain& dom, SymPlan* sp, int* ipw);
int64_t lanczos_gs2_blocks(int64_t n3, int* m);
void lanczos_units(int64_t N, const int64_t* body_offsets, int n_bodies, std::vector<int>& units,
                   std::vector<int>& groups);
// vin of step k; at k = 0, part2 holds the packing kernel's partials of
// |W|^2 and vin writes the header (beta_0, then the two definiteness flags
// *bad0 and *bad1 (0 when null) as ints) to the pinned h_hdr.
int lz_launch_vin(int prec, const BodyFactors& pc, const int* units, int nunits, int64_t n3, int k,
                  const double* src, const double* part2, int ncol2, double* V, double* d_ab, double* h_ab,
                  double* h_flag, void* rec, int recw, const double* B, double* h_hdr, const int* bad0,
                  const int* bad1, hipStream_t st);
// Records, B and the |W|^2 partials (lz_pack_blocks of them) for npad
// blobs; clears *bad.
// Also copies the call's tables (nwords ints) from pinned host memory htab
// (the device's address of it) to the device block dtab.
int64_t lz_pack_blocks(int64_t npad);
int lz_launch_pack(int prec, const double* pos, const double* W, int64_t N, int64_t npad, int recw, double a,
                   const Domain& dom, void* rec, double* B, double* sqp, int* bad, const int* htab, int* dtab,
                   int nwords, hipStream_t st);
// out = L (V c) for nv <= kLanczosCoefArgs coefficients (passed by value).
constexpr int kLanczosCoefArgs = 448;
int lz_launch_fin(const BodyFactors& pc, const int* units, int nunits, int64_t n3, const double* V, const double* c,
                  int nv, double* out, hipStream_t st);
// ypre: when given, the product mu0 B_i sum(partials) already summed by the
// symmetric epilogue ([N][3]); the kernel then reads it instead of gathering
// the partials of its own entries (which is latency-bound but uncoalesced:
// the better choice for small problems only).
int lz_launch_out(int prec, const BodyFactors& pc, const int* units, const LanczosGroup* ginfo, int ngroups,
                  const double* tpart, const void* spart, const SymPlan& sp, const double* B, double mu0, int64_t n3,
                  int k, const double* V, const double* d_ab, double* w, double* part1, const double* ypre,
                  hipStream_t st);
int lz_launch_gs2(const double* w, double* yo, int64_t n3, const double* V, int k, const double* part1, int ngroups,
                  double* part2, double* d_ab, double* gc1, hipStream_t st);

// Fused GMRES steps of the rigid solve (rigid_step.hip), with the Lanczos
// gs2 kernel (gc1: where its block 0 keeps c1 for the next pre).
// pre publishes column k - 1 of the Hessenberg matrix into the pinned
// slot hslots + ((k - 1) mod PinnedSlots::kSlots) slot and sets h_flag[k - 1].
// At k = 0, part2 holds the right-hand side kernel's partials of |b|^2 and
// pre writes the header (|b|, then the flags *bad0 and *bad1 (0 when null)
// as ints) to the pinned h_hdr.
int rg_launch_pre(int prec, const BodyFactors& pc, const double* Wall, const double* Nall, int n_bodies, int64_t n3,
                  int64_t ld, const double* src, const double* part2, int ncol2, const double* gc1, double* hslots,
                  int slot, double* h_flag, int k, double* V, double* zl, double* zu, void* rec, int recw,
                  const double* B, double* h_hdr, const int* bad0, const int* bad1, hipStream_t st);
// b = [-slip | -F, -T] (n3 + n6 entries), the partials of |b|^2
// (rg_rhs_blocks of them), the records' positions (zero force slots) and B
// for npad blobs, the tables (nwords ints) from pinned host memory htab to
// dtab; clears *bad.
// x = P^-1 (V y) into lam_out (3N) and U_out (6 n_bodies), for nv <=
// kLanczosCoefArgs coefficients y (passed by value); V_j at V + j ld.
int rg_launch_fin(const BodyFactors& pc, const double* Wall, const double* Nall, int n_bodies, int64_t n3, int64_t ld,
                  const double* V, const double* y, int nv, double* lam_out, double* U_out, hipStream_t st);
int64_t rg_rhs_blocks(int64_t n);
int rg_launch_rhs(int prec, const double* pos, int64_t N, int64_t npad, int recw, double a, const Domain& dom,
                  void* rec, double* B, const double* slip, const double* FT, int64_t n3, int64_t n6, double* b,
                  double* sqp, int* bad, const int* htab, int* dtab, int nwords, hipStream_t st);
// ypre: as for lz_launch_out.
int rg_launch_out(int prec, const double* pos, const double* q, const int* bofs, int n_bodies, const double* tpart,
                  const void* spart, const SymPlan& sp, const double* B, double mu0, const double* zl,
                  const double* zu, int64_t n3, int64_t ld, const double* V, int k, double* w, double* part1,
                  const double* ypre, hipStream_t st);

// Whether the fused Krylov steps sum the product's partials with the
// symmetric epilogue first (groups of 256 blobs: large problems).
inline bool krylov_presum(const SymPlan& sp) { return sp.G == 256; }

// Krylov building blocks (krylov.hip).
// Block-diagonal preconditioner factors: per body the Cholesky factor L_p of
// its own block M^(pp) (other bodies ignored, wall kept) and L_p^-1; with no
// body structure, the per-blob diagonal square root.
struct BodyFactors {
    bool diag = true;
    int nb = 0;
    int* bofs = nullptr;      // device [nb + 1] blob offsets
    int64_t* lofs = nullptr;  // device [nb + 1] offsets of the (3 n_p)^2 blocks
    double* L = nullptr;      // per body L_p then L_p^-1 (at 2 lofs[p]); or the diagonal [3N]
    int* flag = nullptr;      // device int set by the build when a block is not positive definite
    // mode 0: out = L v; 1: out = L^-1 v; 2: out = L^-T v.  With nc > 0 the
    // input is first v - sum_{j < nc} c[j] V_j (V_j at V + j n3, the terms
    // subtracted in order); with scale it is then divided by scale[0] and,
    // with store, written there too.
    int apply(int mode, const double* v, double* out, int64_t n3, hipStream_t st, const double* scale = nullptr,
              double* store = nullptr, const double* V = nullptr, const double* c = nullptr, int nc = 0) const;
};
size_t body_factors_bytes(int64_t N, int n_bodies);
// Builds the factors on the stream; sets *notspd (device int, zeroed by the
// caller) when a block is not positive definite.  body_offsets: host.
int body_factors_build(const double* pos, int64_t N, double a, double eta, const int64_t* body_offsets, int n_bodies,
                       Arena& ar, hipStream_t st, BodyFactors& pc, int* notspd);
// The two steps of body_factors_build for callers that place the tables
// themselves: the host tables (blob offsets hb, factor offsets hl = prefix
// sums of (3 n_p)^2, the largest body nmax), then the build launch for pc
// with bofs, lofs and L (2 hl[nb] doubles; 3N for no bodies) set and the
// tables on the device when the launch runs.
void body_factors_tables(const int64_t* body_offsets, int n_bodies, std::vector<int>& hb, std::vector<int64_t>& hl,
                         int* nmax);
int body_factors_launch(const double* pos, int64_t N, double a, double eta, const BodyFactors& pc, int nmax,
                        int* notspd, hipStream_t st);
// Small host tables gathered into one block: add() returns each part's
// byte offset (parts 256-byte aligned).
struct TableBlock {
    std::vector<char> host;
    size_t add(const void* src, size_t bytes) {
        const size_t o = align_up(host.size());
        host.resize(o + bytes);
        if (bytes) std::memcpy(host.data() + o, src, bytes);
        return o;
    }
};
// Vector kernels (FP64, length n, basis vectors V_j at V + j ld):
//   dots:   out[j] = V_j . w (j < nv), or out[0] = |w| when nv == 0, with a
//           fixed-order finish; out[copy_idx] is also copied to copy_to;
//           partial holds max(nv, 1) (nv + 1 with_norm) dot_chunks(n) doubles, ticket one
//           zeroed unsigned that the kernel re-arms;
//   update_dots: the update w = win - bscale[0] vprev - sum_{j < nsub}
//           csub[j] V_j (terms when given; written to wout when there is
//           one) then the dots of w, in one pass; with nh > 0 the
//           kernel's finishing block then copies hsrc[0..nh) (device
//           memory, which may include this pass's out) to hdst (the device
//           alias of pinned host memory), so the host reads the results
//           after an event without a separate copy; with_norm (nv > 0)
//           also puts |w|^2 in out[nv] and, with beta_out, writes
//           sqrt(|w|^2 - sum_j out[j]^2) there: the norm of w - V out when
//           the V_j are orthonormal (before the results are copied; copy_to
//           then receives this value instead of out[copy_idx]);
//   comb:   out = sum_{j < nv} c[j] V_j.
// Asynchronous upload of a small host array (which the caller may free at
// once) through a library-owned pinned ring.
int stage_upload(const void* src, size_t bytes, void* dst, hipStream_t st);
int64_t dot_chunks(int64_t n);
int vec_dots(const double* V, int64_t ld, int nv, const double* w, int64_t n, double* partial, unsigned* ticket,
             double* out, int copy_idx, double* copy_to, hipStream_t st);
int vec_update_dots(const double* win, double* wout, int64_t n, const double* vprev, const double* bscale,
                    const double* V, int64_t ld, const double* csub, int nsub, int nv, double* partial,
                    unsigned* ticket, double* out, int copy_idx, double* copy_to, hipStream_t st,
                    double* hdst = nullptr, const double* hsrc = nullptr, int nh = 0, bool with_norm = false,
                    double* beta_out = nullptr);
int vec_comb(const double* V, int64_t ld, int nv, const double* c, double* out, int64_t n, hipStream_t st);
// Krylov drivers keep kSpeculateDepth steps queued beyond the one the host
// examines (a step needs only device data from the previous one), so the GPU
// does not wait for the host between steps, but only while one product is
// cheap against the host's per-step latency (about 0.1 ms): above this many
// pairs the speculative steps, wasted after the last iteration, cost more
// than they hide, and step k + 1 is queued after the host has examined k.
constexpr double kSpeculatePairs = 4.0e8;
constexpr int kSpeculateDepth = 2;
// Highest step index to have queued while the host examines step k, with at
// most `depth` steps beyond k, and none beyond the step at which a geometric
// extrapolation of the last two convergence measures m1 (step k - 1) and m2
// (step k - 2) reaches tol (so that few queued steps are wasted).
inline int speculate_to(int k, int depth, double m1, double m2, double tol) {
    if (depth <= 0) return k;
    int need = 1 << 20;  // steps after k - 1 until convergence
    if (m1 > tol && m2 > m1 && m1 > 0.0)
        need = std::max(1, (int)std::ceil(std::log(tol / m1) / std::log(m1 / m2)));
    return std::max(k, std::min(k + depth, k - 1 + need));
}

// Library-owned pinned host buffer plus two events for per-iteration
// device->host copies of a solver; the caller holds mu while using it.
// Two banks used by alternate calls, so that a call does not wait for the
// copies (possibly of speculative steps still queued) of the one before.
struct PinnedSlots {
    static constexpr int kSlots = 4;  // steps in flight at most (kSpeculateDepth + 1)
    struct Bank {
        double* p = nullptr;   // host address
        double* dp = nullptr;  // the same memory as kernels address it
        size_t cap = 0;
        hipEvent_t ev[kSlots] = {};
        hipEvent_t tail = nullptr;  // after the last copy into p of the call that used it
    };
    std::mutex mu;
    Bank bank[2];
    int cur = 0;
    double* p = nullptr;     // the current call's bank
    double* dp = nullptr;    // its device alias (kernels write results there)
    hipEvent_t* ev = nullptr;
    // Switches bank, waits for the copies of the call that last used it, then
    // makes p hold bytes.
    int reserve(size_t bytes);
    // Marks the end of this call's copies (the solvers return without
    // waiting for the speculative steps still queued).
    int release(hipStream_t st);
};
// Calls release on every return path of a solver holding the slots.
struct SlotRelease {
    PinnedSlots& s;
    hipStream_t st;
    ~SlotRelease() { (void)s.release(st); }
};

// Lanczos (lanczos.hip)
size_t lanczos_ws_bytes(int64_t N, int max_iter, int n_bodies, int prec);
// pre: factors already built for these positions and bodies (then not rebuilt).
int lanczos_sqrt(const double* pos, const double* W, double* out, int64_t N, double a, double eta,
                 const int64_t* body_offsets, int n_bodies, double tol, int max_iter, int prec, Arena& ar,
                 int* iters, double* err, hipStream_t st, const Domain& dom = Domain{},
                 const BodyFactors* pre = nullptr);
int tridiag_sqrt_coeffs(const double* alpha, const double* beta, int k, double beta0, double* c);

// Rigid multiblobs (rigid.hip)
size_t rigid_ws_bytes(int64_t N, int max_iter, int n_bodies, int prec);
int rigid_solve(const double* pos, const double* q, const int64_t* body_offsets, int n_bodies, const double* slip,
                const double* FT, double* lam_out, double* U_out, int64_t N, double a, double eta, double tol,
                int max_iter, int prec, Arena& ar, int* iters, double* res_out, hipStream_t st,
                const Domain& dom = Domain{}, const BodyFactors* pre = nullptr);

// Body kinematics and the Trapezoidal Slip step (ts.hip)
int body_blobs(const double* q, const double* theta, const double* ref, const int* bofs_dev, int nb, double* pos,
               hipStream_t st);
int body_move(const double* q, const double* theta, const double* U, const double* U2, double h, int nb,
              double* q_out, double* theta_out, hipStream_t st);
size_t ts_state_bytes(int64_t N, int nb);
size_t ts_ws_bytes(int64_t N, int max_iter, int nb, int prec);
int ts_predict(const double* q, const double* theta, const double* ref, const int64_t* body_offsets, int nb,
               int64_t N, const double* Lp, const double* FT, const double* Ws, const double* Wn, double kT,
               double dt, double delta, double a, double eta, const Domain& dom, double tol, int max_iter, int prec,
               double* q_t, double* theta_t, double* pos_t, double* state, Arena& ar, int* iters, hipStream_t st);
int ts_correct(const double* q, const double* theta, const double* q_t, const double* theta_t, const double* ref,
               const int64_t* body_offsets, int nb, int64_t N, const double* FT_t, const double* state, double dt,
               double a, double eta, const Domain& dom, double tol, int max_iter, int prec, double* q_next,
               double* theta_next, Arena& ar, int* iters, hipStream_t st);

int emt_step(const double* q, const double* theta, const double* ref, const int64_t* body_offsets, int nb, int64_t N,
             const double* Lp, const double* FT, const double* Wf, const double* Wt, const double* Wn, double kT,
             double dt, double delta, double a, double eta, const Domain& dom, double tol, int max_iter, int prec,
             double* q_next, double* theta_next, Arena& ar, int* iters, hipStream_t st);

int emrfd_step(const double* q, const double* theta, const double* ref, const int64_t* body_offsets, int nb,
               int64_t N, const double* Lp, const double* FT, const double* Wf, const double* Wt, const double* Wn,
               double kT, double dt, double delta, double a, double eta, const Domain& dom, double tol, int max_iter,
               int prec, double* q_next, double* theta_next, Arena& ar, int* iters, hipStream_t st);

// Derivatives (vjp.hip)
size_t vjp_ws_bytes(int64_t N, int prec);
int vjp(const double* pos, const double* f, const double* g, double* grad_pos, double* grad_f, int64_t N, double a,
        double eta, int prec, Arena& ar, hipStream_t st);
int divergence(const double* pos, double* div, int64_t N, double a, double eta, int prec, Arena& ar,
               hipStream_t st);

#define RPYW_HIP(call)                          \
    do {                                        \
        hipError_t e_ = (call);                 \
        if (e_ != hipSuccess) return RPYW_EHIP; \
    } while (0)

}  // namespace rpyw
