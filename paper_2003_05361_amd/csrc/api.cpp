// C ABI of the restricted additive Schwarz solver: setup (host plan + upload),
// solve (work tables, persistent launch, verification / resume), queries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <queue>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/ras.h"
#include "device.hpp"
#include "plan.hpp"

namespace ras {
// kernels.hip
const void* select_kernel(int solver, int storage, bool async, int ell_width, int rclass);
int cg_rows_class(int rows_per_member);
hipError_t launch_solver(const void* kern, int solver, const Params& P, const int* band_args, size_t lds,
                         hipStream_t st, bool coop);
hipError_t occupancy(const void* kern, int solver, size_t lds, int* per_cu);
hipError_t launch_residual(int64_t n, const int64_t* rp, const int32_t* ci, const double* va, const double* b,
                           const double* x, double* parts, int nparts, double* out, hipStream_t st);
hipError_t launch_copy(int64_t n, const double* src, double* dst, hipStream_t st);
hipError_t launch_stamp(InstState* ist, int n, hipStream_t st);
hipError_t noalloc_scratch(void** ptr);
hipError_t launch_band_factor(const FactorJob* jobs, int njobs, int storage, int max_n, hipStream_t st);
}  // namespace ras

using namespace ras;

namespace {

thread_local std::string g_err;

ras_status fail(ras_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) throw Error{RAS_E_HIP, std::string(what) + ": " + hipGetErrorString(e)};
}

// Owning device allocation.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { reset(); }
    void reset() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t n) {
        reset();
        if (n == 0) return;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            throw Error{RAS_E_NOMEM, "hipMalloc(" + std::to_string(n) + " bytes) failed: " + hipGetErrorString(e)};
        }
        bytes = n;
    }
    void ensure(size_t n) {
        if (bytes < n) alloc(n);
    }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

size_t ct_size(int storage) { return storage == RAS_STORAGE_FP64 ? 8 : 4; }

int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

struct ras_plan : public Plan {};

namespace {
// Shape key -> best CG team size found by ras_autotune (process-wide).
std::mutex g_tune_mu;
std::map<std::tuple<int64_t, int32_t, int32_t, int32_t, int32_t, int32_t>, int> g_tune;
}  // namespace

struct ras_handle {
    std::unique_ptr<ras_plan> plan;  // host plan (factors dropped after upload)
    hipStream_t stream = nullptr;
    int device = 0;
    int64_t clock_khz = 0;
    int num_cu = 0;
    int solver = 0, storage = 0, cg_iters = 0;
    int max_n = 0, max_w = 0, max_K = 0, uniform_K = 0;
    int max_w_rowmajor = -1;  // widest band kept row-major (w > kSlabMaxW), -1 if none
    bool any_slab = false;
    bool sparse = false;      // sparse Cholesky solver: device local order = elimination order
    int64_t max_sparse_values = 0;  // sparse Cholesky: largest vector plus block slots kept in LDS
    int64_t sum_n = 0;
    int64_t sum_snap = 0;  // sum over subdomains of n + n_ext (asynchronous snapshot size per right-hand side)
    ras_plan_stats stats{};
    DevBuf omega, ell_val, ell_valf, ell_gcol, ell_lcol, band_f, band_b, scale, invd, ext, sp_idx, sp_val;
    DevBuf csr_rp, csr_ci, csr_va, nbr;
    DevBuf tri_g;  // FP16 slab: packed float32 inverses of the block triangles (both passes)
    // host-written control words (cancel, per-subdomain pause), pinned and coherent so
    // that a running asynchronous kernel sees the host's writes
    struct Control {
        int32_t* host = nullptr;
        int32_t* dev = nullptr;
        ~Control() {
            if (host) (void)hipHostFree(host);
        }
    } ctl;
    std::vector<SubDev> subs;  // host copy with device pointers
    // CG team windows: for team size kTeamSizes[t], per subdomain and member the
    // LDS window [lo, hi) of local rows its rows reference
    std::vector<int32_t> win[5];
    int max_win[5] = {0, 0, 0, 0, 0};
    int tuned_team = 0;
    // last solve
    std::vector<std::vector<double>> hist, hist_t;
    std::vector<std::vector<int64_t>> counts;
    std::vector<std::vector<double>> phase_s;  // [rhs][P * 4] seconds per subdomain and phase
    DevBuf ws_red;  // reduction slots of ras_relative_residual
    // timing events of the solves on this handle, created once at setup
    struct Events {
        hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
        ~Events() {
            for (hipEvent_t& v : e)
                if (v) (void)hipEventDestroy(v);
        }
    } ev;
};

namespace {

template <class F>
ras_status guarded(F&& f) {
    try {
        return f();
    } catch (const Error& e) {
        return fail(e.status, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(RAS_E_NOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(RAS_E_ARG, e.what());
    }
}

// Status and message of the exception being handled, mapped as guarded() maps
// them; for the server's threads, where nothing may escape.
std::pair<ras_status, std::string> current_error() {
    try {
        throw;
    } catch (const Error& e) {
        return {e.status, e.msg};
    } catch (const std::bad_alloc&) {
        return {RAS_E_NOMEM, "host allocation failed"};
    } catch (const std::exception& e) {
        return {RAS_E_ARG, e.what()};
    } catch (...) {
        return {RAS_E_STATE, "unknown exception"};
    }
}

constexpr size_t kLdsLimit = 160 * 1024 - 4096;  // leave room for the kernels' static LDS

// host_factor: banded Cholesky factors computed here (plans that are queried on
// the host); otherwise upload() factors on the device
void build_plan(const ras_csr* A, const ras_partition* part, int32_t overlap, const ras_local* local, Plan& plan,
                bool host_factor = true) {
    if (!A || !part || !local) throw Error{RAS_E_ARG, "null argument"};
    if (overlap < 0) throw Error{RAS_E_ARG, "overlap must be >= 0"};
    if (local->kind != RAS_LOCAL_CHOL_BANDED && local->kind != RAS_LOCAL_CG && local->kind != RAS_LOCAL_CHOL_SPARSE)
        throw Error{RAS_E_ARG, "unknown local solver"};
    if (local->storage < RAS_STORAGE_FP64 || local->storage > RAS_STORAGE_FP16_ROWSCALED)
        throw Error{RAS_E_ARG, "unknown storage"};
    if (local->kind == RAS_LOCAL_CG && local->storage == RAS_STORAGE_FP16_ROWSCALED)
        throw Error{RAS_E_ARG, "FP16_ROWSCALED storage applies to the Cholesky factor only"};
    if (local->kind == RAS_LOCAL_CG && local->cg_iters < 1) throw Error{RAS_E_ARG, "cg_iters must be >= 1"};
    if (local->transmission != RAS_TRANSMISSION_DIRICHLET && local->transmission != RAS_TRANSMISSION_ROBIN)
        throw Error{RAS_E_ARG, "unknown transmission condition"};
    if (local->transmission == RAS_TRANSMISSION_ROBIN) {
        if (local->kind == RAS_LOCAL_CG)
            throw Error{RAS_E_ARG, "Robin transmission needs a direct local solver (CHOL_BANDED or CHOL_SPARSE)"};
        if (!(local->robin_q > 0.0 && local->robin_q <= 1.0)) throw Error{RAS_E_ARG, "robin_q must be in (0, 1]"};
    }
    validate_csr(*A);
    plan.n = A->n;
    plan.nnz = A->row_ptr[A->n];
    plan.overlap = overlap;
    plan.local = *local;
    plan.row_ptr.assign(A->row_ptr, A->row_ptr + A->n + 1);
    plan.col.assign(A->col, A->col + plan.nnz);
    plan.val.assign(A->val, A->val + plan.nnz);
    plan.owner = make_owner(*A, *part, &plan.P);
    build_overlap(plan);
    if (local->kind == RAS_LOCAL_CHOL_BANDED) {
        if (host_factor) {
            factor_local(plan);
        } else {
            // bands beyond the device factorisation's column buffer are factored here
            parallel_for(plan.P, [&](int64_t p, int) {
                if (plan.subs[p].w > kMaxFactorW) factor_one(plan, plan.subs[p], static_cast<int32_t>(p));
            });
        }
    }
    if (local->kind == RAS_LOCAL_CHOL_SPARSE) {
        if (local->storage == RAS_STORAGE_FP16_ROWSCALED)
            throw Error{RAS_E_ARG, "FP16_ROWSCALED storage applies to the banded Cholesky factor only"};
        const int64_t lim = ras_sparse_max_rows(local->storage);
        for (int32_t p = 0; p < plan.P; ++p)
            if (static_cast<int64_t>(plan.subs[p].omega.size()) > lim)
                throw Error{RAS_E_UNSUPPORTED, "subdomain " + std::to_string(p) + " has " +
                                                   std::to_string(plan.subs[p].omega.size()) +
                                                   " local rows; the sparse solver keeps at most " +
                                                   std::to_string(lim) + " in LDS"};
        sparse_factor_local(plan, kLdsLimit, local->storage == RAS_STORAGE_FP64 ? sizeof(double) : sizeof(float));
    }
}

void plan_stats(const Plan& plan, ras_plan_stats* o) {
    std::memset(o, 0, sizeof(*o));
    o->n = plan.n;
    o->nnz = plan.nnz;
    o->parts = plan.P;
    o->min_local_rows = INT64_MAX;
    for (const auto& s : plan.subs) {
        const int64_t n = static_cast<int64_t>(s.omega.size());
        o->max_ell_width = std::max(o->max_ell_width, s.ell_width);
        o->sum_local_rows += n;
        o->min_local_rows = std::min(o->min_local_rows, n);
        o->max_local_rows = std::max(o->max_local_rows, n);
        o->max_band = std::max(o->max_band, s.w);
        o->band_entries += plan.local.kind == RAS_LOCAL_CHOL_SPARSE ? static_cast<int64_t>(s.sf.lj.size()) + n
                                                                    : n * (s.w + 1);
    }
}

int64_t n_pad_of(int64_t n) { return (n + 63) / 64 * 64; }

// entries of one stored factor: slab layout (whole blocks of kBandRows rows,
// w entries per row) for w <= kSlabMaxW, else row-major [n][w + 1]
int64_t band_elems(int64_t n, int w) {
    if (w <= kSlabMaxW) return (n + kBandRows - 1) / kBandRows * kBandRows * w;
    return n * (w + 1);
}
constexpr int64_t kSlabTailBytes = 4096;

// Upload the plan: ELL rows of A on every overlapping set, local column map,
// factors in the storage type (forward L and reversed transpose) or the sparse
// solve schedules, global CSR.
// Banded Cholesky factors of the listed subdomains computed on the device
// (float64, in a temporary band buffer), then laid out in the storage type the
// solves read (band_f, band_b, invd, FP16 scales) by device kernels.
void device_factor(ras_handle& h, const Plan& plan, const std::vector<int>& ps) {
    const int st = plan.local.storage;
    std::vector<int64_t> loff(ps.size() + 1, 0);
    int max_n = 0;
    for (size_t k = 0; k < ps.size(); ++k) {
        const auto& s = plan.subs[ps[k]];
        loff[k + 1] = loff[k] + static_cast<int64_t>(s.omega.size()) * (s.w + 1);
        max_n = std::max<int>(max_n, static_cast<int>(s.omega.size()));
    }
    DevBuf L, jobs_d, fail_d;
    L.alloc(std::max<int64_t>(loff.back(), 1) * sizeof(double));
    fail_d.alloc(ps.size() * sizeof(int32_t));
    std::vector<FactorJob> jobs(ps.size());
    for (size_t k = 0; k < ps.size(); ++k) {
        const SubDev& d = h.subs[ps[k]];
        FactorJob& j = jobs[k];
        j.ell_val = d.ell_val;
        j.ell_lcol = d.ell_lcol;
        j.n = d.n;
        j.n_pad = d.n_pad;
        j.K = d.K;
        j.w = d.w;
        j.L = L.as<double>() + loff[k];
        j.fail = fail_d.as<int32_t>() + k;
        j.band_f = const_cast<void*>(d.band_f);
        j.band_b = const_cast<void*>(d.band_b);
        j.invd = const_cast<void*>(d.invd);
        j.scale = const_cast<float*>(d.scale);
        j.slab = d.slab;
        j.tri_inv = d.tri_inv;
        j.tri_g[0] = const_cast<float*>(d.tri_g[0]);
        j.tri_g[1] = const_cast<float*>(d.tri_g[1]);
        j.robin_shift = robin_shift_factor(plan.local);
    }
    jobs_d.alloc(jobs.size() * sizeof(FactorJob));
    hip_check(hipMemcpy(jobs_d.p, jobs.data(), jobs.size() * sizeof(FactorJob), hipMemcpyHostToDevice), "copy jobs");
    hip_check(launch_band_factor(jobs_d.as<FactorJob>(), static_cast<int>(jobs.size()), st, max_n, h.stream),
              "band factorisation");
    std::vector<int32_t> fail(ps.size());
    hip_check(hipMemcpyAsync(fail.data(), fail_d.p, ps.size() * sizeof(int32_t), hipMemcpyDeviceToHost, h.stream),
              "copy factor status");
    hip_check(hipStreamSynchronize(h.stream), "band factorisation");
    for (size_t k = 0; k < ps.size(); ++k)
        if (fail[k] >= 0)
            throw Error{RAS_E_NOT_SPD, "non-positive pivot in subdomain " + std::to_string(ps[k]) + " at local row " +
                                           std::to_string(fail[k])};
}

// Host form of the device's block inverses: the strictly lower part of the
// inverse of each 32-row block's diagonal triangle of L (rev: of its reversed
// transpose), float64 (FP32: from the float32-rounded triangle), written to the
// block's triangle slots of the slab layout.
void store_block_inverses(const double* L, int64_t n, int w, int st, bool rev, unsigned char* dst,
                          const uint16_t* Lh = nullptr, const float* scale = nullptr, float* gdst = nullptr) {
    constexpr int BR = kBandRows;
    const int64_t ld = w + 1;
    double T[BR][BR], G[BR][BR];
    for (int64_t t0 = 0, blk = 0; t0 < n; t0 += BR, ++blk) {
        for (int r = 0; r < BR; ++r)
            for (int c = 0; c < BR; ++c) {
                double v = r == c ? 1.0 : 0.0;
                if (c <= r && t0 + r < n) {
                    const int64_t i = rev ? n - 1 - t0 - c : t0 + r;
                    v = L[i * ld + (c - r + w)];
                    if (st == RAS_STORAGE_FP32) v = static_cast<double>(static_cast<float>(v));
                    if (st == RAS_STORAGE_FP16_ROWSCALED) {
                        _Float16 hv;
                        std::memcpy(&hv, &Lh[i * ld + (c - r + w)], 2);
                        v = static_cast<double>(static_cast<float>(hv) * scale[i]);
                    }
                }
                T[r][c] = v;
            }
        for (int m = 0; m < BR; ++m)
            for (int r = 0; r < BR; ++r) {
                if (r < m) {
                    G[r][m] = 0.0;
                    continue;
                }
                double s = r == m ? 1.0 : 0.0;
                for (int k = m; k < r; ++k) s -= T[r][k] * G[k][m];
                G[r][m] = s / T[r][r];
            }
        for (int r = 0; r < BR; ++r)
            for (int c = 0; c < r; ++c) {
                if (st == RAS_STORAGE_FP16_ROWSCALED) {
                    gdst[blk * kTriPackFloats + (r * (r - 1)) / 2 + c] = t0 + r < n ? static_cast<float>(G[r][c]) : 0.0f;
                    continue;
                }
                if (t0 + r >= n) continue;
                const int64_t di = (blk * w + (w - r + c)) * BR + r;
                if (st == RAS_STORAGE_FP64) reinterpret_cast<double*>(dst)[di] = G[r][c];
                else reinterpret_cast<float*>(dst)[di] = static_cast<float>(G[r][c]);
            }
    }
}

void upload(ras_handle& h, const Plan& plan) {
    const int P = plan.P;
    const bool sparse = plan.local.kind == RAS_LOCAL_CHOL_SPARSE;
    const bool chol = plan.local.kind == RAS_LOCAL_CHOL_BANDED;
    h.sparse = sparse;
    const int st = plan.local.storage;
    h.solver = plan.local.kind;
    h.storage = st;
    h.cg_iters = plan.local.cg_iters;
    std::vector<int64_t> row_off(P + 1, 0), ell_off(P + 1, 0), band_off(P + 1, 0), trig_off(P + 1, 0);
    int uniformK = -1;
    for (int p = 0; p < P; ++p) {
        const auto& s = plan.subs[p];
        const int64_t n = static_cast<int64_t>(s.omega.size());
        row_off[p + 1] = row_off[p] + n;
        ell_off[p + 1] = ell_off[p] + n_pad_of(n) * s.ell_width;
        // 64-element aligned starts (16-byte aligned blocks for the 16-byte loads)
        band_off[p + 1] = band_off[p] + (chol ? (band_elems(n, s.w) + 63) / 64 * 64 : 0);
        if (chol && s.w <= kSlabMaxW) h.any_slab = true;
        // FP16 slab subdomains: packed triangle inverses, both passes
        trig_off[p + 1] = trig_off[p] + (chol && st == RAS_STORAGE_FP16_ROWSCALED && tri_inverse_ok(s.w, st)
                                             ? 2 * ((n + kBandRows - 1) / kBandRows) * kTriPackFloats
                                             : 0);
        if (chol && s.w > kSlabMaxW) h.max_w_rowmajor = std::max(h.max_w_rowmajor, s.w);
        h.max_n = std::max<int>(h.max_n, static_cast<int>(n));
        h.max_w = std::max(h.max_w, s.w);
        h.max_K = std::max(h.max_K, s.ell_width);
        if (uniformK == -1) uniformK = s.ell_width;
        else if (uniformK != s.ell_width) uniformK = 0;
    }
    h.uniform_K = uniformK > 0 ? uniformK : 0;
    h.sum_n = row_off[P];
    const size_t cts = ct_size(st);
    const size_t sts = st == RAS_STORAGE_FP64 ? 8 : st == RAS_STORAGE_FP32 ? 4 : 2;
    int64_t sp_idx_used = 0, sp_val_used = 0;
    if (sparse) {
        // per subdomain and pass (lane layout): the wave table (int32) and the items'
        // 16-bit columns in the index buffer, the items' values in the value buffer,
        // every array 16-byte aligned; loads run ahead of use, so both buffers end
        // with 2 * kSparseLead rounds of slack
        int64_t ni = 0, nv = 0;  // bytes
        for (int p = 0; p < P; ++p)
            for (int k = 0; k < 2; ++k) {
                const SparseLanes& q = plan.subs[p].lanes[k];
                const int64_t ne = static_cast<int64_t>(q.col.size());
                ni += (4 * static_cast<int64_t>(q.wave.size()) + 15) / 16 * 16 + (2 * ne + 15) / 16 * 16;
                nv += (ne * static_cast<int64_t>(sts) + 15) / 16 * 16;
                h.max_sparse_values = std::max<int64_t>(
                    h.max_sparse_values, static_cast<int64_t>(plan.subs[p].omega.size()) + plan.subs[p].sched[k].slots);
            }
        ni += 2 * kSparseLead * 64 * 2;
        nv += 2 * kSparseLead * 64 * static_cast<int64_t>(sts);
        h.sp_idx.alloc(std::max<int64_t>(ni, 16));
        h.sp_val.alloc(std::max<int64_t>(nv, 16));
        hip_check(hipMemset(h.sp_idx.p, 0, h.sp_idx.bytes), "clear sparse index");
        hip_check(hipMemset(h.sp_val.p, 0, h.sp_val.bytes), "clear sparse values");
    }
    h.omega.alloc(row_off[P] * sizeof(int32_t));
    h.ell_val.alloc(ell_off[P] * sizeof(double));
    if (!chol && st == RAS_STORAGE_FP32) h.ell_valf.alloc(ell_off[P] * sizeof(float));
    h.ell_gcol.alloc(ell_off[P] * sizeof(int32_t));
    h.ell_lcol.alloc(ell_off[P] * sizeof(int32_t));
    if (sparse) h.invd.alloc(row_off[P] * cts);
    if (chol) {
        // tail: the last load round of a slab block may read up to one round past its end
        h.band_f.alloc(band_off[P] * sts + kSlabTailBytes);
        h.band_b.alloc(band_off[P] * sts + kSlabTailBytes);
        // rows past the end of a subdomain's last slab block read as zero
        hip_check(hipMemset(h.band_f.p, 0, band_off[P] * sts + kSlabTailBytes), "clear band");
        hip_check(hipMemset(h.band_b.p, 0, band_off[P] * sts + kSlabTailBytes), "clear band");
        h.invd.alloc(row_off[P] * cts);
        if (st == RAS_STORAGE_FP16_ROWSCALED) h.scale.alloc(row_off[P] * sizeof(float));
        if (trig_off[P] > 0) h.tri_g.alloc(trig_off[P] * sizeof(float));
    }
    h.csr_rp.alloc((plan.n + 1) * sizeof(int64_t));
    h.csr_ci.alloc(plan.nnz * sizeof(int32_t));
    h.csr_va.alloc(plan.nnz * sizeof(double));
    hip_check(hipMemcpy(h.csr_rp.p, plan.row_ptr.data(), (plan.n + 1) * sizeof(int64_t), hipMemcpyHostToDevice),
              "copy row_ptr");
    hip_check(hipMemcpy(h.csr_ci.p, plan.col.data(), plan.nnz * sizeof(int32_t), hipMemcpyHostToDevice), "copy col");
    hip_check(hipMemcpy(h.csr_va.p, plan.val.data(), plan.nnz * sizeof(double), hipMemcpyHostToDevice), "copy val");

    h.subs.resize(P);
    std::vector<int> dev_factor;  // banded subdomains factored on the device
    std::vector<int32_t> om;
    std::vector<double> ev;
    std::vector<float> evf;
    std::vector<int32_t> eg, el, xe, ext_all;
    std::vector<int64_t> ext_off{0};
    std::vector<unsigned char> bf, bb, iv;
    std::vector<float> sc;
    for (int p = 0; p < P; ++p) {
        const auto& s = plan.subs[p];
        const int64_t n = static_cast<int64_t>(s.omega.size());
        const int64_t np = n_pad_of(n);
        const int K = s.ell_width;
        // device local order: ascending global id, or the elimination order of the
        // sparse factor (device row i is omega position dpos[i])
        std::vector<int32_t> dpos(n), drow(n);
        for (int64_t i = 0; i < n; ++i) dpos[i] = sparse ? s.sf.perm[i] : static_cast<int32_t>(i);
        for (int64_t i = 0; i < n; ++i) drow[dpos[i]] = static_cast<int32_t>(i);
        om.resize(n);
        for (int64_t i = 0; i < n; ++i) om[i] = s.owned[dpos[i]] ? s.omega[dpos[i]] : ~s.omega[dpos[i]];
        ev.assign(np * K, 0.0);
        eg.assign(np * K, 0);
        el.assign(np * K, 0);
        xe = external_set(plan, s);
        for (int64_t i = 0; i < n; ++i) {
            const int32_t g = s.omega[dpos[i]];
            int k = 0;
            for (int64_t e = plan.row_ptr[g]; e < plan.row_ptr[g + 1]; ++e, ++k) {
                const int32_t c = plan.col[e];
                ev[k * np + i] = plan.val[e];
                eg[k * np + i] = c;
                auto it = std::lower_bound(s.omega.begin(), s.omega.end(), c);
                if (it != s.omega.end() && *it == c)
                    el[k * np + i] = drow[it - s.omega.begin()];
                else
                    el[k * np + i] = static_cast<int32_t>(n + (std::lower_bound(xe.begin(), xe.end(), c) - xe.begin()));
            }
            for (; k < K; ++k) {  // padding: value 0 times the row's own x
                eg[k * np + i] = g;
                el[k * np + i] = static_cast<int32_t>(i);
            }
        }
        ext_all.insert(ext_all.end(), xe.begin(), xe.end());
        ext_off.push_back(static_cast<int64_t>(ext_all.size()));
        {
            // per-row reach of the local columns, then the window of every team member
            std::vector<int32_t> rmin(n), rmax(n);
            for (int64_t i = 0; i < n; ++i) {
                int32_t a = static_cast<int32_t>(i), b = static_cast<int32_t>(i);
                for (int k = 0; k < K; ++k) {
                    const int32_t c = el[k * np + i];
                    if (c < n) {
                        a = std::min(a, c);
                        b = std::max(b, c);
                    }
                }
                rmin[i] = a;
                rmax[i] = b;
            }
            for (int t = 0; t < 5; ++t) {
                const int T = kTeamSizes[t];
                for (int m = 0; m < T; ++m) {
                    const int64_t lo = m * n / T, hi = (m + 1) * n / T;
                    int32_t a = static_cast<int32_t>(lo), b = static_cast<int32_t>(hi);
                    for (int64_t i = lo; i < hi; ++i) {
                        a = std::min(a, rmin[i]);
                        b = std::max(b, rmax[i] + 1);
                    }
                    h.win[t].push_back(a);
                    h.win[t].push_back(b);
                    h.max_win[t] = std::max(h.max_win[t], b - a);
                }
            }
        }
        hip_check(hipMemcpy(h.omega.as<int32_t>() + row_off[p], om.data(), n * sizeof(int32_t), hipMemcpyHostToDevice),
                  "copy omega");
        hip_check(hipMemcpy(h.ell_val.as<double>() + ell_off[p], ev.data(), np * K * sizeof(double),
                            hipMemcpyHostToDevice),
                  "copy ell_val");
        if (h.ell_valf.p) {
            evf.resize(np * K);
            for (int64_t e = 0; e < np * K; ++e) evf[e] = static_cast<float>(ev[e]);
            hip_check(hipMemcpy(h.ell_valf.as<float>() + ell_off[p], evf.data(), np * K * sizeof(float),
                                hipMemcpyHostToDevice),
                      "copy ell_valf");
        }
        hip_check(hipMemcpy(h.ell_gcol.as<int32_t>() + ell_off[p], eg.data(), np * K * sizeof(int32_t),
                            hipMemcpyHostToDevice),
                  "copy ell_gcol");
        hip_check(hipMemcpy(h.ell_lcol.as<int32_t>() + ell_off[p], el.data(), np * K * sizeof(int32_t),
                            hipMemcpyHostToDevice),
                  "copy ell_lcol");
        SubDev d{};
        d.omega = h.omega.as<int32_t>() + row_off[p];
        d.ell_val = h.ell_val.as<double>() + ell_off[p];
        d.ell_valf = h.ell_valf.p ? h.ell_valf.as<float>() + ell_off[p] : nullptr;
        d.ell_gcol = h.ell_gcol.as<int32_t>() + ell_off[p];
        d.ell_lcol = h.ell_lcol.as<int32_t>() + ell_off[p];
        d.n = static_cast<int32_t>(n);
        d.n_pad = static_cast<int32_t>(np);
        d.K = K;
        d.w = s.w;
        d.row_off = row_off[p];
        if (chol) d.tri_inv = tri_inverse_ok(s.w, st) ? 1 : 0;
        if (trig_off[p + 1] > trig_off[p]) {
            const int64_t half = (trig_off[p + 1] - trig_off[p]) / 2;
            d.tri_g[0] = h.tri_g.as<float>() + trig_off[p];
            d.tri_g[1] = h.tri_g.as<float>() + trig_off[p] + half;
        }
        if (chol && s.L.empty()) {
            // factored on the device after this loop
            d.slab = s.w <= kSlabMaxW ? 1 : 0;
            d.band_f = static_cast<char*>(h.band_f.p) + band_off[p] * sts;
            d.band_b = static_cast<char*>(h.band_b.p) + band_off[p] * sts;
            d.invd = static_cast<char*>(h.invd.p) + row_off[p] * cts;
            if (st == RAS_STORAGE_FP16_ROWSCALED) d.scale = h.scale.as<float>() + row_off[p];
            dev_factor.push_back(p);
        } else if (chol) {
            const int64_t ld = s.w + 1;
            const int w = s.w;
            const double* L = s.L.data();
            const bool slab = w <= kSlabMaxW;
            const int64_t elems = band_elems(n, w);
            bf.assign(elems * sts, 0);
            bb.assign(elems * sts, 0);
            iv.resize(n * cts);
            // destination index of entry (t, o): row-major [t][o], or slab block
            // t / BR stored [o][t % BR] (diagonal not stored in the slab)
            auto dst = [&](int64_t t, int64_t o) -> int64_t {
                if (!slab) return t * ld + o;
                const int64_t j = t / kBandRows, r = t % kBandRows;
                return (j * w + o) * kBandRows + r;
            };
            const int64_t olim = slab ? w : ld;
            for (int64_t t = 0; t < n; ++t) {
                for (int64_t o = 0; o < olim; ++o) {
                    const int64_t r = (n - 1 - t) + w - o;  // row of L read by the reversed transpose
                    const int64_t fi = t * ld + o;
                    const int64_t di = dst(t, o);
                    if (st == RAS_STORAGE_FP64) {
                        reinterpret_cast<double*>(bf.data())[di] = L[fi];
                        reinterpret_cast<double*>(bb.data())[di] = r < n ? L[r * ld + o] : 0.0;
                    } else if (st == RAS_STORAGE_FP32) {
                        reinterpret_cast<float*>(bf.data())[di] = static_cast<float>(L[fi]);
                        reinterpret_cast<float*>(bb.data())[di] = r < n ? static_cast<float>(L[r * ld + o]) : 0.0f;
                    } else {
                        reinterpret_cast<uint16_t*>(bf.data())[di] = s.Lh[fi];
                        reinterpret_cast<uint16_t*>(bb.data())[di] = r < n ? s.Lh[r * ld + o] : 0;
                    }
                }
                // reciprocal of the diagonal as the triangular solves see it
                const int64_t di = t * ld + s.w;
                if (st == RAS_STORAGE_FP64) {
                    reinterpret_cast<double*>(iv.data())[t] = 1.0 / L[di];
                } else if (st == RAS_STORAGE_FP32) {
                    reinterpret_cast<float*>(iv.data())[t] = static_cast<float>(1.0 / static_cast<double>(static_cast<float>(L[di])));
                } else {
                    _Float16 hv;
                    std::memcpy(&hv, &s.Lh[di], 2);
                    const float deq = static_cast<float>(hv) * s.scale[t];
                    reinterpret_cast<float*>(iv.data())[t] = static_cast<float>(1.0 / static_cast<double>(deq));
                }
            }
            d.slab = slab ? 1 : 0;
            if (d.tri_inv) {
                // the inverse of every block's triangle: in the triangle slots (FP64 / FP32)
                // or packed in float32 beside the factor (FP16), as the device factorisation writes it
                const int64_t half = (trig_off[p + 1] - trig_off[p]) / 2;
                std::vector<float> gh(2 * half);
                for (int pass = 0; pass < 2; ++pass)
                    store_block_inverses(L, n, w, st, pass == 1, pass == 0 ? bf.data() : bb.data(), s.Lh.data(),
                                         s.scale.data(), gh.data() + pass * half);
                if (half > 0)
                    hip_check(hipMemcpy(h.tri_g.as<float>() + trig_off[p], gh.data(), gh.size() * sizeof(float),
                                        hipMemcpyHostToDevice),
                              "copy triangle inverses");
            }
            hip_check(hipMemcpy(static_cast<char*>(h.band_f.p) + band_off[p] * sts, bf.data(), elems * sts,
                                hipMemcpyHostToDevice),
                      "copy band_f");
            hip_check(hipMemcpy(static_cast<char*>(h.band_b.p) + band_off[p] * sts, bb.data(), elems * sts,
                                hipMemcpyHostToDevice),
                      "copy band_b");
            hip_check(hipMemcpy(static_cast<char*>(h.invd.p) + row_off[p] * cts, iv.data(), n * cts,
                                hipMemcpyHostToDevice),
                      "copy invd");
            d.band_f = static_cast<char*>(h.band_f.p) + band_off[p] * sts;
            d.band_b = static_cast<char*>(h.band_b.p) + band_off[p] * sts;
            d.invd = static_cast<char*>(h.invd.p) + row_off[p] * cts;
            if (st == RAS_STORAGE_FP16_ROWSCALED) {
                hip_check(hipMemcpy(h.scale.as<float>() + row_off[p], s.scale.data(), n * sizeof(float),
                                    hipMemcpyHostToDevice),
                          "copy scale");
                d.scale = h.scale.as<float>() + row_off[p];
            }
        }
        if (sparse) {
            const SparseFactor& F = s.sf;
            std::vector<unsigned char> idx, vals;
            int64_t ioff[2][2], voff[2];
            auto put = [](std::vector<unsigned char>& to, const void* from, size_t bytes) {
                const unsigned char* c = static_cast<const unsigned char*>(from);
                to.insert(to.end(), c, c + bytes);
                while (to.size() % 16) to.push_back(0);  // 16-byte aligned arrays
            };
            for (int k = 0; k < 2; ++k) {
                const SparseLanes& q = s.lanes[k];
                ioff[k][0] = sp_idx_used + static_cast<int64_t>(idx.size());
                put(idx, q.wave.data(), q.wave.size() * sizeof(int32_t));
                ioff[k][1] = sp_idx_used + static_cast<int64_t>(idx.size());
                {
                    // the columns of rounds 2m and 2m + 1 in one word per lane
                    std::vector<uint32_t> words(q.col.size() / 2);
                    for (size_t m = 0; m < words.size() / 64; ++m)
                        for (size_t l = 0; l < 64; ++l)
                            words[m * 64 + l] = static_cast<uint32_t>(q.col[(2 * m) * 64 + l]) |
                                                static_cast<uint32_t>(q.col[(2 * m + 1) * 64 + l]) << 16;
                    put(idx, words.data(), words.size() * sizeof(uint32_t));
                }
                voff[k] = sp_val_used + static_cast<int64_t>(vals.size());
                for (size_t e = 0; e < q.val.size(); ++e) {
                    const double x = q.val[e];
                    if (st == RAS_STORAGE_FP64) {
                        const unsigned char* b = reinterpret_cast<const unsigned char*>(&x);
                        vals.insert(vals.end(), b, b + 8);
                    } else {
                        // a terminator's payload is an integer in the value's bits: keep its low 32 bits
                        float f = static_cast<float>(x);
                        if (q.col[e] == kSparseTerm) {
                            uint64_t bits;
                            std::memcpy(&bits, &x, sizeof bits);
                            const uint32_t lo = static_cast<uint32_t>(bits);
                            std::memcpy(&f, &lo, sizeof f);
                        }
                        const unsigned char* b = reinterpret_cast<const unsigned char*>(&f);
                        vals.insert(vals.end(), b, b + 4);
                    }
                }
                while (vals.size() % 16) vals.push_back(0);
                d.sp_nlev[k] = static_cast<int32_t>(s.sched[k].step.size()) - 1;
            }
            hip_check(hipMemcpy(static_cast<char*>(h.sp_idx.p) + sp_idx_used, idx.data(), idx.size(),
                                hipMemcpyHostToDevice),
                      "copy sparse index");
            hip_check(hipMemcpy(static_cast<char*>(h.sp_val.p) + sp_val_used, vals.data(), vals.size(),
                                hipMemcpyHostToDevice),
                      "copy sparse values");
            for (int k = 0; k < 2; ++k) {
                d.sp_wave[k] = reinterpret_cast<const int32_t*>(static_cast<char*>(h.sp_idx.p) + ioff[k][0]);
                d.sp_col[k] = reinterpret_cast<const uint32_t*>(static_cast<char*>(h.sp_idx.p) + ioff[k][1]);
                d.sp_val[k] = static_cast<char*>(h.sp_val.p) + voff[k];
            }
            sp_idx_used += static_cast<int64_t>(idx.size());
            sp_val_used += static_cast<int64_t>(vals.size());
            iv.resize(n * cts);
            for (int64_t i = 0; i < n; ++i) {
                if (st == RAS_STORAGE_FP64)
                    reinterpret_cast<double*>(iv.data())[i] = 1.0 / F.d[i];
                else
                    reinterpret_cast<float*>(iv.data())[i] =
                        static_cast<float>(1.0 / static_cast<double>(static_cast<float>(F.d[i])));
            }
            hip_check(hipMemcpy(static_cast<char*>(h.invd.p) + row_off[p] * cts, iv.data(), n * cts,
                                hipMemcpyHostToDevice),
                      "copy invd");
            d.invd = static_cast<char*>(h.invd.p) + row_off[p] * cts;
            d.sparse = 1;
        }
        h.subs[p] = d;
    }
    if (!dev_factor.empty()) device_factor(h, plan, dev_factor);
    // control words: cancel, then one pause word per subdomain
    {
        void* hp = nullptr;
        hip_check(hipHostMalloc(&hp, (1 + static_cast<size_t>(P)) * sizeof(int32_t),
                                hipHostMallocMapped | hipHostMallocCoherent),
                  "control words");
        h.ctl.host = static_cast<int32_t*>(hp);
        std::memset(h.ctl.host, 0, (1 + static_cast<size_t>(P)) * sizeof(int32_t));
        void* dp = nullptr;
        hip_check(hipHostGetDevicePointer(&dp, hp, 0), "control words (device address)");
        h.ctl.dev = static_cast<int32_t*>(dp);
    }
    // neighbours: subdomains owning a column read by a row of Omega_p (the
    // residual's interface columns included); used by decentralized detection
    {
        std::vector<int32_t> all, ptr(P + 1, 0), mark(P, -1);
        for (int p = 0; p < P; ++p) {
            for (int32_t g : plan.subs[p].omega)
                for (int64_t e = plan.row_ptr[g]; e < plan.row_ptr[g + 1]; ++e) {
                    const int32_t q = plan.owner[plan.col[e]];
                    if (q != p && mark[q] != p) {
                        mark[q] = p;
                        all.push_back(q);
                    }
                }
            std::sort(all.begin() + ptr[p], all.end());
            ptr[p + 1] = static_cast<int32_t>(all.size());
        }
        h.nbr.alloc(std::max<size_t>(1, all.size()) * sizeof(int32_t));
        if (!all.empty())
            hip_check(hipMemcpy(h.nbr.p, all.data(), all.size() * sizeof(int32_t), hipMemcpyHostToDevice), "copy nbr");
        for (int p = 0; p < P; ++p) {
            h.subs[p].nbr = h.nbr.as<int32_t>() + ptr[p];
            h.subs[p].n_nbr = ptr[p + 1] - ptr[p];
        }
    }
    // external columns of every subdomain, and the snapshot offsets (n + n_ext per subdomain)
    {
        h.ext.alloc(std::max<size_t>(1, ext_all.size()) * sizeof(int32_t));
        if (!ext_all.empty())
            hip_check(hipMemcpy(h.ext.p, ext_all.data(), ext_all.size() * sizeof(int32_t), hipMemcpyHostToDevice),
                      "copy ext");
        int64_t so = 0;
        for (int p = 0; p < P; ++p) {
            h.subs[p].ext = h.ext.as<int32_t>() + ext_off[p];
            h.subs[p].n_ext = static_cast<int32_t>(ext_off[p + 1] - ext_off[p]);
            h.subs[p].snap_off = so;
            so += h.subs[p].n + h.subs[p].n_ext;
        }
        h.sum_snap = so;
    }
    plan_stats(plan, &h.stats);
    h.stats.device_bytes = static_cast<int64_t>(h.omega.bytes + h.ell_val.bytes + h.ell_valf.bytes + h.ell_gcol.bytes +
                                                h.ell_lcol.bytes + h.band_f.bytes + h.band_b.bytes + h.invd.bytes +
                                                h.scale.bytes + h.csr_rp.bytes + h.csr_ci.bytes + h.csr_va.bytes +
                                                h.ext.bytes + h.sp_idx.bytes + h.sp_val.bytes + h.tri_g.bytes);
}

void drop_factors(Plan& plan) {
    for (auto& s : plan.subs) {
        std::vector<double>().swap(s.L);
        std::vector<uint16_t>().swap(s.Lh);
        std::vector<float>().swap(s.scale);
        for (SparseSchedule& q : s.sched) q = SparseSchedule{};
        for (SparseLanes& q : s.lanes) q = SparseLanes{};
    }
}



struct InstSpec {
    ras_handle* h;
    const double* b;
    double* x;
    int rhs;
    double tol = -1.0;     // per-system tolerance (< 0: the solve options' tol)
    double bnorm2 = -1.0;  // ||b||^2 if already known (< 0: computed by the solve)
};

// Where a solve's workspace lives: a fresh allocation (default), a buffer that
// is reused and grown across solves (serving), or a fixed caller-visible area
// that must not be exceeded (no allocation at all).
struct Workspace {
    DevBuf* reuse = nullptr;
    void* fixed = nullptr;
    size_t fixed_bytes = 0;
};

// One persistent solve over a set of right-hand sides of one or more systems.
ras_status run_solve(std::vector<InstSpec>& specs, const ras_solve_opts& o, ras_solve_info* info,
                     const Workspace& where = Workspace{}) {
    ras_handle& h0 = *specs[0].h;
    hipStream_t stream = h0.stream;
    hip_check(hipSetDevice(h0.device), "hipSetDevice");
    const bool sync = o.mode == RAS_MODE_SYNC;
    const bool ordered = o.mode == RAS_MODE_ORDERED;
    if (o.mode != RAS_MODE_SYNC && o.mode != RAS_MODE_ASYNC && o.mode != RAS_MODE_ORDERED)
        throw Error{RAS_E_ARG, "unknown mode"};
    if (!(o.tol >= 0.0) || o.max_sweeps < 1) throw Error{RAS_E_ARG, "tol must be >= 0 and max_sweeps >= 1"};
    if (o.detect != RAS_DETECT_CENTRAL && o.detect != RAS_DETECT_DECENTRAL && o.detect != RAS_DETECT_ESTIMATE)
        throw Error{RAS_E_ARG, "unknown detector"};
    if (!(o.pace <= 16.0)) throw Error{RAS_E_ARG, "pace must be at most 16 (negative: library choice)"};
    if (!(o.detect_factor >= 0.0)) throw Error{RAS_E_ARG, "detect_factor must be >= 0 (0: 1)"};
    // the detector's threshold; SYNC stops on the exact residual of each sweep
    const double detect_factor = (sync || o.detect_factor == 0.0) ? 1.0 : o.detect_factor;
    // distinct handles, in first-use order
    std::vector<ras_handle*> hs;
    for (auto& sp : specs)
        if (std::find(hs.begin(), hs.end(), sp.h) == hs.end()) hs.push_back(sp.h);
    int max_n = 0, max_w = 0, K = -1;
    for (ras_handle* h : hs) {
        if (h->solver != h0.solver || h->storage != h0.storage || h->cg_iters != h0.cg_iters)
            throw Error{RAS_E_ARG, "batched systems must share the local solver, storage and CG iterations"};
        max_n = std::max(max_n, h->max_n);
        max_w = std::max(max_w, h->max_w);
        if (K == -1) K = h->uniform_K;
        else if (K != h->uniform_K) K = 0;
    }
    const int ninst = static_cast<int>(specs.size());
    std::vector<double> tol_v(ninst);
    for (int i = 0; i < ninst; ++i) tol_v[i] = specs[i].tol >= 0.0 ? specs[i].tol : o.tol;
    int nitems_total = 0;
    for (auto& sp : specs) nitems_total += sp.h->plan->P;

    // kernel configuration: team size T (CG), rows-per-thread class, LDS bytes
    struct Cfg {
        int tidx = -1, T = 1, rclass = 0, winm = 0, per_cu = 0;
        int band_args[3] = {0, 0, 0};
        size_t lds = 0;
        const void* kern = nullptr;
    };
    auto make_cfg = [&](int tidx) {
        Cfg c;
        c.tidx = tidx;
        if (h0.solver == RAS_LOCAL_CG) {
            c.T = kTeamSizes[tidx];
            int maxwin = 0;
            for (ras_handle* h : hs) maxwin = std::max(maxwin, h->max_win[tidx]);
            c.lds = (static_cast<size_t>(maxwin) + 1) * ct_size(h0.storage);
            c.rclass = cg_rows_class((max_n + c.T - 1) / c.T);
            if (c.rclass < 0) return c;
            c.kern = select_kernel(h0.solver, h0.storage, !sync, K, c.rclass);
        } else {
            if (tidx != 0) return c;
            // LDS: slab stages + solution window (2w + 2 blocks, a power of two)
            // + partial sums, and / or the window + stage of the row-major pass
            const size_t cts = ct_size(h0.storage);
            const int sts = h0.storage == RAS_STORAGE_FP64 ? 8 : h0.storage == RAS_STORAGE_FP32 ? 4 : 2;
            int wrm = -1, wslab = -1;
            size_t wsparse = 0;
            for (ras_handle* h : hs) {
                wrm = std::max(wrm, h->max_w_rowmajor);
                if (h->any_slab) wslab = std::max(wslab, std::min(h->max_w, kSlabMaxW));
                // y and the dense blocks' slots in LDS
                if (h->sparse) wsparse = std::max(wsparse, static_cast<size_t>(h->max_sparse_values) * cts);
            }
            const int win = next_pow2(2 * max_w + 2 * kBandRows);
            size_t bytes = 0;
            if (wslab >= 0) bytes = std::max(bytes, slab_lds_bytes(sts, static_cast<int>(cts), wslab, win));
            if (wrm >= 0) bytes = std::max(bytes, (static_cast<size_t>(win) + static_cast<size_t>(kBandRows) * (wrm + 1)) * cts);
            bytes = std::max(bytes, wsparse);
            c.rclass = kBandRows;
            c.winm = win - 1;
            c.lds = bytes;
            c.band_args[0] = std::max(wrm, 0);
            c.band_args[1] = c.winm;
            c.band_args[2] = wslab >= 0 ? static_cast<int>(slab_stage_bytes(sts, wslab)) : 0;
            c.kern = select_kernel(h0.solver, h0.storage, !sync, K, c.rclass);
        }
        if (!c.kern || c.lds > kLdsLimit) {
            c.kern = nullptr;
            return c;
        }
        if (occupancy(c.kern, h0.solver, c.lds, &c.per_cu) != hipSuccess || c.per_cu < 1) c.kern = nullptr;
        return c;
    };
    auto busy_wgs = [&](const Cfg& c) {
        const int teams = std::min(nitems_total, c.per_cu * h0.num_cu / c.T);
        return teams * c.T;
    };
    Cfg cfg;
    int want_team = o.team > 0 ? o.team : (h0.solver == RAS_LOCAL_CG ? h0.tuned_team : 0);
    if (want_team == 0 && h0.solver == RAS_LOCAL_CG && hs.size() == 1) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find({h0.plan->n, h0.plan->P, h0.max_n, h0.uniform_K, h0.storage, h0.cg_iters});
        if (it != g_tune.end()) want_team = it->second;
    }
    if (want_team > 0) {
        for (int t = 0; t < 5; ++t)
            if (kTeamSizes[t] == want_team) cfg = make_cfg(t);
        if (!cfg.kern && o.team > 0)
            throw Error{RAS_E_UNSUPPORTED, "team size " + std::to_string(o.team) + " not available for this shape"};
    }
    if (!cfg.kern) {
        // heuristic: the smallest team that keeps every CU busy, without splitting a
        // subdomain into members of fewer than two rows per thread; the ordered
        // (single-team) mode takes the smallest team that fits
        Cfg best;
        for (int t = 0; t < 5; ++t) {
            Cfg c = make_cfg(t);
            if (!c.kern) continue;
            if (!best.kern) {
                best = c;
                if (ordered) break;
                continue;
            }
            if ((max_n + c.T - 1) / c.T < 2 * kCgThreads) break;
            if (busy_wgs(best) >= h0.num_cu) break;
            if (busy_wgs(c) > busy_wgs(best)) best = c;
        }
        cfg = best;
    }
    if (!cfg.kern)
        throw Error{RAS_E_UNSUPPORTED, "subdomains too large for the on-chip kernels (rows per workgroup or LDS); "
                                       "use more subdomains"};
    const void* kern = cfg.kern;
    const size_t lds = cfg.lds;
    const int T = cfg.T;

    // subdomain table: handle order; per-instance items
    std::vector<SubDev> subs;
    std::vector<int32_t> team_win;
    std::vector<int> sub_base(hs.size());
    for (size_t k = 0; k < hs.size(); ++k) {
        sub_base[k] = static_cast<int>(subs.size());
        subs.insert(subs.end(), hs[k]->subs.begin(), hs[k]->subs.end());
        const auto& wv = hs[k]->win[h0.solver == RAS_LOCAL_CG ? cfg.tidx : 0];
        team_win.insert(team_win.end(), wv.begin(), wv.end());
    }
    std::vector<ItemDev> items;
    std::vector<double> cost;
    std::vector<InstDev> insts(ninst);
    int64_t scratch_elems = 0;
    std::vector<int64_t> scratch_off(ninst), x1_off(ninst), snap_off(ninst);
    int64_t x1_elems = 0, snap_elems = 0;
    for (int i = 0; i < ninst; ++i) {
        ras_handle* h = specs[i].h;
        const int hk = static_cast<int>(std::find(hs.begin(), hs.end(), h) - hs.begin());
        insts[i].item_begin = static_cast<int32_t>(items.size());
        insts[i].item_count = h->plan->P;
        for (int p = 0; p < h->plan->P; ++p) {
            items.push_back(ItemDev{i, sub_base[hk] + p});
            const SubDev& sd = h->subs[p];
            cost.push_back(h->solver == RAS_LOCAL_CG ? static_cast<double>(sd.n) * sd.K * (h->cg_iters + 1)
                                                     : static_cast<double>(sd.n) * (2.0 * (sd.w + 1) + sd.K));
        }
        scratch_off[i] = scratch_elems;
        scratch_elems += h->sum_n;
        x1_off[i] = x1_elems;
        x1_elems += sync ? h->plan->n : 0;
        snap_off[i] = snap_elems;
        snap_elems += sync ? 0 : h->sum_snap;
    }
    const int nitems = static_cast<int>(items.size());

    // teams: co-resident capacity, balanced static item lists (LPT)
    int nteams = ordered ? 1 : std::min(nitems, cfg.per_cu * h0.num_cu / T);
    if (o.workgroups > 0) nteams = std::min(nteams, std::max(1, o.workgroups / T));
    if (nteams < 1) nteams = 1;
    const int G = nteams * T;
    std::vector<std::vector<int>> lists(nteams);
    {
        std::vector<int> order(nitems);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        using Load = std::pair<double, int>;
        std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
        for (int g = 0; g < nteams; ++g) heap.push({0.0, g});
        for (int it : order) {
            Load l = heap.top();
            heap.pop();
            lists[l.second].push_back(it);
            heap.push({l.first + cost[it], l.second});
        }
        for (auto& l : lists) std::sort(l.begin(), l.end());
    }
    // workgroup -> (team, member): the members of a team get workgroup ids that are
    // equal modulo 8, so the round-robin placement of workgroups over the eight
    // XCDs keeps a team (and its barrier and halo traffic) inside one XCD's L2
    std::vector<int32_t> wg_team(G), wg_member(G), team_first_wg(nteams);
    for (int grp = 0; grp * 8 < nteams; ++grp) {
        const int gs = std::min(8, nteams - grp * 8);
        const int basewg = grp * 8 * T;
        for (int m = 0; m < T; ++m)
            for (int l = 0; l < gs; ++l) {
                const int g = basewg + m * gs + l;
                wg_team[g] = grp * 8 + l;
                wg_member[g] = m;
                if (m == 0) team_first_wg[grp * 8 + l] = g;
            }
    }
    std::vector<int32_t> team_ptr(nteams + 1, 0), team_items;
    std::vector<int> owner_wg(nitems, 0);
    for (int t = 0; t < nteams; ++t) {
        if (static_cast<int>(lists[t].size()) > kMaxItemsPerWg)
            throw Error{RAS_E_UNSUPPORTED, "too many work items per team"};
        for (int it : lists[t]) {
            team_items.push_back(it);
            owner_wg[it] = team_first_wg[t];
        }
        team_ptr[t + 1] = static_cast<int32_t>(team_items.size());
    }

    // device workspace (one block, carved)
    // synchronous history: one entry per sweep; asynchronous: one per detector check
    const int64_t hist_cap = std::min<int64_t>(o.max_sweeps + 1, sync ? (1 << 20) : (1 << 16));
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        size_t at = off;
        off += align(bytes);
        return at;
    };
    const size_t o_subs = carve(subs.size() * sizeof(SubDev));
    const size_t o_items = carve(items.size() * sizeof(ItemDev));
    const size_t o_insts = carve(insts.size() * sizeof(InstDev));
    const size_t o_ist = carve(insts.size() * sizeof(InstState));
    const size_t o_res2 = carve(2 * nitems * sizeof(double));
    const size_t o_conv = carve(nitems * sizeof(int32_t));
    const size_t o_gflag = carve(nitems * sizeof(int32_t));
    const size_t o_solves = carve(nitems * sizeof(int64_t));
    const size_t o_phase = carve(4 * static_cast<size_t>(nitems) * sizeof(int64_t));
    const size_t o_version = carve(nitems * sizeof(uint32_t));
    const size_t o_tptr = carve((nteams + 1) * sizeof(int32_t));
    const size_t o_titems = carve(team_items.size() * sizeof(int32_t));
    const size_t o_wgteam = carve(G * sizeof(int32_t));
    const size_t o_wgmember = carve(G * sizeof(int32_t));
    const size_t o_twin = carve(team_win.size() * sizeof(int32_t));
    const size_t o_tbar = carve(2 * nteams * sizeof(uint32_t));
    const size_t o_tbuf = carve(static_cast<size_t>(nteams) * 8 * T * sizeof(double));
    const size_t o_bar = carve(sizeof(GridBarrier));
    const size_t o_scr = carve(scratch_elems * ct_size(h0.storage));
    const size_t o_x1 = carve(x1_elems * sizeof(double));
    const size_t o_snap = carve(snap_elems * sizeof(double));
    const size_t o_hist = carve(2 * static_cast<size_t>(ninst) * hist_cap * sizeof(double));
    const int nparts = 512;
    // reduction slots: partial sums (reused launch after launch on the stream) and two
    // results per right-hand side, so that all norms of a step come back in one copy
    const size_t o_red = carve((2 * nparts + 2 * static_cast<size_t>(ninst)) * sizeof(double));
    DevBuf ws;
    char* base = nullptr;
    if (where.fixed) {
        if (off > where.fixed_bytes)
            throw Error{RAS_E_NOMEM, "solve workspace needs " + std::to_string(off) +
                                         " bytes; the fixed no-allocation scratch holds " +
                                         std::to_string(where.fixed_bytes)};
        base = static_cast<char*>(where.fixed);
    } else if (where.reuse) {
        where.reuse->ensure(off);
        base = where.reuse->as<char>();
    } else {
        ws.alloc(off);
        base = ws.as<char>();
    }
    for (int i = 0; i < ninst; ++i) {
        InstDev& in = insts[i];
        in.b = specs[i].b;
        in.x0 = specs[i].x;
        in.x1 = sync ? reinterpret_cast<double*>(base + o_x1) + x1_off[i] : nullptr;
        in.scratch = base + o_scr + scratch_off[i] * ct_size(h0.storage);
        in.snap = sync ? nullptr : reinterpret_cast<double*>(base + o_snap) + snap_off[i];
        in.hist = reinterpret_cast<double*>(base + o_hist) + static_cast<size_t>(i) * hist_cap;
        in.hist_t = reinterpret_cast<double*>(base + o_hist) + static_cast<size_t>(ninst + i) * hist_cap;
        in.hist_cap = hist_cap;
        in.max_sweeps = o.max_sweeps;
        in.tol2 = (tol_v[i] * detect_factor) * (tol_v[i] * detect_factor);
        in.leader = owner_wg[in.item_begin];
        in.ctl = ordered ? nullptr : specs[i].h->ctl.dev;  // ORDERED ignores pauses and cancels
        if (specs[i].h->ctl.host) __atomic_store_n(specs[i].h->ctl.host, 0, __ATOMIC_SEQ_CST);  // a new solve: not cancelled
    }
    {
        // ||b||^2 of the right-hand sides not given one (deterministic two-pass
        // reductions), all returned in one copy
        double* red0 = reinterpret_cast<double*>(base + o_red);
        std::vector<double> out(2 * static_cast<size_t>(ninst), 0.0);
        bool any = false;
        for (int i = 0; i < ninst; ++i) {
            if (specs[i].bnorm2 >= 0.0) continue;
            ras_handle* h = specs[i].h;
            hip_check(launch_residual(h->plan->n, h->csr_rp.as<int64_t>(), h->csr_ci.as<int32_t>(),
                                      h->csr_va.as<double>(), specs[i].b, nullptr, red0, nparts,
                                      red0 + 2 * nparts + 2 * i, stream),
                      "norm of b");
            any = true;
        }
        if (any) {
            hip_check(hipMemcpyAsync(out.data(), red0 + 2 * nparts, out.size() * sizeof(double), hipMemcpyDeviceToHost,
                                     stream),
                      "copy norms");
            hip_check(hipStreamSynchronize(stream), "sync norms");
        }
        for (int i = 0; i < ninst; ++i) {
            insts[i].bnorm2 = specs[i].bnorm2 >= 0.0 ? specs[i].bnorm2 : out[2 * i + 1];
            if (!(insts[i].bnorm2 > 0.0)) throw Error{RAS_E_ARG, "right-hand side " + std::to_string(i) + " is zero"};
        }
    }
    std::vector<InstState> ist(ninst);
    for (auto& s : ist) {
        s.stop = 0;
        s.result_buf = 0;
        s.sweeps = 0;
        s.hist_len = 0;
        s.stopped_at = -1;
        s.t0 = 0;
    }
    GridBarrier bar{0, 0, INT64_MAX};
    auto up = [&](size_t o_, const void* src, size_t bytes) {
        if (bytes) hip_check(hipMemcpyAsync(base + o_, src, bytes, hipMemcpyHostToDevice, stream), "upload tables");
    };
    up(o_subs, subs.data(), subs.size() * sizeof(SubDev));
    up(o_items, items.data(), items.size() * sizeof(ItemDev));
    up(o_insts, insts.data(), insts.size() * sizeof(InstDev));
    up(o_ist, ist.data(), ist.size() * sizeof(InstState));
    up(o_tptr, team_ptr.data(), team_ptr.size() * sizeof(int32_t));
    up(o_titems, team_items.data(), team_items.size() * sizeof(int32_t));
    up(o_wgteam, wg_team.data(), wg_team.size() * sizeof(int32_t));
    up(o_wgmember, wg_member.data(), wg_member.size() * sizeof(int32_t));
    up(o_twin, team_win.data(), team_win.size() * sizeof(int32_t));
    hip_check(hipMemsetAsync(base + o_tbar, 0, 2 * nteams * sizeof(uint32_t), stream), "clear");
    up(o_bar, &bar, sizeof(bar));
    hip_check(hipMemsetAsync(base + o_res2, 0, 2 * nitems * sizeof(double), stream), "clear");
    hip_check(hipMemsetAsync(base + o_conv, 0, nitems * sizeof(int32_t), stream), "clear");
    hip_check(hipMemsetAsync(base + o_gflag, 0, nitems * sizeof(int32_t), stream), "clear");
    hip_check(hipMemsetAsync(base + o_solves, 0, nitems * sizeof(int64_t), stream), "clear");
    hip_check(hipMemsetAsync(base + o_phase, 0, 4 * static_cast<size_t>(nitems) * sizeof(int64_t), stream), "clear");
    hip_check(hipMemsetAsync(base + o_version, 0, nitems * sizeof(uint32_t), stream), "clear");
    if (sync)  // x^0 lives in the caller's buffer; the other buffer is filled by the first sweep
        hip_check(hipMemsetAsync(base + o_x1, 0, x1_elems * sizeof(double), stream), "clear");

    Params P{};
    P.subs = reinterpret_cast<const SubDev*>(base + o_subs);
    P.items = reinterpret_cast<const ItemDev*>(base + o_items);
    P.insts = reinterpret_cast<const InstDev*>(base + o_insts);
    P.ist = reinterpret_cast<InstState*>(base + o_ist);
    P.res2_own = reinterpret_cast<double*>(base + o_res2);
    P.conv = reinterpret_cast<int32_t*>(base + o_conv);
    P.gflag = reinterpret_cast<int32_t*>(base + o_gflag);
    P.detect = o.detect;
    // library choice: direct (Cholesky) solves run few, long, evenly timed updates, where
    // reading the neighbours' latest update saves about a third of the updates; CG
    // subdomains are many and unevenly timed, where waiting costs more than it saves
    const double pace = o.pace < 0.0 ? (h0.solver != RAS_LOCAL_CG ? 0.25 : 0.0) : o.pace;
    P.pace = o.mode == RAS_MODE_ASYNC ? pace : 0.0;
    P.solves = reinterpret_cast<int64_t*>(base + o_solves);
    P.phase = reinterpret_cast<int64_t*>(base + o_phase);
    P.version = reinterpret_cast<uint32_t*>(base + o_version);
    P.team_ptr = reinterpret_cast<const int32_t*>(base + o_tptr);
    P.team_items = reinterpret_cast<const int32_t*>(base + o_titems);
    P.wg_team = reinterpret_cast<const int32_t*>(base + o_wgteam);
    P.wg_member = reinterpret_cast<const int32_t*>(base + o_wgmember);
    P.team_win = reinterpret_cast<const int32_t*>(base + o_twin);
    P.team_bar = reinterpret_cast<uint32_t*>(base + o_tbar);
    P.team_buf = reinterpret_cast<double*>(base + o_tbuf);
    P.team_size = T;
    P.bar = reinterpret_cast<GridBarrier*>(base + o_bar);
    P.n_items = nitems;
    P.n_insts = ninst;
    P.n_wg = G;
    P.cg_iters = h0.cg_iters;
    P.max_ticks = o.max_seconds > 0 ? static_cast<int64_t>(o.max_seconds * h0.clock_khz * 1000.0) : 0;
    P.sweep0 = 0;

    hipEvent_t ev0 = h0.ev.e[0], ev1 = h0.ev.e[1], ek0 = h0.ev.e[2], ek1 = h0.ev.e[3];
    double kernel_s = 0.0;
    hip_check(launch_stamp(P.ist, ninst, stream), "stamp");
    hip_check(hipEventRecord(ev0, stream), "event record");

    std::vector<std::vector<double>> hist(ninst), hist_t(ninst);
    std::vector<double> relres(ninst, NAN);
    std::vector<int> verified(ninst, 0);
    std::vector<int> launches(ninst, 0);
    const double tick_s = 1.0 / (static_cast<double>(h0.clock_khz) * 1000.0);
    double* red = reinterpret_cast<double*>(base + o_red);
    // exact relative residuals of the listed right-hand sides (the verification of
    // Sec. 3.3.2): one reduction launch each, one copy and one wait for all
    std::vector<double> vout(2 * static_cast<size_t>(ninst));
    auto exact_relres = [&](const std::vector<int>& which) {
        if (which.empty()) return;
        for (int i : which) {
            ras_handle* h = specs[i].h;
            hip_check(launch_residual(h->plan->n, h->csr_rp.as<int64_t>(), h->csr_ci.as<int32_t>(),
                                      h->csr_va.as<double>(), specs[i].b, specs[i].x, red, nparts,
                                      red + 2 * nparts + 2 * i, stream),
                      "verification residual");
        }
        hip_check(hipMemcpyAsync(vout.data(), red + 2 * nparts, vout.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 stream),
                  "copy");
        hip_check(hipStreamSynchronize(stream), "sync verification");
        for (int i : which) relres[i] = std::sqrt(vout[2 * i] / vout[2 * i + 1]);
    };
    std::vector<int64_t> solves_h(nitems);
    std::vector<int32_t> step(ninst, RAS_STEP_RESUME);
    for (int launch = 0;; ++launch) {
        hip_check(hipEventRecord(ek0, stream), "event record");
        hip_check(launch_solver(kern, h0.solver, P, cfg.band_args, lds, stream, sync || T > 1),
                  "persistent kernel launch");
        hip_check(hipEventRecord(ek1, stream), "event record");
        hip_check(hipStreamSynchronize(stream), "persistent kernel");
        {
            float kms = 0.0f;
            hip_check(hipEventElapsedTime(&kms, ek0, ek1), "elapsed");
            kernel_s += kms * 1e-3;
        }
        for (int i = 0; i < ninst; ++i)
            if (!verified[i]) ++launches[i];
        hip_check(hipMemcpyAsync(ist.data(), P.ist, ninst * sizeof(InstState), hipMemcpyDeviceToHost, stream),
                  "copy state");
        hip_check(hipMemcpyAsync(solves_h.data(), P.solves, nitems * sizeof(int64_t), hipMemcpyDeviceToHost, stream),
                  "copy counts");
        hip_check(hipStreamSynchronize(stream), "copy state");
        // collect the history entries written by this launch (one wait for all)
        {
            std::vector<std::vector<double>> hv(ninst), ht(ninst);
            bool any = false;
            for (int i = 0; i < ninst; ++i) {
                const int64_t len = std::min(ist[i].hist_len, hist_cap);
                if (len <= 0) continue;
                hv[i].resize(len);
                ht[i].resize(len);
                hip_check(hipMemcpyAsync(hv[i].data(), insts[i].hist, len * sizeof(double), hipMemcpyDeviceToHost,
                                         stream),
                          "hist");
                hip_check(hipMemcpyAsync(ht[i].data(), insts[i].hist_t, len * sizeof(double), hipMemcpyDeviceToHost,
                                         stream),
                          "hist");
                any = true;
            }
            if (any) hip_check(hipStreamSynchronize(stream), "hist");
            for (int i = 0; i < ninst; ++i)
                for (size_t k = 0; k < hv[i].size(); ++k) {
                    hist[i].push_back(hv[i][k]);
                    hist_t[i].push_back(ht[i][k] * tick_s);
                }
        }
        if (sync) {
            std::vector<int> all(ninst);
            std::iota(all.begin(), all.end(), 0);
            for (int i = 0; i < ninst; ++i)
                if (ist[i].result_buf == 1)
                    hip_check(launch_copy(specs[i].h->plan->n, insts[i].x1, insts[i].x0, stream), "copy result");
            exact_relres(all);
            for (int i = 0; i < ninst; ++i) {
                verified[i] = 1;
                // a synchronous solve ran its sweeps: only the verified residual decides
                step[i] = !std::isfinite(relres[i]) ? RAS_STEP_DIVERGED
                          : relres[i] < tol_v[i]    ? RAS_STEP_CONVERGED
                                                    : RAS_STEP_LIMIT;
            }
            break;
        }
        // asynchronous: verify the global criterion after termination (Sec. 3.3.2)
        bool again = false;
        float ms_now = 0.0f;
        hip_check(hipEventRecord(ev1, stream), "event");
        hip_check(hipEventSynchronize(ev1), "event");
        hip_check(hipEventElapsedTime(&ms_now, ev0, ev1), "elapsed");
        std::vector<int> pending;
        for (int i = 0; i < ninst; ++i)
            if (!verified[i]) pending.push_back(i);
        exact_relres(pending);
        for (int i = 0; i < ninst; ++i) {
            if (verified[i]) continue;
            hist[i].push_back(relres[i]);
            hist_t[i].push_back(ms_now * 1e-3);
            int64_t mn = INT64_MAX;
            for (int k = 0; k < insts[i].item_count; ++k) mn = std::min(mn, solves_h[insts[i].item_begin + k]);
            step[i] = ras_async_next_step(ist[i].stop, relres[i], tol_v[i], mn, o.max_sweeps, ms_now * 1e-3,
                                          o.max_seconds, ordered ? 1 : 0);
            if (step[i] != RAS_STEP_RESUME) {
                verified[i] = 1;
                continue;
            }
            // resume: clear this instance's stop flag and its detection flags
            ist[i].stop = 0;
            hip_check(hipMemsetAsync(P.gflag + insts[i].item_begin, 0, insts[i].item_count * sizeof(int32_t), stream),
                      "clear flags");
            hip_check(hipMemsetAsync(P.conv + insts[i].item_begin, 0, insts[i].item_count * sizeof(int32_t), stream),
                      "clear flags");
            again = true;
        }
        if (!again) break;
        if (launch > 10000) {  // give up resuming: report what the last verification found
            for (int i = 0; i < ninst; ++i)
                if (step[i] == RAS_STEP_RESUME) step[i] = RAS_STEP_LIMIT;
            break;
        }
        for (int i = 0; i < ninst; ++i) {
            if (verified[i]) ist[i].stop = 1;  // keep finished systems parked
            ist[i].hist_len = 0;
        }
        hip_check(hipMemcpy(P.ist, ist.data(), ninst * sizeof(InstState), hipMemcpyHostToDevice), "resume state");
    }
    hip_check(hipEventRecord(ev1, stream), "event");
    hip_check(hipEventSynchronize(ev1), "event");
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, ev0, ev1), "elapsed");
    hip_check(hipMemcpy(solves_h.data(), P.solves, nitems * sizeof(int64_t), hipMemcpyDeviceToHost), "copy counts");
    std::vector<int64_t> phase_h(4 * static_cast<size_t>(nitems));
    hip_check(hipMemcpy(phase_h.data(), P.phase, phase_h.size() * sizeof(int64_t), hipMemcpyDeviceToHost),
              "copy phases");

    ras_status status = RAS_OK;
    for (int i = 0; i < ninst; ++i) {
        ras_solve_info& inf = info[i];
        std::memset(&inf, 0, sizeof(inf));
        inf.converged = step[i] == RAS_STEP_CONVERGED;
        inf.launches = launches[i];
        inf.rel_residual = relres[i];
        inf.seconds = ms * 1e-3;
        inf.kernel_seconds = kernel_s;
        int64_t mn = INT64_MAX, mx = 0, tot = 0;
        std::vector<int64_t> cnt(insts[i].item_count);
        for (int k = 0; k < insts[i].item_count; ++k) {
            // synchronous: every subdomain applied exactly `sweeps` updates to the
            // returned iterate (the speculative update of the last sweep is dropped)
            const int64_t c = sync ? ist[i].sweeps : solves_h[insts[i].item_begin + k];
            cnt[k] = c;
            mn = std::min(mn, c);
            mx = std::max(mx, c);
            tot += c;
        }
        inf.min_local_solves = mn;
        inf.max_local_solves = mx;
        inf.total_local_solves = tot;
        inf.sweeps = sync ? ist[i].sweeps : mx;
        ras_handle* h = specs[i].h;
        const int r = specs[i].rhs;
        if (static_cast<int>(h->hist.size()) <= r) {
            h->hist.resize(r + 1);
            h->hist_t.resize(r + 1);
            h->counts.resize(r + 1);
        }
        h->hist[r] = std::move(hist[i]);
        h->hist_t[r] = std::move(hist_t[i]);
        h->counts[r] = std::move(cnt);
        if (static_cast<int>(h->phase_s.size()) <= r) h->phase_s.resize(r + 1);
        std::vector<double> ph(4 * static_cast<size_t>(insts[i].item_count));
        for (size_t k = 0; k < ph.size(); ++k)
            ph[k] = static_cast<double>(phase_h[4 * static_cast<size_t>(insts[i].item_begin) + k]) * tick_s;
        h->phase_s[r] = std::move(ph);
        const ras_status si = ras_final_status(step[i]);
        if (si < 0) status = si;
        else if (si > 0 && status == RAS_OK) status = si;
    }
    if (status == RAS_E_DIVERGED) g_err = "non-finite residual";
    else if (status == RAS_NOT_CONVERGED) g_err = "tolerance not reached within max_sweeps / max_seconds";
    return status;
}

void init_device(ras_handle& h, void* stream) {
    h.stream = static_cast<hipStream_t>(stream);
    hip_check(hipGetDevice(&h.device), "hipGetDevice");
    int khz = 0;
    hip_check(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h.device), "wall clock rate");
    h.clock_khz = khz > 0 ? khz : 100000;
    hip_check(hipDeviceGetAttribute(&h.num_cu, hipDeviceAttributeMultiprocessorCount, h.device), "CU count");
    for (hipEvent_t& e : h.ev.e)
        if (!e) hip_check(hipEventCreate(&e), "event");
}


// ------------------------------------------------------------------------------ serving
// Device bytes a system will hold while admitted: its handle (matrix data,
// factors, global CSR) plus per right-hand side b, x, the local vector and the
// history of the batched solve.
int64_t estimate_device_bytes(const Plan& plan, int nrhs) {
    const bool chol = plan.local.kind == RAS_LOCAL_CHOL_BANDED;
    const int64_t cts = ct_size(plan.local.storage);
    const int64_t sts = plan.local.storage == RAS_STORAGE_FP64 ? 8 : plan.local.storage == RAS_STORAGE_FP32 ? 4 : 2;
    int64_t bytes = (plan.n + 1) * 8 + plan.nnz * 12 + 2048;
    int64_t sum_n = 0;
    for (const auto& sd : plan.subs) {
        const int64_t n = static_cast<int64_t>(sd.omega.size());
        sum_n += n;
        const int64_t ell = n_pad_of(n) * sd.ell_width;
        bytes += 8 * n + ell * (8 + 4 + 4 + (!chol && plan.local.storage == RAS_STORAGE_FP32 ? 4 : 0)) + 512;
        if (chol) bytes += 2 * ((band_elems(n, sd.w) + 63) / 64 * 64) * sts + n * cts + (plan.local.storage == 2 ? 4 * n : 0);
        if (chol && plan.local.storage == RAS_STORAGE_FP16_ROWSCALED && tri_inverse_ok(sd.w, plan.local.storage))
            bytes += 2 * ((n + kBandRows - 1) / kBandRows) * kTriPackBytes;
        // the float64 band of the device factorisation, held while the system is set up
        if (chol && sd.L.empty()) bytes += 8 * n * (sd.w + 1);
        if (plan.local.kind == RAS_LOCAL_CHOL_SPARSE) {
            for (const SparseLanes& q : sd.lanes)
                bytes += 4 * static_cast<int64_t>(q.wave.size()) + static_cast<int64_t>(q.col.size()) * (2 + sts) + 48;
            bytes += n * cts + 2 * kSparseLead * 64 * (2 + sts);
        }
    }
    if (chol) bytes += 2 * kSlabTailBytes;
    // per right-hand side: b, x, local vector, x snapshot (omega plus an external layer,
    // bounded by 2 n_p), history
    bytes += nrhs * (16 * plan.n + sum_n * cts + 2 * 8 * sum_n + 2 * 8 * 65536 + 64 * plan.P);
    return bytes;
}

struct SrvRequest {
    uint64_t ticket = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> va;
    std::vector<int32_t> owner;
    ras_partition part{};
    int32_t overlap = 0;
    ras_local local{};
    std::vector<double> b;
    int nrhs = 1;
    double tol = 1e-8;
    std::chrono::steady_clock::time_point t_submit;
    std::unique_ptr<ras_plan> plan;
    int64_t bytes = 0;
};

struct SrvSystem {
    uint64_t ticket = 0;
    ras_handle* h = nullptr;
    DevBuf b, x;
    std::vector<double> bnorm2;  // ||b||^2 per right-hand side, computed once at admission
    int nrhs = 1;
    int64_t n = 0;
    double tol = 1e-8;
    int64_t bytes = 0;
    std::chrono::steady_clock::time_point t_submit;
    std::vector<ras_solve_info> acc;  // accumulated over slices
    ~SrvSystem() {
        if (h) delete h;
    }
};

struct SrvResult {
    ras_status status = RAS_OK;
    std::string msg;
    std::vector<double> x;
    std::vector<ras_solve_info> info;
    double latency = 0.0;
};

}  // namespace

struct ras_server {
    int64_t budget = 0;
    double slice = 0.02;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_plan, cv_admit, cv_done;
    std::deque<std::unique_ptr<SrvRequest>> submitted, planned;
    std::vector<std::unique_ptr<SrvSystem>> active;
    std::unordered_map<uint64_t, SrvResult> results;
    std::unordered_map<uint64_t, int> state;  // 0 queued, 1 planned, 2 active, 3 done
    uint64_t next_ticket = 1;
    bool stop = false;
    int64_t in_use = 0, peak = 0, slices = 0, submitted_n = 0, completed_n = 0;
    double device_seconds = 0.0;
    DevBuf ws;   // slice workspace, reused (grown when a larger batch needs it)
    DevBuf red;  // reduction slots for the admission norms
    std::thread planner, driver;

    void finish(uint64_t ticket, SrvResult&& r) {
        results[ticket] = std::move(r);
        state[ticket] = 3;
        ++completed_n;
        cv_done.notify_all();
    }

    void plan_loop() {
        for (;;) {
            std::unique_ptr<SrvRequest> rq;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_plan.wait(lk, [&] { return stop || !submitted.empty(); });
                if (stop) return;
                rq = std::move(submitted.front());
                submitted.pop_front();
            }
            SrvResult err;
            try {
                ras_csr A{static_cast<int64_t>(rq->rp.size()) - 1, rq->rp.data(), rq->ci.data(), rq->va.data()};
                if (!rq->owner.empty()) rq->part.owner = rq->owner.data();
                rq->plan = std::make_unique<ras_plan>();
                // partition and overlap here; the factors are computed on the device at admission
                build_plan(&A, &rq->part, rq->overlap, &rq->local, *rq->plan, false);
                rq->bytes = estimate_device_bytes(*rq->plan, rq->nrhs);
                std::vector<int64_t>().swap(rq->rp);
                std::vector<int32_t>().swap(rq->ci);
                std::vector<double>().swap(rq->va);
            } catch (...) {
                std::tie(err.status, err.msg) = current_error();
            }
            std::lock_guard<std::mutex> lk(mu);
            if (err.status != RAS_OK) {
                finish(rq->ticket, std::move(err));
                continue;
            }
            if (rq->bytes > budget) {
                SrvResult r;
                r.status = RAS_E_NOMEM;
                r.msg = "system needs " + std::to_string(rq->bytes) + " device bytes, above the server budget";
                finish(rq->ticket, std::move(r));
                continue;
            }
            state[rq->ticket] = 1;
            planned.push_back(std::move(rq));
            cv_admit.notify_all();
        }
    }

    // Upload one planned request (outside the lock).
    std::unique_ptr<SrvSystem> admit(SrvRequest& rq) {
        auto sys = std::make_unique<SrvSystem>();
        sys->ticket = rq.ticket;
        sys->nrhs = rq.nrhs;
        sys->n = rq.plan->n;
        sys->tol = rq.tol;
        sys->bytes = rq.bytes;
        sys->t_submit = rq.t_submit;
        auto h = std::make_unique<ras_handle>();
        init_device(*h, stream);
        upload(*h, *rq.plan);
        drop_factors(*rq.plan);
        rq.plan->row_ptr.clear();
        rq.plan->col.clear();
        rq.plan->val.clear();
        h->plan = std::move(rq.plan);
        const size_t vb = static_cast<size_t>(sys->nrhs) * sys->n * sizeof(double);
        sys->b.alloc(vb);
        sys->x.alloc(vb);
        hip_check(hipMemcpyAsync(sys->b.p, rq.b.data(), vb, hipMemcpyHostToDevice, stream), "upload b");
        hip_check(hipMemsetAsync(sys->x.p, 0, vb, stream), "clear x");
        // ||b||^2 of every right-hand side, once (the slices reuse it)
        const int nparts = 512;
        red.ensure((2 * nparts + 2 * static_cast<size_t>(sys->nrhs)) * sizeof(double));
        double* r0 = red.as<double>();
        for (int r = 0; r < sys->nrhs; ++r)
            hip_check(launch_residual(sys->n, h->csr_rp.as<int64_t>(), h->csr_ci.as<int32_t>(), h->csr_va.as<double>(),
                                      sys->b.as<double>() + r * sys->n, nullptr, r0, nparts, r0 + 2 * nparts + 2 * r,
                                      stream),
                      "norm of b");
        std::vector<double> out(2 * static_cast<size_t>(sys->nrhs));
        hip_check(hipMemcpyAsync(out.data(), r0 + 2 * nparts, out.size() * sizeof(double), hipMemcpyDeviceToHost, stream),
                  "copy norms");
        hip_check(hipStreamSynchronize(stream), "admit");
        sys->bnorm2.resize(sys->nrhs);
        for (int r = 0; r < sys->nrhs; ++r) sys->bnorm2[r] = out[2 * r + 1];
        sys->h = h.release();
        sys->acc.assign(sys->nrhs, ras_solve_info{});
        return sys;
    }

    // The result of a finished system: the solution copied to the host (no lock
    // held, so submitters and pollers do not wait on the copy).
    SrvResult collect(SrvSystem& sys, ras_status st, const std::string& msg) {
        SrvResult r;
        r.status = st;
        r.msg = msg;
        if (st >= 0) {
            r.x.resize(static_cast<size_t>(sys.nrhs) * sys.n);
            if (hipMemcpy(r.x.data(), sys.x.p, r.x.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
                r.status = RAS_E_HIP;
                r.msg = "copy result";
            }
        }
        r.info = sys.acc;
        r.latency = std::chrono::duration<double>(std::chrono::steady_clock::now() - sys.t_submit).count();
        return r;
    }

    void drive_loop() {
        // without its device the thread still answers every request (RAS_E_HIP)
        const bool device_ok = hipSetDevice(device) == hipSuccess;
        for (;;) {
            // admission by budget: the oldest planned systems that fit
            for (;;) {
                std::unique_ptr<SrvRequest> rq;
                {
                    std::unique_lock<std::mutex> lk(mu);
                    if (stop) return;
                    if (active.empty() && planned.empty()) {
                        cv_admit.wait(lk, [&] { return stop || !planned.empty(); });
                        if (stop) return;
                    }
                    if (planned.empty() || (!active.empty() && in_use + planned.front()->bytes > budget)) break;
                    rq = std::move(planned.front());
                    planned.pop_front();
                    in_use += rq->bytes;
                    peak = std::max(peak, in_use);
                    state[rq->ticket] = 2;
                }
                try {
                    if (!device_ok) throw Error{RAS_E_HIP, "hipSetDevice failed on the server's driver thread"};
                    auto sys = admit(*rq);
                    std::lock_guard<std::mutex> lk(mu);
                    active.push_back(std::move(sys));
                } catch (...) {
                    SrvResult r;
                    std::tie(r.status, r.msg) = current_error();
                    std::lock_guard<std::mutex> lk(mu);
                    in_use -= rq->bytes;
                    finish(rq->ticket, std::move(r));
                }
            }
            // one slice: every admitted system, grouped by local solver
            std::map<std::tuple<int, int, int>, std::vector<SrvSystem*>> groups;
            for (auto& sp : active)
                groups[{sp->h->solver, sp->h->storage, sp->h->cg_iters}].push_back(sp.get());
            const auto t0 = std::chrono::steady_clock::now();
            std::vector<std::pair<SrvSystem*, std::pair<ras_status, std::string>>> done;
            for (auto& kv : groups) {
                std::vector<InstSpec> specs;
                for (SrvSystem* sy : kv.second)
                    for (int r = 0; r < sy->nrhs; ++r)
                        specs.push_back(InstSpec{sy->h, sy->b.as<double>() + r * sy->n, sy->x.as<double>() + r * sy->n,
                                                 r, sy->tol, sy->bnorm2[r]});
                ras_solve_opts o{};
                o.mode = RAS_MODE_ASYNC;
                o.pace = -1.0;  // library choice per local solver
                o.tol = kv.second.front()->tol;
                o.max_sweeps = INT64_MAX / 4;
                o.max_seconds = slice;
                std::vector<ras_solve_info> infos(specs.size());
                ras_status st = RAS_OK;
                std::string msg;
                try {
                    Workspace where;
                    where.reuse = &ws;
                    st = run_solve(specs, o, infos.data(), where);
                } catch (...) {
                    std::tie(st, msg) = current_error();
                }
                size_t k = 0;
                for (SrvSystem* sy : kv.second) {
                    bool all = true;
                    for (int r = 0; r < sy->nrhs; ++r, ++k) {
                        if (st < 0 && st != RAS_E_DIVERGED) {
                            all = false;
                            continue;
                        }
                        ras_solve_info& a = sy->acc[r];
                        const ras_solve_info& f = infos[k];
                        a.converged = f.converged;
                        a.launches += f.launches;
                        a.sweeps += f.sweeps;
                        a.total_local_solves += f.total_local_solves;
                        a.min_local_solves += f.min_local_solves;
                        a.max_local_solves += f.max_local_solves;
                        a.rel_residual = f.rel_residual;
                        a.seconds += f.seconds;
                        a.kernel_seconds += f.kernel_seconds;
                        all = all && f.converged;
                    }
                    if (st < 0 && st != RAS_E_DIVERGED) done.push_back({sy, {st, msg}});
                    else if (all) done.push_back({sy, {RAS_OK, std::string()}});
                    else
                        for (int r = 0; r < sy->nrhs; ++r)
                            if (!std::isfinite(sy->acc[r].rel_residual)) {
                                done.push_back({sy, {RAS_E_DIVERGED, "non-finite residual"}});
                                break;
                            }
                }
            }
            const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            std::vector<SrvResult> outs;
            outs.reserve(done.size());
            for (auto& d : done) {
                try {
                    outs.push_back(collect(*d.first, d.second.first, d.second.second));
                } catch (...) {
                    SrvResult r;
                    std::tie(r.status, r.msg) = current_error();
                    outs.push_back(std::move(r));
                }
            }
            std::lock_guard<std::mutex> lk(mu);
            ++slices;
            device_seconds += dt;
            for (size_t j = 0; j < done.size(); ++j) {
                const auto& d = done[j];
                finish(d.first->ticket, std::move(outs[j]));
                in_use -= d.first->bytes;
                for (size_t i = 0; i < active.size(); ++i)
                    if (active[i].get() == d.first) {
                        active.erase(active.begin() + static_cast<long>(i));
                        break;
                    }
            }
        }
    }
};

namespace {
}  // namespace

extern "C" {

const char* ras_last_error(void) { return g_err.c_str(); }
const char* ras_version(void) { return "ras-mi355x 0.1 (gfx950)"; }

ras_status ras_plan_create(const ras_csr* A, const ras_partition* part, int32_t overlap, const ras_local* local,
                           ras_plan** out) {
    return guarded([&] {
        if (!out) throw Error{RAS_E_ARG, "null output"};
        auto plan = std::make_unique<ras_plan>();
        build_plan(A, part, overlap, local, *plan);
        *out = plan.release();
        return RAS_OK;
    });
}

ras_status ras_plan_get_stats(const ras_plan* plan, ras_plan_stats* out) {
    return guarded([&] {
        if (!plan || !out) throw Error{RAS_E_ARG, "null argument"};
        plan_stats(*plan, out);
        return RAS_OK;
    });
}

static void copy_sets(const Plan& plan, int32_t* owner, int64_t* omega_ptr, int32_t* omega_idx) {
    if (owner) std::copy(plan.owner.begin(), plan.owner.end(), owner);
    int64_t acc = 0;
    if (omega_ptr) omega_ptr[0] = 0;
    for (int p = 0; p < plan.P; ++p) {
        const auto& om = plan.subs[p].omega;
        if (omega_idx) std::copy(om.begin(), om.end(), omega_idx + acc);
        acc += static_cast<int64_t>(om.size());
        if (omega_ptr) omega_ptr[p + 1] = acc;
    }
}

ras_status ras_plan_sets(const ras_plan* plan, int32_t* owner, int64_t* omega_ptr, int32_t* omega_idx) {
    return guarded([&] {
        if (!plan) throw Error{RAS_E_ARG, "null plan"};
        copy_sets(*plan, owner, omega_ptr, omega_idx);
        return RAS_OK;
    });
}

ras_status ras_plan_comm_volume(const ras_plan* plan, int64_t* volume) {
    return guarded([&] {
        if (!plan || !volume) throw Error{RAS_E_ARG, "null argument"};
        comm_volume(*plan, volume);
        return RAS_OK;
    });
}

int64_t ras_sparse_max_rows(int32_t storage) {
    if (storage == RAS_STORAGE_FP64) return static_cast<int64_t>(kLdsLimit / sizeof(double));
    if (storage == RAS_STORAGE_FP32) return static_cast<int64_t>(kLdsLimit / sizeof(float));
    return 0;
}

ras_status ras_plan_sparse_factor(const ras_plan* plan, int32_t p, int32_t* perm, int64_t* row_ptr, int32_t* col,
                                  double* val, double* diag, int64_t* nnz) {
    return guarded([&] {
        if (!plan) throw Error{RAS_E_ARG, "null plan"};
        if (p < 0 || p >= plan->P) throw Error{RAS_E_ARG, "subdomain out of range"};
        if (plan->local.kind != RAS_LOCAL_CHOL_SPARSE) throw Error{RAS_E_STATE, "plan has no sparse factors"};
        const SparseFactor& F = plan->subs[p].sf;
        if (F.perm.size() != plan->subs[p].omega.size()) throw Error{RAS_E_STATE, "factor released"};
        if (nnz) *nnz = static_cast<int64_t>(F.lj.size());
        if (perm) std::copy(F.perm.begin(), F.perm.end(), perm);
        if (row_ptr) std::copy(F.lp.begin(), F.lp.end(), row_ptr);
        if (col) std::copy(F.lj.begin(), F.lj.end(), col);
        if (val) std::copy(F.lx.begin(), F.lx.end(), val);
        if (diag) std::copy(F.d.begin(), F.d.end(), diag);
        return RAS_OK;
    });
}

ras_status ras_plan_sparse_schedule(const ras_plan* plan, int32_t p, int32_t pass, int32_t* nsteps, int64_t* nrec,
                                    int64_t* nent, int32_t* slots, int32_t* min_block, int32_t* step_ptr,
                                    int32_t* meta, int32_t* col, double* val) {
    return guarded([&] {
        if (!plan) throw Error{RAS_E_ARG, "null plan"};
        if (p < 0 || p >= plan->P) throw Error{RAS_E_ARG, "subdomain out of range"};
        if (pass != 0 && pass != 1) throw Error{RAS_E_ARG, "pass must be 0 (forward) or 1 (backward)"};
        if (plan->local.kind != RAS_LOCAL_CHOL_SPARSE) throw Error{RAS_E_STATE, "plan has no sparse factors"};
        const Subdomain& sd = plan->subs[p];
        const SparseSchedule& q = sd.sched[pass];
        if (q.step.empty()) throw Error{RAS_E_STATE, "schedule released"};
        if (nsteps) *nsteps = static_cast<int32_t>(q.step.size()) - 1;
        if (nrec) *nrec = static_cast<int64_t>(q.meta.size() / 4);
        if (nent) *nent = static_cast<int64_t>(q.col.size());
        if (slots) *slots = q.slots;
        if (min_block) *min_block = sd.min_block;
        if (step_ptr) std::copy(q.step.begin(), q.step.end(), step_ptr);
        if (meta) std::copy(q.meta.begin(), q.meta.end(), meta);
        if (col) std::copy(q.col.begin(), q.col.end(), col);
        if (val) std::copy(q.val.begin(), q.val.end(), val);
        return RAS_OK;
    });
}

ras_status ras_plan_sparse_lanes(const ras_plan* plan, int32_t p, int32_t pass, int32_t* waves, int64_t* nitems,
                                 int32_t* wave, int32_t* col, double* val) {
    return guarded([&] {
        if (!plan) throw Error{RAS_E_ARG, "null plan"};
        if (p < 0 || p >= plan->P) throw Error{RAS_E_ARG, "subdomain out of range"};
        if (pass != 0 && pass != 1) throw Error{RAS_E_ARG, "pass must be 0 (forward) or 1 (backward)"};
        if (plan->local.kind != RAS_LOCAL_CHOL_SPARSE) throw Error{RAS_E_STATE, "plan has no sparse factors"};
        const SparseLanes& q = plan->subs[p].lanes[pass];
        if (q.wave.empty()) throw Error{RAS_E_STATE, "schedule released"};
        if (waves) *waves = kSparseWaves;
        if (nitems) *nitems = static_cast<int64_t>(q.col.size());
        if (wave) std::copy(q.wave.begin(), q.wave.end(), wave);
        if (col) std::copy(q.col.begin(), q.col.end(), col);
        if (val) std::copy(q.val.begin(), q.val.end(), val);
        return RAS_OK;
    });
}

ras_status ras_plan_factor(const ras_plan* plan, int32_t p, double* band, int32_t* w) {
    return guarded([&] {
        if (!plan || !w) throw Error{RAS_E_ARG, "null argument"};
        if (p < 0 || p >= plan->P) throw Error{RAS_E_ARG, "subdomain out of range"};
        const auto& s = plan->subs[p];
        *w = s.w;
        if (!band) return RAS_OK;
        if (plan->local.kind != RAS_LOCAL_CHOL_BANDED) throw Error{RAS_E_STATE, "plan has no Cholesky factors"};
        if (s.L.empty() && !s.omega.empty()) throw Error{RAS_E_STATE, "factor released"};
        *w = s.w;
        if (band) std::copy(s.L.begin(), s.L.end(), band);
        return RAS_OK;
    });
}

ras_status ras_plan_factor_fp16(const ras_plan* plan, int32_t p, uint16_t* half_bits, float* scale) {
    return guarded([&] {
        if (!plan) throw Error{RAS_E_ARG, "null plan"};
        if (plan->local.kind != RAS_LOCAL_CHOL_BANDED || plan->local.storage != RAS_STORAGE_FP16_ROWSCALED)
            throw Error{RAS_E_STATE, "plan has no FP16 row-scaled factors"};
        if (p < 0 || p >= plan->P) throw Error{RAS_E_ARG, "subdomain out of range"};
        const auto& s = plan->subs[p];
        if (half_bits) std::copy(s.Lh.begin(), s.Lh.end(), half_bits);
        if (scale) std::copy(s.scale.begin(), s.scale.end(), scale);
        return RAS_OK;
    });
}

void ras_plan_destroy(ras_plan* plan) { delete plan; }

ras_status ras_setup_from_plan(const ras_plan* plan, void* hip_stream, ras_handle** out) {
    return guarded([&] {
        if (!plan || !out) throw Error{RAS_E_ARG, "null argument"};
        auto h = std::make_unique<ras_handle>();
        init_device(*h, hip_stream);
        upload(*h, *plan);
        h->plan = std::make_unique<ras_plan>();
        Plan& keep = *h->plan;
        keep.n = plan->n;
        keep.nnz = plan->nnz;
        keep.P = plan->P;
        keep.overlap = plan->overlap;
        keep.local = plan->local;
        keep.owner = plan->owner;
        keep.subs.resize(plan->P);
        for (int p = 0; p < plan->P; ++p) {
            keep.subs[p].omega = plan->subs[p].omega;
            keep.subs[p].w = plan->subs[p].w;
            keep.subs[p].ell_width = plan->subs[p].ell_width;
            keep.subs[p].n_owned = plan->subs[p].n_owned;
        }
        hip_check(hipDeviceSynchronize(), "upload");
        *out = h.release();
        return RAS_OK;
    });
}

ras_status ras_setup(const ras_csr* A, const ras_partition* part, int32_t overlap, const ras_local* local,
                     void* hip_stream, ras_handle** out) {
    return guarded([&] {
        if (!out) throw Error{RAS_E_ARG, "null output"};
        auto plan = std::make_unique<ras_plan>();
        build_plan(A, part, overlap, local, *plan, false);  // banded factors: on the device, in upload
        auto h = std::make_unique<ras_handle>();
        init_device(*h, hip_stream);
        upload(*h, *plan);
        drop_factors(*plan);
        plan->row_ptr.clear();
        plan->col.clear();
        plan->val.clear();
        h->plan = std::move(plan);
        hip_check(hipDeviceSynchronize(), "upload");
        *out = h.release();
        return RAS_OK;
    });
}

ras_status ras_handle_get_stats(const ras_handle* h, ras_plan_stats* out) {
    return guarded([&] {
        if (!h || !out) throw Error{RAS_E_ARG, "null argument"};
        *out = h->stats;
        return RAS_OK;
    });
}

ras_status ras_solve(ras_handle* h, const double* b_dev, double* x_dev, int32_t nrhs, const ras_solve_opts* opts,
                     ras_solve_info* info) {
    return guarded([&] {
        if (!h || !b_dev || !x_dev || !opts || !info || nrhs < 1) throw Error{RAS_E_ARG, "invalid argument"};
        std::vector<InstSpec> specs;
        for (int r = 0; r < nrhs; ++r)
            specs.push_back(InstSpec{h, b_dev + static_cast<int64_t>(r) * h->plan->n,
                                     x_dev + static_cast<int64_t>(r) * h->plan->n, r});
        h->hist.clear();
        h->hist_t.clear();
        h->counts.clear();
        return run_solve(specs, *opts, info);
    });
}

ras_status ras_solve_noalloc(ras_handle* h, const double* b_dev, double* x_dev, int32_t nrhs,
                             const ras_solve_opts* opts, ras_solve_info* info) {
    return guarded([&] {
        if (!h || !b_dev || !x_dev || !opts || !info || nrhs < 1) throw Error{RAS_E_ARG, "invalid argument"};
        hip_check(hipSetDevice(h->device), "hipSetDevice");
        Workspace where;
        hip_check(noalloc_scratch(&where.fixed), "address of the no-allocation scratch");
        where.fixed_bytes = kNoAllocScratchBytes;
        std::vector<InstSpec> specs;
        for (int r = 0; r < nrhs; ++r)
            specs.push_back(InstSpec{h, b_dev + static_cast<int64_t>(r) * h->plan->n,
                                     x_dev + static_cast<int64_t>(r) * h->plan->n, r});
        h->hist.clear();
        h->hist_t.clear();
        h->counts.clear();
        return run_solve(specs, *opts, info, where);
    });
}

ras_status ras_batch_solve(int32_t m, ras_handle* const* hs, const double* const* b_dev, double* const* x_dev,
                           const int32_t* nrhs, const ras_solve_opts* opts, ras_solve_info* info) {
    return guarded([&] {
        if (m < 1 || !hs || !b_dev || !x_dev || !nrhs || !opts || !info) throw Error{RAS_E_ARG, "invalid argument"};
        std::vector<InstSpec> specs;
        for (int k = 0; k < m; ++k) {
            if (!hs[k] || !b_dev[k] || !x_dev[k] || nrhs[k] < 1) throw Error{RAS_E_ARG, "invalid batch entry"};
            if (hs[k]->stream != hs[0]->stream) throw Error{RAS_E_ARG, "batched handles must share a stream"};
            hs[k]->hist.clear();
            hs[k]->hist_t.clear();
            hs[k]->counts.clear();
            for (int r = 0; r < nrhs[k]; ++r)
                specs.push_back(InstSpec{hs[k], b_dev[k] + static_cast<int64_t>(r) * hs[k]->plan->n,
                                         x_dev[k] + static_cast<int64_t>(r) * hs[k]->plan->n, r});
        }
        return run_solve(specs, *opts, info);
    });
}

ras_status ras_residual_history(const ras_handle* h, int32_t rhs, double* t_sec, double* relres, int64_t cap,
                                 int64_t* len) {
    return guarded([&] {
        if (!h || !len) throw Error{RAS_E_ARG, "null argument"};
        if (rhs < 0 || rhs >= static_cast<int32_t>(h->hist.size())) throw Error{RAS_E_STATE, "no history for this rhs"};
        const auto& hv = h->hist[rhs];
        const auto& ht = h->hist_t[rhs];
        *len = static_cast<int64_t>(hv.size());
        const int64_t c = std::min<int64_t>(cap, *len);
        if (relres) std::copy(hv.begin(), hv.begin() + c, relres);
        if (t_sec) std::copy(ht.begin(), ht.begin() + c, t_sec);
        return RAS_OK;
    });
}

ras_status ras_local_solve_counts(const ras_handle* h, int32_t rhs, int64_t* counts) {
    return guarded([&] {
        if (!h || !counts) throw Error{RAS_E_ARG, "null argument"};
        if (rhs < 0 || rhs >= static_cast<int32_t>(h->counts.size())) throw Error{RAS_E_STATE, "no counts for this rhs"};
        std::copy(h->counts[rhs].begin(), h->counts[rhs].end(), counts);
        return RAS_OK;
    });
}

ras_status ras_partition_sets(const ras_handle* h, int32_t* owner, int64_t* omega_ptr, int32_t* omega_idx) {
    return guarded([&] {
        if (!h) throw Error{RAS_E_ARG, "null handle"};
        copy_sets(*h->plan, owner, omega_ptr, omega_idx);
        return RAS_OK;
    });
}

ras_status ras_phase_seconds(const ras_handle* h, int32_t rhs, double* seconds) {
    return guarded([&] {
        if (!h || !seconds) throw Error{RAS_E_ARG, "null argument"};
        if (rhs < 0 || rhs >= static_cast<int32_t>(h->phase_s.size()) || h->phase_s[rhs].empty())
            throw Error{RAS_E_STATE, "no solve recorded for this rhs"};
        std::copy(h->phase_s[rhs].begin(), h->phase_s[rhs].end(), seconds);
        return RAS_OK;
    });
}

ras_status ras_handle_factor(const ras_handle* h, int32_t p, double* band, int32_t* w) {
    return guarded([&] {
        if (!h || !w) throw Error{RAS_E_ARG, "null argument"};
        if (h->solver != RAS_LOCAL_CHOL_BANDED) throw Error{RAS_E_STATE, "the local solver is not banded Cholesky"};
        if (p < 0 || p >= static_cast<int32_t>(h->subs.size())) throw Error{RAS_E_ARG, "subdomain out of range"};
        const SubDev& d = h->subs[p];
        *w = d.w;
        if (!band) return RAS_OK;
        hip_check(hipSetDevice(h->device), "hipSetDevice");
        const int64_t n = d.n, ld = d.w + 1;
        const size_t sts = h->storage == RAS_STORAGE_FP64 ? 8 : h->storage == RAS_STORAGE_FP32 ? 4 : 2;
        const size_t cts = ct_size(h->storage);
        const int64_t elems = band_elems(n, d.w);
        std::vector<unsigned char> bf(elems * sts), iv(n * cts);
        std::vector<float> sc(n, 1.0f);
        hip_check(hipStreamSynchronize(h->stream), "sync");
        hip_check(hipMemcpy(bf.data(), d.band_f, bf.size(), hipMemcpyDeviceToHost), "copy band");
        hip_check(hipMemcpy(iv.data(), d.invd, iv.size(), hipMemcpyDeviceToHost), "copy invd");
        if (d.scale) hip_check(hipMemcpy(sc.data(), d.scale, n * sizeof(float), hipMemcpyDeviceToHost), "copy scale");
        auto entry = [&](int64_t i) -> double {
            if (h->storage == RAS_STORAGE_FP64) return reinterpret_cast<const double*>(bf.data())[i];
            if (h->storage == RAS_STORAGE_FP32) return reinterpret_cast<const float*>(bf.data())[i];
            _Float16 hv;
            std::memcpy(&hv, bf.data() + 2 * i, 2);
            return static_cast<double>(static_cast<float>(hv));
        };
        for (int64_t t = 0; t < n; ++t) {
            const double rs = h->storage == RAS_STORAGE_FP16_ROWSCALED ? static_cast<double>(sc[t]) : 1.0;
            for (int64_t o = 0; o < d.w; ++o) {
                const int64_t di = d.slab ? ((t / kBandRows) * d.w + o) * kBandRows + t % kBandRows : t * ld + o;
                band[t * ld + o] = entry(di) * rs;
            }
            const double inv = h->storage == RAS_STORAGE_FP64 ? reinterpret_cast<const double*>(iv.data())[t]
                                                               : reinterpret_cast<const float*>(iv.data())[t];
            band[t * ld + d.w] = 1.0 / inv;
        }
        if (d.tri_inv && h->storage != RAS_STORAGE_FP16_ROWSCALED) {
            // the triangle slots hold G = T^-1 per 32-row block (diagonal: the reciprocals
            // just read); invert back in float64 to report the factor's own triangle
            constexpr int BR = kBandRows;
            for (int64_t t0 = 0; t0 < n; t0 += BR) {
                const int nb = static_cast<int>(std::min<int64_t>(BR, n - t0));
                double G[BR][BR], T[BR][BR];
                for (int r = 0; r < nb; ++r)
                    for (int c = 0; c < nb; ++c)
                        G[r][c] = c > r ? 0.0 : c == r ? 1.0 / band[(t0 + r) * ld + d.w]
                                                       : band[(t0 + r) * ld + (c - r + d.w)];
                for (int m = 0; m < nb; ++m)
                    for (int r = 0; r < nb; ++r) {
                        if (r < m) {
                            T[r][m] = 0.0;
                            continue;
                        }
                        double s = r == m ? 1.0 : 0.0;
                        for (int k = m; k < r; ++k) s -= G[r][k] * T[k][m];
                        T[r][m] = s / G[r][r];
                    }
                for (int r = 0; r < nb; ++r)
                    for (int c = 0; c < r; ++c) band[(t0 + r) * ld + (c - r + d.w)] = T[r][c];
            }
        }
        return RAS_OK;
    });
}

ras_status ras_relative_residual(ras_handle* h, const double* b_dev, const double* x_dev, double* relres) {
    return guarded([&] {
        if (!h || !b_dev || !x_dev || !relres) throw Error{RAS_E_ARG, "null argument"};
        hip_check(hipSetDevice(h->device), "hipSetDevice");
        const int nparts = 512;
        h->ws_red.ensure((2 * nparts + 2) * sizeof(double));
        double* red = h->ws_red.as<double>();
        hip_check(launch_residual(h->plan->n, h->csr_rp.as<int64_t>(), h->csr_ci.as<int32_t>(), h->csr_va.as<double>(),
                                  b_dev, x_dev, red, nparts, red + 2 * nparts, h->stream),
                  "residual");
        double out[2];
        hip_check(hipMemcpyAsync(out, red + 2 * nparts, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy");
        hip_check(hipStreamSynchronize(h->stream), "sync");
        *relres = std::sqrt(out[0] / out[1]);
        return RAS_OK;
    });
}

void ras_destroy(ras_handle* h) { delete h; }

ras_status ras_pause(ras_handle* h, int32_t p, int32_t paused) {
    return guarded([&] {
        if (!h || !h->ctl.host) throw Error{RAS_E_ARG, "null handle"};
        if (p < 0 || p >= h->plan->P) throw Error{RAS_E_ARG, "subdomain out of range"};
        __atomic_store_n(h->ctl.host + 1 + p, paused ? 1 : 0, __ATOMIC_SEQ_CST);
        return RAS_OK;
    });
}

ras_status ras_cancel(ras_handle* h) {
    return guarded([&] {
        if (!h || !h->ctl.host) throw Error{RAS_E_ARG, "null handle"};
        __atomic_store_n(h->ctl.host, 1, __ATOMIC_SEQ_CST);
        return RAS_OK;
    });
}

ras_status ras_autotune(ras_handle* h, const double* b_dev, double* x_dev, int32_t sweeps, int32_t* best_team,
                        double* best_ms_per_sweep) {
    return guarded([&] {
        if (!h || !b_dev || !x_dev || sweeps < 1) throw Error{RAS_E_ARG, "invalid argument"};
        hip_check(hipSetDevice(h->device), "hipSetDevice");
        int best = 1;
        double best_ms = INFINITY;
        if (h->solver == RAS_LOCAL_CG) {
            // two rounds over the feasible team sizes, the faster of each size's two
            // timings counts (the first launch of a kernel variant carries one-time costs)
            double ms_of[5] = {INFINITY, INFINITY, INFINITY, INFINITY, INFINITY};
            for (int round = 0; round < 2; ++round) {
                for (int t = 0; t < 5; ++t) {
                    const int T = kTeamSizes[t];
                    if (round == 1 && !(ms_of[t] < INFINITY)) continue;
                    ras_solve_opts o{};
                    o.mode = RAS_MODE_SYNC;
                    o.tol = 0.0;
                    o.max_sweeps = sweeps;
                    o.team = T;
                    hip_check(hipMemsetAsync(x_dev, 0, h->plan->n * sizeof(double), h->stream), "clear x");
                    std::vector<InstSpec> specs{InstSpec{h, b_dev, x_dev, 0}};
                    ras_solve_info info{};
                    try {
                        run_solve(specs, o, &info);
                    } catch (const Error& e) {
                        if (e.status == RAS_E_UNSUPPORTED) continue;  // infeasible team size for this shape
                        throw;
                    }
                    ms_of[t] = std::min(ms_of[t], 1e3 * info.kernel_seconds / (sweeps + 1));
                }
            }
            for (int t = 0; t < 5; ++t)
                if (ms_of[t] < best_ms) {
                    best_ms = ms_of[t];
                    best = kTeamSizes[t];
                }
            h->tuned_team = best;
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[{h->plan->n, h->plan->P, h->max_n, h->uniform_K, h->storage, h->cg_iters}] = best;
        } else {
            ras_solve_opts o{};
            o.mode = RAS_MODE_SYNC;
            o.tol = 0.0;
            o.max_sweeps = sweeps;
            hip_check(hipMemsetAsync(x_dev, 0, h->plan->n * sizeof(double), h->stream), "clear x");
            std::vector<InstSpec> specs{InstSpec{h, b_dev, x_dev, 0}};
            ras_solve_info info{};
            run_solve(specs, o, &info);
            best_ms = 1e3 * info.kernel_seconds / (sweeps + 1);
        }
        h->hist.clear();
        h->hist_t.clear();
        h->counts.clear();
        if (best_team) *best_team = best;
        if (best_ms_per_sweep) *best_ms_per_sweep = best_ms;
        return RAS_OK;
    });
}


ras_status ras_server_create(int64_t hbm_budget, double slice_seconds, void* hip_stream, ras_server** out) {
    return guarded([&] {
        if (!out || hbm_budget <= 0 || !(slice_seconds > 0.0)) throw Error{RAS_E_ARG, "invalid server arguments"};
        auto srv = std::make_unique<ras_server>();
        srv->budget = hbm_budget;
        srv->slice = slice_seconds;
        hip_check(hipGetDevice(&srv->device), "hipGetDevice");
        if (hip_stream) {
            srv->stream = static_cast<hipStream_t>(hip_stream);
        } else {
            hip_check(hipStreamCreate(&srv->stream), "hipStreamCreate");
            srv->own_stream = true;
        }
        ras_server* p = srv.get();
        p->planner = std::thread([p] { p->plan_loop(); });
        p->driver = std::thread([p] { p->drive_loop(); });
        *out = srv.release();
        return RAS_OK;
    });
}

ras_status ras_server_submit(ras_server* srv, const ras_csr* A, const ras_partition* part, int32_t overlap,
                             const ras_local* local, const double* b_host, int32_t nrhs, double tol,
                             uint64_t* ticket) {
    return guarded([&] {
        if (!srv || !A || !part || !local || !b_host || nrhs < 1 || !ticket || !(tol >= 0.0) || A->n < 1 ||
            !A->row_ptr || !A->col || !A->val)
            throw Error{RAS_E_ARG, "invalid submission"};
        auto rq = std::make_unique<SrvRequest>();
        const int64_t n = A->n, nnz = A->row_ptr[n];
        if (nnz < 0) throw Error{RAS_E_PATTERN, "row_ptr[n] < 0"};
        rq->rp.assign(A->row_ptr, A->row_ptr + n + 1);
        rq->ci.assign(A->col, A->col + nnz);
        rq->va.assign(A->val, A->val + nnz);
        rq->part = *part;
        if (part->kind == RAS_PART_EXPLICIT && part->owner) rq->owner.assign(part->owner, part->owner + n);
        rq->part.owner = nullptr;
        rq->overlap = overlap;
        rq->local = *local;
        rq->b.assign(b_host, b_host + n * nrhs);
        rq->nrhs = nrhs;
        rq->tol = tol;
        rq->t_submit = std::chrono::steady_clock::now();
        std::lock_guard<std::mutex> lk(srv->mu);
        rq->ticket = srv->next_ticket++;
        *ticket = rq->ticket;
        srv->state[rq->ticket] = 0;
        ++srv->submitted_n;
        srv->submitted.push_back(std::move(rq));
        srv->cv_plan.notify_one();
        return RAS_OK;
    });
}

ras_status ras_server_poll(ras_server* srv, uint64_t ticket, double* x_host, ras_solve_info* info,
                           double* latency_seconds) {
    return guarded([&] {
        if (!srv) throw Error{RAS_E_ARG, "null server"};
        std::lock_guard<std::mutex> lk(srv->mu);
        auto st = srv->state.find(ticket);
        if (st == srv->state.end()) throw Error{RAS_E_ARG, "unknown ticket"};
        if (st->second != 3) return RAS_PENDING;
        SrvResult& r = srv->results[ticket];
        const ras_status status = r.status;
        if (status < 0) {
            g_err = r.msg;
        } else {
            if (x_host) std::copy(r.x.begin(), r.x.end(), x_host);
            if (info) std::copy(r.info.begin(), r.info.end(), info);
        }
        if (latency_seconds) *latency_seconds = r.latency;
        srv->results.erase(ticket);
        srv->state.erase(st);
        return status;
    });
}

ras_status ras_server_wait(ras_server* srv, uint64_t ticket, double timeout_seconds) {
    return guarded([&] {
        if (!srv) throw Error{RAS_E_ARG, "null server"};
        std::unique_lock<std::mutex> lk(srv->mu);
        auto ready = [&] {
            auto st = srv->state.find(ticket);
            return st == srv->state.end() || st->second == 3;
        };
        const bool ok = srv->cv_done.wait_for(lk, std::chrono::duration<double>(std::max(0.0, timeout_seconds)), ready);
        return ok ? RAS_OK : RAS_PENDING;
    });
}

ras_status ras_server_get_stats(ras_server* srv, ras_server_stats* out) {
    return guarded([&] {
        if (!srv || !out) throw Error{RAS_E_ARG, "null argument"};
        std::lock_guard<std::mutex> lk(srv->mu);
        out->submitted = srv->submitted_n;
        out->completed = srv->completed_n;
        out->queued = static_cast<int64_t>(srv->submitted.size() + srv->planned.size());
        out->active = static_cast<int64_t>(srv->active.size());
        out->slices = srv->slices;
        out->in_use_bytes = srv->in_use;
        out->peak_in_use_bytes = srv->peak;
        out->budget_bytes = srv->budget;
        out->device_seconds = srv->device_seconds;
        return RAS_OK;
    });
}

ras_status ras_server_destroy(ras_server* srv) {
    if (!srv) return RAS_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_plan.notify_all();
    srv->cv_admit.notify_all();
    if (srv->planner.joinable()) srv->planner.join();
    if (srv->driver.joinable()) srv->driver.join();
    srv->active.clear();
    ras_status st = RAS_OK;
    if (srv->own_stream && hipStreamDestroy(srv->stream) != hipSuccess) st = fail(RAS_E_HIP, "hipStreamDestroy");
    delete srv;
    return st;
}


}  // extern "C"
