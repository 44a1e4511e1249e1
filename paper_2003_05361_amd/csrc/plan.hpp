// Host-side setup of the restricted additive Schwarz solver (no GPU code).
//
// Builds, from the global CSR matrix and a partition description, the
// per-subdomain data the device kernels consume: owned and overlapping index
// sets (Sec. 3.2.1, Sec. 2.1 Fig. 1), the rows of A on each overlapping set
// (Sec. 3.2.2) and, for the direct local solver, the float64 banded Cholesky
// factor of each local matrix (Sec. 3.3.1).
#pragma once

#include <atomic>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ras.h"

namespace ras {

// Sparse Cholesky factor of a local matrix in elimination order: row k of the
// permuted matrix is row perm[k] of Omega_p's local matrix (ascending global id).
struct SparseFactor {
    std::vector<int32_t> perm;   // elimination order -> position in omega
    std::vector<int64_t> lp;     // [n + 1] rows of the strictly lower part of L
    std::vector<int32_t> lj;     // column of each entry, ascending within a row
    std::vector<double> lx;
    std::vector<int64_t> cp;     // [n + 1] the same entries by columns (rows ascending)
    std::vector<int32_t> ci;
    std::vector<double> cx;
    std::vector<double> d;       // diagonal of L
};

// One triangular pass of a sparse factor as a sequence of parallel steps: the
// records of a step read only values written in earlier steps, and each writes
// one value, the dot product of its entries with the vector (kept in LDS).
// Value slots [0, n) are the rows of the local vector in elimination order;
// slots n.. hold the partial results of dense diagonal blocks between their
// two steps.
struct SparseSchedule {
    std::vector<int32_t> step;   // [nsteps + 1] record ranges of the steps
    std::vector<int32_t> meta;   // 4 per record: slot written, first entry, end of entries, 0
    std::vector<int32_t> col;    // slot read by each entry
    std::vector<double> val;
    int32_t slots = 0;           // value slots beyond n
};

// A schedule dealt out to the lanes of one workgroup (the device layout of a
// pass): wave w's rounds are wave[2w] .. wave[2w] + wave[2w+1] - 1, round r's
// items col / val[r * 64 + lane]; see kSparseWaves for the item semantics.
struct SparseLanes {
    std::vector<int32_t> wave;
    std::vector<uint16_t> col;
    std::vector<double> val;  // a terminator's value holds dest | g << 24 in its low 32 bits
};

struct Subdomain {
    std::vector<int32_t> omega;  // overlapping set, ascending global ids
    std::vector<uint8_t> owned;  // owned[i] != 0 iff omega[i] is owned by this subdomain
    int32_t n_owned = 0;
    int32_t ell_width = 0;       // max stored entries in a row of A over omega
    int32_t w = 0;               // lower half-bandwidth of A[omega, omega]
    std::vector<double> L;       // Cholesky: row-major lower band, L[i*(w+1) + (j-i+w)]
    std::vector<uint16_t> Lh;    // FP16_ROWSCALED: float16 bits of L / scale(row)
    std::vector<float> scale;    // FP16_ROWSCALED: per-row scale
    SparseFactor sf;             // sparse Cholesky solver only
    SparseSchedule sched[2];     // sparse Cholesky: forward (L) and backward (L^T) passes
    SparseLanes lanes[2];        // the same passes in the device's lane layout
    int32_t min_block = 0;       // sparse Cholesky: smallest dense block solved by its inverse (0: none)
};

struct Plan {
    int64_t n = 0;
    int64_t nnz = 0;
    int32_t P = 0;
    int32_t overlap = 0;
    ras_local local{};
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    std::vector<int32_t> owner;
    std::vector<Subdomain> subs;
};

// Thrown inside the library only; the C entry points turn it into a status.
struct Error {
    ras_status status;
    std::string msg;
};

void validate_csr(const ras_csr& A);
std::vector<int32_t> make_owner(const ras_csr& A, const ras_partition& part, int32_t* P_out);
void build_overlap(Plan& plan);
// ext(Omega_p): columns stored in Omega_p's rows that lie outside Omega_p (ascending, unique)
std::vector<int32_t> external_set(const Plan& plan, const Subdomain& sd);
// volume[p*P + q] = |(Omega_p u ext(Omega_p)) n O_q| for q != p, 0 on the diagonal
void comm_volume(const Plan& plan, int64_t* volume);
void factor_local(Plan& plan);
// Robin transmission (ORAS): the local matrix's diagonal is reduced by this
// factor times the row's coupling to points outside the subdomain (0: Dirichlet)
inline double robin_shift_factor(const ras_local& l) {
    return l.transmission == RAS_TRANSMISSION_ROBIN ? 1.0 - l.robin_q : 0.0;
}
// float64 banded Cholesky factor of one subdomain's local matrix on the host (sd.L)
void factor_one(const Plan& plan, Subdomain& sd, int32_t p);
// Sparse factors and their solve schedules; lds_bytes bounds each subdomain's
// vector plus block slots, value_bytes is the size of one value in LDS
void sparse_factor_local(Plan& plan, size_t lds_bytes, size_t value_bytes);
// Dense diagonal blocks of a sparse factor: maximal runs [s_i, s_{i+1}) of
// consecutive rows whose diagonal block of L is a full triangle
std::vector<int32_t> dense_runs(const SparseFactor& F);
// Schedule of one pass; blocks of at least min_block rows (0: none) are solved by
// the explicit inverse of their diagonal triangle
void sparse_schedule(const SparseFactor& F, const std::vector<int32_t>& runs, int32_t min_block, bool forward,
                     SparseSchedule* out);
// Lane layout of a schedule: the records of each step dealt out to the lanes
// longest first, each to the least loaded lane, and the lanes grouped into
// waves by load
void pack_schedule(const SparseSchedule& q, SparseLanes* out);
uint16_t f64_to_f16_rne(double d);

uint64_t splitmix64_next(uint64_t& state);

int worker_count();

// Runs f(i, worker) for i in [0, count) on up to worker_count() threads.
template <class F>
inline void parallel_for(int64_t count, F&& f) {
    int nw = static_cast<int>(std::min<int64_t>(worker_count(), count));
    if (nw <= 1) {
        for (int64_t i = 0; i < count; ++i) f(i, 0);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<std::thread> ts;
    std::vector<Error> errs(nw, Error{RAS_OK, {}});
    for (int t = 0; t < nw; ++t) {
        ts.emplace_back([&, t] {
            try {
                for (int64_t i; (i = next.fetch_add(1)) < count;) f(i, t);
            } catch (const Error& e) {
                errs[t] = e;
                next.store(count);
            }
        });
    }
    for (auto& th : ts) th.join();
    for (auto& e : errs)
        if (e.status != RAS_OK) throw e;
}


}  // namespace ras
