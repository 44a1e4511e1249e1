// Device-side data layout shared by the upload code and the kernels.
//
// Everything the persistent kernels touch lives in HBM in flat arrays owned by
// a handle (matrix data) or by a solve (per right-hand side state).  A "work
// item" is one subdomain of one right-hand side; a launch processes a table of
// items that may come from several systems (batching).
#pragma once

#include <cstddef>
#include <cstdint>

#include "../../include/ras.h"

namespace ras {

constexpr int kCgThreads = 256;     // workgroup size of the CG kernels
constexpr int kMaxTeam = 16;        // workgroups cooperating on one subdomain (CG)
constexpr int kTeamSizes[5] = {1, 2, 4, 8, 16};
constexpr int kBandThreads = 512;   // workgroup size of the banded-solve kernels
constexpr int kBandRows = 32;       // rows per block of the banded triangular solves
// Block-transposed ("slab") factor layout, used for half-bandwidths up to
// kSlabMaxW: the factor is cut into blocks of kBandRows rows and block j is
// stored as the dense array S_j[o][r] = L[j*kBandRows + r][o] (o < w: the w
// sub-diagonal offsets of the row, r < kBandRows: the row in the block), zero
// for rows past n; the diagonal is kept apart as its reciprocal.  One block
// is w * kBandRows contiguous entries, so a wavefront reading a fixed o for
// consecutive r touches consecutive addresses.
constexpr int kSlabMaxW = 144;
constexpr int kSlabFarWaves = 4;    // waves of the off-diagonal sums
constexpr int kSlabParts = 2 * kSlabFarWaves;  // far partial sums per row (one per half-wave)
constexpr int kSlabLead[3] = {2, 3, 4};  // blocks in flight: FP64, FP32, FP16 storage
constexpr int kSlabWinTail = 16;    // mirrored slots after the solution window
constexpr int kMaxFactorW = 1024;  // widest band the device factorisation takes
// Sparse triangular passes as lane streams: a pass is a sequence of steps whose
// records (one dot product each, writing one value of the vector in LDS) read
// only values of earlier steps.  In each step the records are dealt out to
// groups of G = 2^g consecutive lanes (g chosen per step; G > 1 for steps with
// few, long records), and each wave then streams its own rounds, one item per
// lane and round: a 16-bit column and a value in the storage type.  A record's
// entries go round-robin over its group's lanes, which add val * y[col] to their
// sums; a terminator item (column kSparseTerm, value bits dest | g << 24 in the
// low 32 bits) in every lane of the group, in the same round, has the group sum
// its lanes and the first lane write the total to slot dest; padding items
// (0, 0) fill a lane's rounds; every step of every wave ends with a marker round
// (column kSparseMark in every lane) at which the workgroup synchronises.  A
// wave's round count is a multiple of kSparseLead (padding rounds after its
// last marker), and the columns of rounds 2m and 2m + 1 share one 32-bit word
// per lane (low half, high half): word m * 64 + lane.
// Loads run kSparseLead rounds ahead of use, so the item arrays carry
// 2 * kSparseLead rounds of slack after their last wave.
constexpr int kSparseWaves = kBandThreads / 64;
constexpr int32_t kSparseTerm = 0xfffe;
constexpr int32_t kSparseMark = 0xffff;
constexpr int32_t kSparseMaxSlots = 0xfffe;  // vector rows plus block slots
constexpr int kSparseGroupShift = 24;
constexpr int kSparseLead = 8;
// The slab layout stores, per 32-row block, the strictly lower triangle of the
// block's diagonal triangle at offsets o >= w - r (row r); its inverse has no
// more nonzeros only if every such position has a slot, i.e. w >= kBandRows - 1.
// FP64 / FP32 store the inverse in those slots; FP16 keeps the factor's own
// (row-scaled, quantised) entries there and the inverse of the dequantised
// triangle, in float32, in a separate packed array (kTriPackBytes per block).
inline bool tri_inverse_ok(int w, int storage) {
    (void)storage;
    return w <= kSlabMaxW && w >= kBandRows - 1;
}
constexpr int kTriPackFloats = 512;  // 496 strictly lower entries (row r at r (r - 1) / 2), padded
constexpr int kTriPackBytes = kTriPackFloats * 4;
// fixed device workspace of ras_solve_noalloc (per device, held until process exit)
constexpr size_t kNoAllocScratchBytes = RAS_NOALLOC_SCRATCH_BYTES;
// row stride (compute-type entries) of the near + triangle buffer: 2 blocks
// of columns plus padding that keeps 16-byte rows aligned and spreads the
// rows of a wavefront over the LDS banks
constexpr int slab_nt_stride(int compute_bytes) { return 2 * kBandRows + (compute_bytes == 8 ? 2 : 4); }
// LDS bytes of the slab pass: stages of (factor block + 512 bytes of row
// data), solution window + mirrored tail, near + triangle entries [2][rows][stride], row
// data [2][3][rows], far partial sums [2][parts][rows], results [2][rows]
inline size_t slab_stage_bytes(int storage_bytes, int max_w) {
    return (static_cast<size_t>(kBandRows) * max_w * storage_bytes + 1023) / 1024 * 1024;
}
inline size_t slab_lds_bytes(int storage_bytes, int compute_bytes, int max_w, int win) {
    const int lead = kSlabLead[storage_bytes == 8 ? 0 : storage_bytes == 4 ? 1 : 2];
    const size_t elems = static_cast<size_t>(win) + kSlabWinTail + 2 * kBandRows * slab_nt_stride(compute_bytes) + 2 * 3 * kBandRows +
                         2 * kSlabParts * kBandRows + 2 * kBandRows + kBandRows;  // ..., results, broadcast
    const size_t tri = storage_bytes == 2 ? kTriPackBytes : 0;  // FP16: the block's packed triangle inverse
    return (lead + 1) * (slab_stage_bytes(storage_bytes, max_w) + tri + 512) + elems * compute_bytes;
}
constexpr int kMaxItemsPerWg = 1024;  // work items one workgroup may own

// Static data of one subdomain (setup output, Sec. 3.2.2 / Sec. 3.3.1).
struct SubDev {
    const int32_t* omega;     // [n] global id g (owned row) or ~g (overlap row), ascending g
    const double* ell_val;    // [K][n_pad] values of A's rows on omega (float64)
    const float* ell_valf;    // [K][n_pad] float32 copy (CG with FP32 storage), else null
    const int32_t* ell_gcol;  // [K][n_pad] global column (padding: the row's own g)
    const int32_t* ell_lcol;  // [K][n_pad] slot of the column: local index in omega (< n), or
                              // n + position in ext for an external column; padding: the row itself
    const void* band_f;       // factor L: slab layout if slab, else [n][w+1] row-major lower band
    const void* band_b;       // reversed transpose J L^T J, same layout as band_f
    const float* scale;       // [n] FP16 row scale of L (null otherwise)
    const void* invd;         // [n] 1 / L_ii in the local compute type
    int32_t n, n_pad, K, w;
    int64_t row_off;          // offset of this subdomain in per-RHS scratch vectors
    const int32_t* nbr;       // [n_nbr] subdomains (of the same system) owning a point this one reads
    int32_t n_nbr;
    int32_t slab;             // 1: band_f / band_b in the slab layout (w <= kSlabMaxW)
    const int32_t* ext;       // [n_ext] global ids of the columns outside omega that omega's rows read
    int32_t n_ext;
    int32_t tri_inv;          // slab: the solver applies each block's triangle as its inverse, read from
                              // the triangle slots (FP64/FP32) or from tri_g (FP16), see tri_inverse_ok
    int64_t snap_off;         // offset of this subdomain's x snapshot (n + n_ext values) per right-hand side
    const float* tri_g[2];    // FP16 slab: packed float32 block-triangle inverses of L and of J L^T J
    // sparse Cholesky (local rows in elimination order); pass 0 = L (forward), 1 = L^T (backward),
    // as a lane stream (see kSparseWaves): wave w of the workgroup streams rounds
    // sp_wave[pass][2w] .. + sp_wave[pass][2w + 1] - 1, round r being the items
    // (half r % 2 of sp_col[pass][(r / 2) * 64 + lane], sp_val[pass][r * 64 + lane])
    const int32_t* sp_wave[2];
    const uint32_t* sp_col[2];
    const void* sp_val[2];    // storage type
    int32_t sp_nlev[2];       // steps of the pass
    int32_t sparse;           // 1: sparse Cholesky factor (sp_* valid)
    int32_t pad3_;
};

// Device factorisation of one subdomain's banded local matrix (Sec. 3.3.1: the
// Cholesky factor is computed once, at setup): A_p's lower band is gathered from
// the subdomain's ELL rows (local columns) into L[n][w+1] (row-major, diagonal at
// offset w) and factored in place in float64.  fail receives the first local row
// with a non-positive (or non-finite) pivot, or -1.
struct FactorJob {
    const double* ell_val;
    const int32_t* ell_lcol;
    int32_t n, n_pad, K, w;
    double* L;
    int32_t* fail;
    // layout of the factor as the triangular solves read it (see the upload code)
    void* band_f;        // L in the storage type: slab blocks [o][r] (w <= kSlabMaxW) or row-major [n][w+1]
    void* band_b;        // the reversed transpose J L^T J, same layout
    void* invd;          // [n] 1 / L_ii as the solves see it (compute type)
    float* scale;        // [n] FP16 row scales (FP16_ROWSCALED only)
    float* tri_g[2];     // FP16: packed block-triangle inverses (forward, backward), else null
    int32_t slab;
    int32_t tri_inv;     // store the block triangles inverted (see SubDev)
    double robin_shift;  // Robin transmission: diagonal minus robin_shift * (coupling outside omega)
};

// One work item: subdomain `sub` of right-hand side (instance) `inst`.
struct ItemDev {
    int32_t inst;
    int32_t sub;
};

// One right-hand side of one system.
struct InstDev {
    const double* b;          // [n]
    double* x0;               // [n] caller's x (initial guess in, result out)
    double* x1;               // [n] second buffer (synchronous mode)
    void* scratch;            // [sum n_p] local vector in the compute type (CG: exchanged residual, band: solve vector)
    double* snap;             // asynchronous: [sum (n_p + n_ext_p)] x on omega and its external layer, as one
                              // update read it (every row and the prolongation use these values); else null
    double* hist;             // [hist_cap] relative residual history
    double* hist_t;           // [hist_cap] seconds since start
    int64_t hist_cap;
    int64_t max_sweeps;
    double tol2;              // tol^2
    double bnorm2;            // ||b||^2 (filled on device before the solve)
    int32_t item_begin;       // items of this instance are [item_begin, item_begin + item_count)
    int32_t item_count;
    int32_t leader;           // workgroup owning item_begin (runs the detector / records history)
    int32_t pad_;
    // host-written control words of the system's handle (pinned, coherent host
    // memory; asynchronous mode): ctl[0] != 0 cancels the solve, ctl[1 + p] != 0
    // pauses subdomain p (it takes no updates while set); null: none
    const int32_t* ctl;
};

// Mutable per-instance state.
struct InstState {
    int32_t stop;             // async: 0 running, 1 converged (detector), 2 time limit, 3 exhausted
    int32_t result_buf;       // sync: buffer (0/1) that holds the returned iterate
    int64_t sweeps;           // sync: sweeps applied; async: detector passes
    int64_t hist_len;
    int64_t stopped_at;       // sync: sweep of the stop decision (-1 running)
    int64_t t0;               // wall-clock tick of the first launch
};

struct GridBarrier {
    uint32_t count;
    uint32_t gen;
    int64_t abort_at;         // sync: sweep at which every instance stops (time limit)
};

struct Params {
    const SubDev* subs;
    const ItemDev* items;
    const InstDev* insts;
    InstState* ist;
    double* res2_own;         // [2][n_items] owned residual^2 (sync: by sweep parity)
    int32_t* conv;            // [n_items] local criterion met (async)
    int32_t* gflag;           // [n_items] global-convergence flag (decentralized detection)
    int64_t* solves;          // [n_items] local solves done
    int64_t* phase;           // [n_items][4] wall-clock ticks: residual, local solve, prolongation, other
    uint32_t* version;        // [n_items] published updates (async)
    const int32_t* team_ptr;  // [n_teams + 1]
    const int32_t* team_items;  // item ids per team, in visiting order
    const int32_t* wg_team;   // [n_wg] team of each workgroup
    const int32_t* wg_member; // [n_wg] rank of each workgroup inside its team
    const int32_t* team_win;  // [n_subs][T][2] LDS window [lo, hi) of local rows of each team member
    uint32_t* team_bar;       // [n_teams][2] team barrier ticket counter (64-bit)
    double* team_buf;         // [n_teams][2][T][4] team reduction / broadcast slots
    GridBarrier* bar;
    int32_t n_items;
    int32_t n_insts;
    int32_t n_wg;
    int32_t cg_iters;
    int32_t team_size;        // T (1 for the banded solver)
    int32_t detect;           // 0 centralized, 1 decentralized (asynchronous mode)
    int64_t max_ticks;        // wall-clock ticks allowed (<= 0: unlimited)
    int64_t sweep0;           // sync: first sweep index of this launch
    double pace;              // async: neighbour wait budget, in units of the previous update's duration
};

}  // namespace ras
