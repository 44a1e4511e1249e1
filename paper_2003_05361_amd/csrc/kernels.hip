// Persistent restricted additive Schwarz kernels for gfx950 (CDNA4, wave64).
//
// One launch runs a whole solve (or until a time limit): every workgroup owns
// a static list of work items (subdomain x right-hand side) and repeats, per
// item, one "subdomain update":
//   1. restrict + residual: r_p = b[Omega_p] - (A x)[Omega_p]  (Sec. 3.2.2: the
//      local rows of A with their interface columns; reads neighbour-owned x),
//      plus ||r_p[owned]||^2, ||r_p||^2, ||b_p||^2 (Sec. 3.3.2, eq. local_conv);
//   2. local solve (Sec. 3.3.1): k steps of CG on A_p, or the forward and
//      backward banded triangular solves with the Cholesky factor of A_p;
//   3. restricted prolongation: x[O_p] += delta_p on owned points only
//      (Sec. 2.1, restricted additive Schwarz).
// Synchronous mode (Sec. 2.1, Sec. 3.4 two-sided): x is double-buffered, all
// updates of sweep k read x^k, and one grid barrier separates sweeps.
// Asynchronous mode (Sec. 2.1, Sec. 3.4 one-sided): a single x in place, read
// and written with agent-scope relaxed atomics, no barrier; a per-item
// version counter is bumped with release semantics after each publish.
// Termination (Sec. 2.2, Sec. 3.3.2): synchronous -- the exact global residual
// of x^k is assembled from the owned partial norms after the barrier;
// asynchronous -- a centralized detector (the workgroup holding the system's
// first subdomain) stops the system once every subdomain reports its local
// criterion and the sum of the latest owned residuals is below tolerance; the
// host then verifies the exact residual and resumes if it fails.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "device.hpp"

namespace ras {

// ------------------------------------------------------------------------------ helpers

#define RAS_GLOBAL __attribute__((address_space(1)))
#define RAS_LDS __attribute__((address_space(3)))

// Uniform (SGPR) copies of 32/64-bit values loaded from memory.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int32_t>(v)));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int32_t>(v >> 32)));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}
template <class T>
__device__ __forceinline__ RAS_GLOBAL T* gptr(const T* p) {
    return (RAS_GLOBAL T*)(reinterpret_cast<T*>(uni64(reinterpret_cast<int64_t>(p))));
}

// A subdomain descriptor held in scalar registers with global-memory pointers.
struct SubU {
    RAS_GLOBAL int32_t* omega;
    RAS_GLOBAL double* ell_val;
    RAS_GLOBAL float* ell_valf;
    RAS_GLOBAL int32_t* ell_gcol;
    RAS_GLOBAL int32_t* ell_lcol;
    const void* band_f;
    const void* band_b;
    RAS_GLOBAL float* scale;
    const void* invd;
    int32_t n, n_pad, K, w;
    int64_t row_off;
    RAS_GLOBAL int32_t* ext;
    int32_t n_ext;
    int64_t snap_off;
};

__device__ __forceinline__ SubU load_sub(const SubDev* p) {
    const SubDev d = *p;
    SubU s;
    s.omega = gptr(d.omega);
    s.ell_val = gptr(d.ell_val);
    s.ell_valf = gptr(d.ell_valf);
    s.ell_gcol = gptr(d.ell_gcol);
    s.ell_lcol = gptr(d.ell_lcol);
    s.band_f = reinterpret_cast<const void*>(uni64(reinterpret_cast<int64_t>(d.band_f)));
    s.band_b = reinterpret_cast<const void*>(uni64(reinterpret_cast<int64_t>(d.band_b)));
    s.scale = gptr(d.scale);
    s.invd = reinterpret_cast<const void*>(uni64(reinterpret_cast<int64_t>(d.invd)));
    s.n = uni(d.n);
    s.n_pad = uni(d.n_pad);
    s.K = uni(d.K);
    s.w = uni(d.w);
    s.row_off = uni64(d.row_off);
    s.ext = gptr(d.ext);
    s.n_ext = uni(d.n_ext);
    s.snap_off = uni64(d.snap_off);
    return s;
}

// The per-instance pointers and scalars an update needs, uniform.
struct InstU {
    RAS_GLOBAL double* b;
    RAS_GLOBAL double* x0;
    RAS_GLOBAL double* x1;
    void* scratch;
    RAS_GLOBAL double* snap;
};

__device__ __forceinline__ InstU load_inst(const InstDev* p) {
    const InstDev d = *p;
    InstU u;
    u.b = gptr(d.b);
    u.x0 = gptr(d.x0);
    u.x1 = gptr(d.x1);
    u.scratch = reinterpret_cast<void*>(uni64(reinterpret_cast<int64_t>(d.scratch)));
    u.snap = gptr(d.snap);
    return u;
}

template <bool ATOMIC>
__device__ __forceinline__ double ldx(RAS_GLOBAL double* p) {
    if constexpr (ATOMIC)
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *p;
}

template <bool ATOMIC>
__device__ __forceinline__ void stx(RAS_GLOBAL double* p, double v) {
    if constexpr (ATOMIC)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

template <class T>
__device__ __forceinline__ T ld_rlx(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_rlx(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the workgroup; every thread gets the same value (fixed order):
// per-wave butterfly, then every wave reduces the per-wave partials the same way.
template <int B, class T>
__device__ __forceinline__ T block_sum(T v, T* red) {
    static_assert(B / 64 <= 64, "at most 64 waves");
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    T t = lane < B / 64 ? red[lane] : T(0);
    t = wave_sum(t);
    __syncthreads();
    return t;
}

template <int B>
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* red) {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    constexpr int NW = B / 64;
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = a;
        red[NW + (threadIdx.x >> 6)] = b;
        red[2 * NW + (threadIdx.x >> 6)] = c;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    a = wave_sum(lane < NW ? red[lane] : 0.0);
    b = wave_sum(lane < NW ? red[NW + lane] : 0.0);
    c = wave_sum(lane < NW ? red[2 * NW + lane] : 0.0);
    __syncthreads();
}

// Grid-wide barrier for co-resident workgroups (cooperative launch).  Every
// thread fences its own writes at agent scope before arriving; the last
// arriver opens the next generation with a release store.
__device__ void grid_barrier(GridBarrier* bar, uint32_t nwg) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t g = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t arrived =
            __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nwg - 1) {
            __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar->gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            while (__hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g)
                __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// ------------------------------------------------------------------------------ teams
// A team is T workgroups sharing one subdomain's local solve (CG): member m
// owns local rows [m n / T, (m+1) n / T).  Team-wide values are reduced per
// workgroup, exchanged through global slots and summed in member order, so
// every member obtains bit-identical results.
struct TeamCtx {
    int team, member, T;
    RAS_GLOBAL uint32_t* bar;  // {count, generation}
    RAS_GLOBAL double* buf;    // [2][T][4]
    uint32_t phase;            // barriers passed (slot parity)
    // wall-clock stamps of the current update (thread 0): residual done, local solve done
    int64_t st_res, st_solve;
};

__device__ __forceinline__ TeamCtx make_team(const Params& P) {
    TeamCtx tc;
    tc.team = uni(P.wg_team[blockIdx.x]);
    tc.member = uni(P.wg_member[blockIdx.x]);
    tc.T = P.team_size;
    tc.bar = gptr(P.team_bar) + 2 * tc.team;
    tc.buf = gptr(P.team_buf) + static_cast<int64_t>(tc.team) * 8 * tc.T;
    tc.phase = 0;
    tc.st_res = 0;
    tc.st_solve = 0;
    return tc;
}

// Team barrier without cache-wide fences.  Every value that crosses workgroups
// inside a team (exchanged residual rows, reduction slots) is written and read
// with device-scope relaxed atomics, which go to the device-coherent level and
// never sit in (or are served from) an XCD-private cache line.  Each wave
// drains its memory counters before the workgroup arrives, so those stores
// have completed when the arrival is counted; arrivals increment a 64-bit
// ticket counter and a member leaves barrier k once the counter reaches
// (k + 1) T.  No cache write-back or invalidation is needed, which keeps the
// two barriers of every CG step cheap.
__device__ void team_barrier(TeamCtx& tc) {
    if (tc.T == 1) {
        __syncthreads();
        return;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        RAS_GLOBAL unsigned long long* ctr = (RAS_GLOBAL unsigned long long*)(tc.bar);
        const unsigned long long ticket =
            __hip_atomic_fetch_add(ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long target = (ticket / tc.T + 1) * tc.T;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target)
            __builtin_amdgcn_s_sleep(1);
    }
    __syncthreads();
    ++tc.phase;
}

template <class T>
__device__ __forceinline__ T ldg_dev(RAS_GLOBAL T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void stg_dev(RAS_GLOBAL T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum NV workgroup totals (already block-reduced, uniform) over the team; the
// values flagged in `ct_mask` are summed in the compute type CT.
template <class CT, int NV>
__device__ __forceinline__ void team_sum(TeamCtx& tc, double (&v)[NV], unsigned ct_mask) {
    if (tc.T == 1) return;
    RAS_GLOBAL double* slot = tc.buf + (tc.phase & 1) * 4 * tc.T;
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) stg_dev(slot + 4 * tc.member + k, v[k]);
    team_barrier(tc);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        if ((ct_mask >> k) & 1) {
            CT acc = CT(0);
            for (int m = 0; m < tc.T; ++m) acc += static_cast<CT>(ldg_dev(slot + 4 * m + k));
            v[k] = static_cast<double>(acc);
        } else {
            double acc = 0.0;
            for (int m = 0; m < tc.T; ++m) acc += ldg_dev(slot + 4 * m + k);
            v[k] = acc;
        }
    }
}

// Member 0's value, seen identically by every member of the team.
__device__ __forceinline__ int team_bcast(TeamCtx& tc, int v0, int* lds_flag) {
    if (tc.T == 1) {
        if (threadIdx.x == 0) *lds_flag = v0;
        __syncthreads();
        const int r = *lds_flag;
        __syncthreads();
        return r;
    }
    RAS_GLOBAL double* slot = tc.buf + (tc.phase & 1) * 4 * tc.T;
    if (threadIdx.x == 0 && tc.member == 0) stg_dev(slot, static_cast<double>(v0));
    team_barrier(tc);
    return static_cast<int>(ldg_dev(slot));
}

template <class CT>
__device__ __forceinline__ CT load_as(const void* base, int64_t idx);
template <>
__device__ __forceinline__ double load_as<double>(const void* base, int64_t idx) {
    return static_cast<const double*>(base)[idx];
}
template <>
__device__ __forceinline__ float load_as<float>(const void* base, int64_t idx) {
    return static_cast<const float*>(base)[idx];
}

// ------------------------------------------------------------------------------ residual
// The outer residual is accumulated with compensated (double-word) arithmetic,
// the Dot2 scheme of Ogita, Rump and Oishi (SIAM J. Sci. Comput. 26, 2005):
// each product a x is split exactly into p + pe with one FMA (TwoProduct),
// each running subtraction s - p exactly into t + te (Knuth's TwoSum), and the
// rounding errors te - pe are summed apart and added once at the end.  The
// result is as accurate as if it were computed in twice float64's precision
// and then rounded: near convergence r = b - A x cancels, and a plain float64
// sum carries an absolute error of about eps |A| |x|, which on strongly varying
// coefficients sits at the tolerance itself.  Contraction is off so that the
// compiler cannot fuse p into the subtraction.
struct CompAcc {
    double s, c;
};

__device__ __forceinline__ void comp_sub(CompAcc& r, double a, double x) {
#pragma clang fp contract(off)
    const double p = a * x;
    const double pe = __builtin_fma(a, x, -p);
    const double t = r.s - p;
    const double z = t - r.s;
    const double te = (r.s - (t - z)) - (p + z);
    r.s = t;
    r.c += te - pe;
}

__device__ __forceinline__ double comp_value(const CompAcc& r) { return r.s + r.c; }

// r_i = b_g - sum_k A_{g, col_k} x_{col_k} for local row i (global g).  ELL
// slot k of row i sits at k * n_pad + i.  KT > 0: compile-time row width.
template <int KT, bool ATOMIC>
__device__ __forceinline__ double row_residual(const SubU& s, RAS_GLOBAL double* b, RAS_GLOBAL double* x, int i,
                                               bool& owned, double& bg) {
    const int32_t e = s.omega[i];
    owned = e >= 0;
    const int32_t g = owned ? e : ~e;
    bg = b[g];
    CompAcc acc{bg, 0.0};
    if constexpr (KT > 0) {
        int32_t c[KT];
        double a[KT];
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            c[k] = (s.ell_gcol + static_cast<uint32_t>(k * s.n_pad))[static_cast<uint32_t>(i)];
            a[k] = (s.ell_val + static_cast<uint32_t>(k * s.n_pad))[static_cast<uint32_t>(i)];
        }
#pragma unroll
        for (int k = 0; k < KT; ++k) comp_sub(acc, a[k], ldx<ATOMIC>(x + c[k]));
    } else {
        for (int k = 0; k < s.K; ++k) {
            const uint32_t idx = static_cast<uint32_t>(k * s.n_pad + i);
            comp_sub(acc, s.ell_val[idx], ldx<ATOMIC>(x + s.ell_gcol[idx]));
        }
    }
    return comp_value(acc);
}

// Asynchronous updates read x once.  A residual row reads a neighbour-owned
// value of x that other rows read too; should those reads see different
// versions (the owner updates meanwhile), the exact cancellation in the local
// solve no longer holds and the iteration can diverge, while one version per
// value (any version) keeps it convergent (Sec. 2.1: each subdomain works on
// a local copy of the values it receives).  So an update first copies x on
// omega and its external layer into a snapshot (slots: omega's local order,
// then the external columns), and the residual and the prolongation read
// only the snapshot.  Team members fill disjoint slices with device-scope
// stores; everything reads the snapshot with device-scope loads.
__device__ __forceinline__ void take_snapshot(const SubU& s, RAS_GLOBAL double* x, RAS_GLOBAL double* xs, int lo,
                                              int hi, int nthreads) {
    // four slots per thread at a time: the index loads, then the x loads, in flight together
    constexpr int U = 4;
    for (int k0 = lo + static_cast<int>(threadIdx.x); k0 < hi; k0 += U * nthreads) {
        int32_t g[U];
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = min(k0 + u * nthreads, hi - 1);
            if (k < s.n) {
                const int32_t e = s.omega[k];
                g[u] = e >= 0 ? e : ~e;
            } else {
                g[u] = s.ext[k - s.n];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = ldx<true>(x + g[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * nthreads < hi) stg_dev(xs + k0 + u * nthreads, xv[u]);
    }
}

// b - A x for local row i, x from the snapshot
template <int KT>
__device__ __forceinline__ double row_residual_snap(const SubU& s, RAS_GLOBAL double* b, RAS_GLOBAL double* xs,
                                                    int i, bool& owned, double& bg) {
    const int32_t e = s.omega[i];
    owned = e >= 0;
    const int32_t g = owned ? e : ~e;
    bg = b[g];
    CompAcc acc{bg, 0.0};
    if constexpr (KT > 0) {
        int32_t c[KT];
        double a[KT];
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            c[k] = (s.ell_lcol + static_cast<uint32_t>(k * s.n_pad))[static_cast<uint32_t>(i)];
            a[k] = (s.ell_val + static_cast<uint32_t>(k * s.n_pad))[static_cast<uint32_t>(i)];
        }
#pragma unroll
        for (int k = 0; k < KT; ++k) comp_sub(acc, a[k], ldg_dev(xs + c[k]));
    } else {
        for (int k = 0; k < s.K; ++k) {
            const uint32_t idx = static_cast<uint32_t>(k * s.n_pad + i);
            comp_sub(acc, s.ell_val[idx], ldg_dev(xs + s.ell_lcol[idx]));
        }
    }
    return comp_value(acc);
}

// Residual of every local row of one workgroup's subdomain into v (the local
// solves' right-hand side; LDS when the solve keeps its vector there) with the
// three squared norms, U rows per thread at a time: the independent loads of
// the U rows (omega, the ELL row, then b and the x values) are issued
// together, so a thread waits for two memory round trips per U rows instead of
// per row.  x is the shared vector (global columns) or, asynchronously, the
// update's snapshot (local columns).
template <int KT, int U, bool SNAP, class VP>
__device__ __forceinline__ void residual_rows(const SubU& s, RAS_GLOBAL double* b, RAS_GLOBAL double* x, VP v, int n,
                                              int nthreads, double& own2, double& loc2, double& b2) {
    using CT = typename std::remove_reference<decltype(*v)>::type;
    RAS_GLOBAL const int32_t* cols = SNAP ? s.ell_lcol : s.ell_gcol;
    for (int i0 = static_cast<int>(threadIdx.x); i0 < n; i0 += U * nthreads) {
        int32_t e[U], c[U][KT];
        double a[U][KT], bg[U], xv[U][KT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = min(i0 + u * nthreads, n - 1);
            e[u] = s.omega[i];
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                c[u][k] = (cols + static_cast<uint32_t>(k * s.n_pad))[static_cast<uint32_t>(i)];
                a[u][k] = (s.ell_val + static_cast<uint32_t>(k * s.n_pad))[static_cast<uint32_t>(i)];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            bg[u] = b[e[u] >= 0 ? e[u] : ~e[u]];
#pragma unroll
            for (int k = 0; k < KT; ++k) xv[u][k] = SNAP ? ldg_dev(x + c[u][k]) : x[c[u][k]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * nthreads;
            if (i >= n) break;
            CompAcc acc{bg[u], 0.0};
#pragma unroll
            for (int k = 0; k < KT; ++k) comp_sub(acc, a[u][k], xv[u][k]);
            const double ri = comp_value(acc);
            loc2 += ri * ri;
            b2 += bg[u] * bg[u];
            if (e[u] >= 0) own2 += ri * ri;
            v[i] = static_cast<CT>(ri);
        }
    }
}

// ------------------------------------------------------------------------------ CG update
// Local solve by `cg_iters` steps of Hestenes-Stiefel CG from zero on A_p (the
// local rows and columns of A; external columns read a zero LDS slot), by a
// team of T workgroups.  Each thread holds R rows (tid + j B of its member's
// range) of r, A p and the correction in registers; the search direction p of
// the member's LDS window (own rows plus the halo its rows reach) lives in
// LDS.  After every residual update the member publishes its r through the
// per-item exchange vector; after the team reduction of r'r every member
// rebuilds its halo as p = r + beta p exactly as the owner does.
template <class CT, int KT, int R, bool ASYNC>
struct CgUpdate {
    static constexpr int B = kCgThreads;

    __device__ __forceinline__ void operator()(const Params& P, TeamCtx& tc, const ItemDev& item,
                                               RAS_GLOBAL double* xin, RAS_GLOBAL double* xout, double& own2,
                                               double& loc2, double& b2) {
        extern __shared__ __align__(16) unsigned char smem[];
        __shared__ double red[4 * (B / 64)];
        __shared__ CT redc[B / 64];
        CT* pl = reinterpret_cast<CT*>(smem);
        const SubU s = load_sub(P.subs + item.sub);
        const InstU in = load_inst(P.insts + item.inst);
        const int tid = threadIdx.x;
        const int n = s.n;
        const int T = tc.T;
        const int lo = static_cast<int>(static_cast<int64_t>(tc.member) * n / T);
        const int hi = static_cast<int>(static_cast<int64_t>(tc.member + 1) * n / T);
        const int32_t* wp = P.team_win + 2 * (static_cast<int64_t>(item.sub) * T + tc.member);
        const int wlo = uni(wp[0]);
        const int whi = uni(wp[1]);
        const int zs = whi - wlo;  // zero slot: external columns
        RAS_GLOBAL CT* rg = gptr(static_cast<CT*>(in.scratch)) + s.row_off;
        RAS_GLOBAL CT* val;
        if constexpr (sizeof(CT) == 8)
            val = s.ell_val;
        else
            val = s.ell_valf;
        CT r[R], q[R], d[R];
        uint32_t ownbits = 0;
        double o2 = 0.0, l2 = 0.0, bb = 0.0;
        CT rr = CT(0);
        RAS_GLOBAL double* xs = nullptr;
        if constexpr (ASYNC) {
            xs = in.snap + s.snap_off;
            const int m = n + s.n_ext;
            take_snapshot(s, xin, xs, static_cast<int>(static_cast<int64_t>(tc.member) * m / T),
                          static_cast<int>(static_cast<int64_t>(tc.member + 1) * m / T), B);
            __builtin_amdgcn_s_waitcnt(0);
            team_barrier(tc);
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = lo + tid + j * B;
            r[j] = CT(0);
            q[j] = CT(0);
            d[j] = CT(0);
            if (i < hi) {
                double bg;
                bool ow;
                double ri;
                if constexpr (ASYNC)
                    ri = row_residual_snap<KT>(s, in.b, xs, i, ow, bg);
                else
                    ri = row_residual<KT, false>(s, in.b, xin, i, ow, bg);
                l2 += ri * ri;
                bb += bg * bg;
                if (ow) {
                    o2 += ri * ri;
                    ownbits |= 1u << j;
                }
                r[j] = static_cast<CT>(ri);
                rr += r[j] * r[j];
                pl[i - wlo] = r[j];
                if (T > 1) stg_dev(rg + i, r[j]);
            }
        }
        if (tid == 0) pl[zs] = CT(0);
        double v4[4];
        {
            double a = o2, b = l2, c = bb;
            block_sum3<B>(a, b, c, red);
            v4[0] = a;
            v4[1] = b;
            v4[2] = c;
            v4[3] = static_cast<double>(block_sum<B>(rr, redc));
        }
        team_sum<CT, 4>(tc, v4, 0x8u);
        if (tid == 0) tc.st_res = wall_clock64();
        own2 = v4[0];
        loc2 = v4[1];
        b2 = v4[2];
        CT rho = static_cast<CT>(v4[3]);
        if (T > 1) {
            for (int i = wlo + tid; i < lo; i += B) pl[i - wlo] = ldg_dev(rg + i);
            for (int i = hi + tid; i < whi; i += B) pl[i - wlo] = ldg_dev(rg + i);
            __syncthreads();
        }
        for (int it = 0; it < P.cg_iters; ++it) {
            // the matrix is streamed every iteration: hide the loop invariance of its
            // pointers so the compiler does not park all R*K entries in registers
            RAS_GLOBAL CT* vit = val;
            RAS_GLOBAL int32_t* cit = s.ell_lcol;
            asm volatile("" : "+s"(vit), "+s"(cit));
            CT sp = CT(0);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = lo + tid + j * B;
                if (i < hi) {
                    CT acc = CT(0);
                    if constexpr (KT > 0) {
                        int32_t c[KT];
                        CT a[KT];
#pragma unroll
                        for (int k = 0; k < KT; ++k) {
                            c[k] = (cit + static_cast<uint32_t>(k * s.n_pad))[static_cast<uint32_t>(i)];
                            a[k] = (vit + static_cast<uint32_t>(k * s.n_pad))[static_cast<uint32_t>(i)];
                        }
#pragma unroll
                        for (int k = 0; k < KT; ++k) acc += a[k] * pl[c[k] >= n ? zs : c[k] - wlo];
                    } else {
                        for (int k = 0; k < s.K; ++k) {
                            const uint32_t idx = static_cast<uint32_t>(k * s.n_pad + i);
                            const int c = cit[idx];
                            acc += vit[idx] * pl[c >= n ? zs : c - wlo];
                        }
                    }
                    q[j] = acc;
                    sp += pl[i - wlo] * acc;
                }
            }
            double vs[1] = {static_cast<double>(block_sum<B>(sp, redc))};
            team_sum<CT, 1>(tc, vs, 0x1u);
            const CT sigma = static_cast<CT>(vs[0]);
            if (rho == CT(0) || !(sigma > CT(0))) break;  // breakdown guard (team-uniform)
            const CT alpha = rho / sigma;
            const bool last = it + 1 == P.cg_iters;
            CT rn = CT(0);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = lo + tid + j * B;
                if (i < hi) {
                    d[j] += alpha * pl[i - wlo];
                    r[j] -= alpha * q[j];
                    rn += r[j] * r[j];
                    if (T > 1 && !last) stg_dev(rg + i, r[j]);
                }
            }
            if (last) break;  // p is not needed after the last step
            double vr[1] = {static_cast<double>(block_sum<B>(rn, redc))};
            team_sum<CT, 1>(tc, vr, 0x1u);
            const CT rho_new = static_cast<CT>(vr[0]);
            const CT beta = rho_new / rho;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = lo + tid + j * B;
                if (i < hi) pl[i - wlo] = r[j] + beta * pl[i - wlo];
            }
            if (T > 1) {
                for (int i = wlo + tid; i < lo; i += B) pl[i - wlo] = ldg_dev(rg + i) + beta * pl[i - wlo];
                for (int i = hi + tid; i < whi; i += B) pl[i - wlo] = ldg_dev(rg + i) + beta * pl[i - wlo];
            }
            rho = rho_new;
            __syncthreads();
        }
        if (tid == 0) tc.st_solve = wall_clock64();
        // restricted prolongation: owned points only
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = lo + tid + j * B;
            if (i < hi && ((ownbits >> j) & 1u)) {
                const int32_t g = s.omega[i];
                if constexpr (ASYNC)
                    stx<true>(xout + g, ldg_dev(xs + i) + static_cast<double>(d[j]));
                else
                    stx<false>(xout + g, xin[g] + static_cast<double>(d[j]));
            }
        }
    }
};

// ------------------------------------------------------------------------------ banded solves
template <class ST>
struct StorageTraits;
template <>
struct StorageTraits<double> {
    using CT = double;
    static constexpr bool kHalf = false;
};
template <>
struct StorageTraits<float> {
    using CT = float;
    static constexpr bool kHalf = false;
};
template <>
struct StorageTraits<_Float16> {
    using CT = float;
    static constexpr bool kHalf = true;
};

// Forward substitution with a row-major lower band [n][w+1] (diagonal at
// offset w), in blocks of kBandRows rows: the part of each row reaching into
// earlier blocks is a small GEMV against a sliding LDS window of the solution;
// the triangular diagonal block is solved by one wavefront.  With rev the
// matrix is the reversed transpose of L (backward substitution with L^T) and
// the vector is addressed from the end.
template <class ST>
__device__ void band_pass(RAS_GLOBAL ST* Lb, RAS_GLOBAL float* scale, bool rev,
                          RAS_GLOBAL typename StorageTraits<ST>::CT* invd, int n, int w,
                          RAS_GLOBAL typename StorageTraits<ST>::CT* v, typename StorageTraits<ST>::CT* stage,
                          typename StorageTraits<ST>::CT* win, int winm, typename StorageTraits<ST>::CT* gsum) {
    using CT = typename StorageTraits<ST>::CT;
    constexpr int BR = kBandRows;
    constexpr int NT = kBandThreads;
    constexpr int TPR = NT / BR;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int ld = w + 1;
    const int nblk = (n + BR - 1) / BR;
    for (int bk = 0; bk < nblk; ++bk) {
        const int t0 = bk * BR;
        const int rows = min(BR, n - t0);
        const int cnt = rows * ld;
        RAS_GLOBAL ST* src = Lb + static_cast<int64_t>(t0) * ld;
        for (int e = tid; e < cnt; e += NT) {
            CT val = static_cast<CT>(src[e]);
            if constexpr (StorageTraits<ST>::kHalf) {
                const int rr = e / ld;
                const int o = e - rr * ld;
                const int t = t0 + rr;
                const int lrow = rev ? (n - 1 - t) + w - o : t;
                val = lrow < n ? val * scale[lrow] : CT(0);
            }
            stage[e] = val;
        }
        __syncthreads();
        {
            const int rr = tid / TPR;
            const int sub = tid % TPR;
            const int t = t0 + rr;
            CT acc = CT(0);
            if (rr < rows) {
                const int olo = max(0, w - t);
                const int ohi = w - rr;
                for (int o = olo + sub; o < ohi; o += TPR) acc += stage[rr * ld + o] * win[(t - w + o) & winm];
            }
#pragma unroll
            for (int off = TPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (sub == 0) gsum[rr] = acc;
        }
        __syncthreads();
        if (tid < 64) {
            const int l = lane;
            const int t = t0 + l;
            const bool act = l < rows;
            const int vi = rev ? n - 1 - t : t;
            CT val = act ? static_cast<CT>(v[vi] - gsum[l]) : CT(0);
            const CT dinv = act ? invd[vi] : CT(0);
            CT Ld[BR];
#pragma unroll
            for (int m = 0; m < BR; ++m) Ld[m] = (act && m < l && m >= l - w) ? stage[l * ld + (w - l + m)] : CT(0);
            CT y = CT(0);
#pragma unroll
            for (int m = 0; m < BR; ++m) {
                const CT ym = __shfl(val * dinv, m, 64);
                if (l == m) y = ym;
                val -= Ld[m] * ym;
            }
            if (act) {
                v[vi] = y;
                win[t & winm] = y;
            }
        }
        __syncthreads();
    }
}

// ---- banded solves in the slab layout ---------------------------------------------
// Row t of a block (t = t0 + r) needs sum_o L[t][o] y[t - w + o] over its w
// sub-diagonal entries.  Split by column: "far" columns lie at least two
// blocks back, "near" columns in the previous block, "triangle" columns in
// the block itself.  Far sums of block j only need blocks <= j - 2, so they
// are computed one step ahead of the solver.  Per step (one workgroup
// barrier) the eight waves of the workgroup do:
//   wave 0          solver: near GEMV (a lane per row) and the sequential
//                   triangle of block j - 1, lane broadcasts by readlane;
//   waves 1,2,3,5   block j: far sums from its LDS stage, and a copy of its
//                   near + triangle entries (zero outside the band) and row
//                   data into a row-major buffer the solver reads in 16-byte
//                   pieces without masks;
//   waves 4,6       loaders: block j + D of the factor and its row data
//                   (right-hand side, 1/diagonal, FP16 scale) streamed from
//                   HBM straight into an LDS stage (global_load_lds, no
//                   registers), then a wait for the block due next step;
//   wave 7          store: results of block j - 2 to the local vector.
// Only loaders and the store wave touch global memory, so the LDS reads of
// the other waves never wait for memory; the loaders read no LDS, so their
// in-flight blocks are never drained by a wait the compiler places before
// an LDS access (the store wave reads LDS through an opaque instruction).
// Synchronisation inside a pass is a plain s_barrier after the LDS counter
// drains: no memory fence.
template <class ST>
struct SlabCfg {
    using CT = typename StorageTraits<ST>::CT;
    static constexpr int BR = kBandRows;
    static constexpr int SZ = static_cast<int>(sizeof(ST));
    static constexpr int E = 16 / SZ;                             // entries per 16-byte read
    static constexpr int RT = BR / E;                             // lanes covering one o of a block
    static constexpr int FT = kSlabFarWaves * 64;                 // far threads
    static constexpr int OPC = FT * E / BR;                       // o values per far round
    static constexpr int D = kSlabLead[SZ == 8 ? 0 : SZ == 4 ? 1 : 2];  // blocks in flight
    static constexpr int S = D + 1;                               // LDS stages
    static constexpr int QMAX = (kSlabMaxW * BR * SZ + 1023) / 1024;   // 1 KB pieces of a block
    static constexpr int QH = (QMAX + 1) / 2;                     // pieces per loader wave
    static constexpr int GB = StorageTraits<ST>::kHalf ? kTriPackBytes : 0;  // FP16: triangle inverse bytes
    static constexpr int QW = QH + 1 + (GB > 0 ? 1 : 0);          // + one row-data load (+ one inverse piece)
    static constexpr int NTS = slab_nt_stride(static_cast<int>(sizeof(CT)));  // near/triangle row stride
    static constexpr int CV = 16 / static_cast<int>(sizeof(CT));  // compute-type entries per 16 bytes
    static constexpr int KF = (kSlabMaxW - BR + 7) / 8;           // far columns per thread, widest band
    static_assert(KF <= kSlabWinTail, "mirrored window tail");
    static_assert((D - 1) * QW <= 63, "vmcnt range");
    static_assert(FT == BR * 8, "one far thread per 8 near/triangle entries");
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// wait until at most N vector-memory operations of this wave are outstanding
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N <= 63, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// LDS reads the compiler does not see as such (no memory wait is placed in front)
__device__ __forceinline__ double lds_opaque(const RAS_LDS double* p) {
    double r;
    asm volatile("ds_read_b64 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(r) : "v"(p) : "memory");
    return r;
}
__device__ __forceinline__ float lds_opaque(const RAS_LDS float* p) {
    float r;
    asm volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(r) : "v"(p) : "memory");
    return r;
}

template <class ST>
__device__ __forceinline__ typename StorageTraits<ST>::CT lds_entry(const RAS_LDS unsigned char* p) {
    if constexpr (sizeof(ST) == 2)
        return static_cast<float>(*reinterpret_cast<const RAS_LDS _Float16*>(p));
    else
        return *reinterpret_cast<const RAS_LDS ST*>(p);
}

// the 16 / sizeof(ST) entries of one 16-byte read, in the compute type
template <class ST>
__device__ __forceinline__ void unpack(const u32x4& q, typename StorageTraits<ST>::CT* e) {
    const uint32_t wv[4] = {q[0], q[1], q[2], q[3]};
#pragma unroll
    for (int u = 0; u < 16 / static_cast<int>(sizeof(ST)); ++u) {
        if constexpr (sizeof(ST) == 8) {
            e[u] = __builtin_bit_cast(double, (static_cast<uint64_t>(wv[2 * u + 1]) << 32) | wv[2 * u]);
        } else if constexpr (sizeof(ST) == 4) {
            e[u] = __builtin_bit_cast(float, wv[u]);
        } else {
            const uint16_t hb = static_cast<uint16_t>(wv[u / 2] >> (16 * (u & 1)));
            e[u] = static_cast<float>(__builtin_bit_cast(_Float16, hb));
        }
    }
}

// 16 bytes of compute-type entries from LDS
__device__ __forceinline__ void lds_vec(const RAS_LDS double* p, double* out) {
    const f64x2 q = *reinterpret_cast<const RAS_LDS f64x2*>(p);
    out[0] = q[0];
    out[1] = q[1];
}
__device__ __forceinline__ void lds_vec(const RAS_LDS float* p, float* out) {
    const f32x4 q = *reinterpret_cast<const RAS_LDS f32x4*>(p);
    out[0] = q[0];
    out[1] = q[1];
    out[2] = q[2];
    out[3] = q[3];
}

__device__ __forceinline__ float lane_value(float v, int m) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), m));
}
__device__ __forceinline__ double lane_value(double v, int m) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(b), m));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), m));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// One triangular pass (forward with L, or backward with the reversed
// transpose when rev) over a factor in the slab layout.  LDS:
//   stages [S][stage_bytes + 512]: factor block, then row data (FP64: rhs
//     [BR], 1/diag [BR]; otherwise rhs [BR], 1/diag [BR], scale [BR]);
//   solution window [winm + 1];
//   near + triangle entries [2][BR][NTS] (row r: near columns c < BR of the
//     previous block, then triangle columns BR + m, zero outside the band);
//   row data [2][3][BR]; far partial sums [2][parts][BR]; results [2][BR].
template <class ST>
struct SlabPass {
    using C = SlabCfg<ST>;
    using CT = typename C::CT;
    static constexpr int BR = C::BR, E = C::E, RT = C::RT, OPC = C::OPC, S = C::S, D = C::D, NTS = C::NTS,
                         CV = C::CV;
    static constexpr bool kHalf = StorageTraits<ST>::kHalf;
    static constexpr int kRowBytes = 512;

    RAS_GLOBAL const unsigned char* slab;
    RAS_GLOBAL CT* invd;
    RAS_GLOBAL float* scale;
    RAS_GLOBAL const unsigned char* gtri;  // FP16: packed triangle inverses of this pass (block-major)
    RAS_GLOBAL CT* v;
    RAS_LDS unsigned char* stages;
    RAS_LDS CT* win;
    RAS_LDS CT* nt;
    RAS_LDS CT* rowd;
    RAS_LDS CT* part;
    RAS_LDS CT* yout;
    RAS_LDS CT* bcast;  // [BR] the solver's per-lane values, read back by every lane
    int stage_bytes, n, w, winm, nblk, qlast;
    bool rev;
    bool tri_inv;  // triangle slots hold the inverse of the block's diagonal triangle
    int lane, wave;
    CT uprev;  // solver wave: the previous block's results (lane r: row r)

    __device__ __forceinline__ RAS_LDS unsigned char* stage(int j) const {
        return stages + (j % S) * (stage_bytes + C::GB + kRowBytes);
    }
    __device__ __forceinline__ int row_index(int t) const { return rev ? n - 1 - t : t; }

    // loader k (0 or 1): its pieces of block j (clamped into the factor) and one row-data load
    __device__ __forceinline__ void load_block(int k, int j) {
        const int jj = min(j, nblk - 1);
        RAS_LDS unsigned char* st = stage(j);
        RAS_GLOBAL const unsigned char* src = slab + static_cast<int64_t>(jj) * w * BR * C::SZ + lane * 16;
#pragma unroll
        for (int i = 0; i < C::QH; ++i) {
            const int q = min(2 * i + k, qlast);
            __builtin_amdgcn_global_load_lds(src + q * 1024, (RAS_LDS void*)(st + q * 1024), 16, 0, 0);
        }
        if constexpr (C::GB > 0) {
            // FP16: one 1 KB piece of the block's packed triangle inverse per loader;
            // subdomains without inverses read the first 2 KB of their own band
            // (inside the allocation's tail padding) and ignore them
            const int64_t gofs = tri_inv ? static_cast<int64_t>(jj) * C::GB : 0;
            __builtin_amdgcn_global_load_lds(gtri + gofs + k * 1024 + lane * 16,
                                             (RAS_LDS void*)(st + stage_bytes + k * 1024), 16, 0, 0);
        }
        RAS_LDS unsigned char* rw = st + stage_bytes + C::GB;
        if constexpr (sizeof(CT) == 8) {
            // two dwords per row: lane l carries half l & 1 of row l >> 1
            const int t = min(jj * BR + (lane >> 1), n - 1);
            const RAS_GLOBAL unsigned char* a =
                reinterpret_cast<const RAS_GLOBAL unsigned char*>(k == 0 ? v + row_index(t) : invd + row_index(t));
            __builtin_amdgcn_global_load_lds(a + 4 * (lane & 1), (RAS_LDS void*)(rw + k * 256), 4, 0, 0);
        } else {
            const int t = min(jj * BR + (lane & (BR - 1)), n - 1);
            const int i = row_index(t);
            const RAS_GLOBAL void* a;
            if (k == 0 || !kHalf)
                a = lane < BR ? static_cast<const RAS_GLOBAL void*>(v + i) : static_cast<const RAS_GLOBAL void*>(invd + i);
            else
                a = scale + i;
            __builtin_amdgcn_global_load_lds(a, (RAS_LDS void*)(rw + (k == 0 || !kHalf ? 0 : 256)), 4, 0, 0);
        }
    }

    // far thread f of 4 * 64: far sums, near + triangle entries and row data
    // of block j.  Every LDS read is issued before the first write, so the
    // reads are in flight together.
    __device__ __forceinline__ void far_work(int f, int j) {
        const RAS_LDS unsigned char* st = stage(j);
        const int t0 = j * BR;
        // far sums: thread (row r = f % BR, part p = f / BR) takes the columns
        // o in [p K, p K + K) of row r that lie two or more blocks back
        // (o < w - BR - r).  Consecutive o are one stage row apart and read
        // consecutive window slots (the window has a mirrored tail, so a run
        // of K slots never wraps).
        const int fr = f % BR;
        const int fp = f / BR;
        const int fw = w - BR;
        const int K = (max(fw, 0) + 7) / 8;
        const int ob = fp * K;
        const RAS_LDS CT* wp = win + ((t0 + fr - w + ob) & winm);
        // a fixed number of reads, addresses clamped into range, masks in arithmetic:
        // no branch between the reads, so they are in flight together
        CT fe[C::KF], fy[C::KF];
#pragma unroll
        for (int k = 0; k < C::KF; ++k) {
            fe[k] = lds_entry<ST>(st + (max(min(ob + k, w - 1), 0) * BR + fr) * C::SZ);
            fy[k] = wp[k];
        }
        // near + triangle entries: thread (r = f % BR, d = f / BR) copies the
        // entries at o = w - 2 BR + 1 + d + 8 k (k < 8), i.e. column
        // c = o - (w - BR) + r of row r; a fixed o over consecutive r is a
        // contiguous stage row.  Columns c < 0 belong to the far sums; the
        // slots c >= BR + r (diagonal and above) stay zero from the pass start.
        const int rr = f % BR;
        const int d = f / BR;
        CT ntv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int o = w - 2 * BR + 1 + d + 8 * k;
            ntv[k] = lds_entry<ST>(st + (max(min(o, w - 1), 0) * BR + rr) * C::SZ);
        }
        CT rdv[3];
        if (f < BR) {
            const RAS_LDS unsigned char* rw = st + stage_bytes + C::GB;
            if constexpr (sizeof(CT) == 8) {
                rdv[0] = reinterpret_cast<const RAS_LDS CT*>(rw)[f];
                rdv[1] = reinterpret_cast<const RAS_LDS CT*>(rw + 256)[f];
                rdv[2] = CT(1);
            } else {
                rdv[0] = reinterpret_cast<const RAS_LDS CT*>(rw)[f];
                rdv[1] = reinterpret_cast<const RAS_LDS CT*>(rw)[BR + f];
                rdv[2] = kHalf ? reinterpret_cast<const RAS_LDS CT*>(rw + 256)[f] : CT(1);
            }
        }
        CT acc0 = CT(0), acc1 = CT(0);
#pragma unroll
        for (int k = 0; k < C::KF; k += 2) {
            acc0 += (k < K && ob + k < fw - fr ? fe[k] : CT(0)) * fy[k];
            if (k + 1 < C::KF) acc1 += (k + 1 < K && ob + k + 1 < fw - fr ? fe[k + 1] : CT(0)) * fy[k + 1];
        }
        const CT acc = acc0 + acc1;
        RAS_LDS CT* dst = nt + (j & 1) * BR * NTS + rr * NTS;
        // FP16 with inverses: the store wave writes the triangle columns (from the
        // block's float32 inverse), so they are left out here
        const int cmax = (kHalf && tri_inv) ? BR : 2 * BR;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int o = w - 2 * BR + 1 + d + 8 * k;
            const int c = o - (w - BR) + rr;
            // slots outside the row's near + triangle range go to an unread padding column
            dst[(c >= 0 && c < cmax && o < w) ? c : 2 * BR] = o >= 0 ? ntv[k] : CT(0);
        }
        if (f < BR) {
            RAS_LDS CT* rd = rowd + (j & 1) * 3 * BR + f;
            rd[0] = rdv[0];
            rd[BR] = rdv[1];
            rd[2 * BR] = rdv[2];
        }
        part[((j & 1) * kSlabParts + fp) * BR + fr] = acc;
    }

    __device__ __forceinline__ void solve_block(int j) {
        if (lane >= BR) return;
        const int t0 = j * BR;
        const int r = lane;
        const RAS_LDS CT* rd = rowd + (j & 1) * 3 * BR + r;
        const CT vin = rd[0], dinv = rd[BR], sc = rd[2 * BR];
        const RAS_LDS CT* pb = part + (j & 1) * kSlabParts * BR + r;
        CT fsum = pb[0];
#pragma unroll
        for (int k = 1; k < kSlabParts; ++k) fsum += pb[k * BR];
        const RAS_LDS CT* ntr = nt + (j & 1) * BR * NTS + r * NTS;
        // all reads first (the triangle entries too), so they are in flight together
        CT e[BR], tri[BR];
#pragma unroll
        for (int c = 0; c < BR; c += CV) lds_vec(ntr + c, e + c);
#pragma unroll
        for (int m = 0; m < BR; m += CV) lds_vec(ntr + BR + m, tri + m);
        asm volatile("" ::: "memory");
        // near columns: entries of row r times the previous block's results.  Four-
        // byte compute types read them from the window (contiguous aligned slots, all
        // lanes reading the same address); FP64 takes them from the lanes of this
        // wave that computed them (uprev, zero before the first block), which keeps
        // 64 registers free
        CT a[4] = {CT(0), CT(0), CT(0), CT(0)};
        if constexpr (sizeof(CT) == 4) {
            const RAS_LDS CT* yp = win + ((t0 - BR) & winm);
            CT yb[BR];
#pragma unroll
            for (int c = 0; c < BR; c += CV) lds_vec(yp + c, yb + c);
#pragma unroll
            for (int c = 0; c < BR; ++c) a[c & 3] += e[c] * yb[c];
        } else {
#pragma unroll
            for (int c = 0; c < BR; ++c) a[c & 3] += e[c] * lane_value(uprev, c);
        }
        const CT nsum = (a[0] + a[1]) + (a[2] + a[3]);
        CT u, g;
        if constexpr (kHalf) {
            if (!rev) {
                g = sc * dinv;
                u = (vin - sc * (fsum + nsum)) * dinv;
            } else {
                g = dinv * sc;
                u = (vin - (fsum + nsum)) * g;
            }
        } else {
            g = dinv;
            u = (vin - (fsum + nsum)) * g;
        }
        {
            CT Ld[BR];
#pragma unroll
            for (int m = 0; m < BR; ++m) Ld[m] = tri[m] * g;
            // lane m's value is final once steps 0 .. m - 1 are done; entries
            // with m >= r are zero, so later steps leave it unchanged
#pragma unroll
            for (int m = 0; m < BR - 1; ++m) u -= Ld[m] * lane_value(u, m);
        }
        CT y = u;
        if constexpr (kHalf)
            if (rev) y = u / sc;
        finish_block(j, y, u);
    }

    // the block's results y (to the store wave) and the window values u (y, or y
    // times the row scale in FP16 backward passes), also kept in this wave (FP64)
    __device__ __forceinline__ void finish_block(int j, CT y, CT u) {
        const int t0 = j * BR;
        const int r = lane;
        const int t = t0 + r;
        uprev = t < n ? u : CT(0);
        yout[(j & 1) * BR + r] = y;
        const int slot = t & winm;
        const CT wv = t < n ? u : CT(0);
        win[slot] = wv;
        if (slot < C::KF) win[winm + 1 + slot] = wv;  // mirrored tail
    }

    // Solver step with the block's triangle stored inverted (FP64 / FP32): y = G c,
    // G = T^-1 (diagonal 1 / L_rr; strictly lower part in the triangle slots) and
    // c = v - far - near sums.  Values cross lanes through LDS (one store per lane,
    // broadcast reads; a wave's LDS accesses complete in order), never through a
    // dependent readlane chain.  Entries are read when they are needed, so that the
    // near row, the window and the inverse are not all held in registers at once.
    __device__ __forceinline__ void solve_block_inv(int j) {
        if (lane >= BR) return;
        const int t0 = j * BR;
        const int r = lane;
        const RAS_LDS CT* rd = rowd + (j & 1) * 3 * BR + r;
        const CT vin = rd[0], dinv = rd[BR], sc = rd[2 * BR];
        const RAS_LDS CT* pb = part + (j & 1) * kSlabParts * BR + r;
        CT fsum = pb[0];
#pragma unroll
        for (int k = 1; k < kSlabParts; ++k) fsum += pb[k * BR];
        const RAS_LDS CT* ntr = nt + (j & 1) * BR * NTS + r * NTS;
        const RAS_LDS CT* yp = win + ((t0 - BR) & winm);
        CT a[4] = {CT(0), CT(0), CT(0), CT(0)};
        // reads in flight together: all at once for 4-byte types, eight at a time for
        // float64 (whose 32-entry rows would not fit the registers beside the rest)
        constexpr int CH = sizeof(CT) == 4 ? BR : 8;
#pragma unroll
        for (int c0 = 0; c0 < BR; c0 += CH) {
            CT e[CH], yb[CH];
#pragma unroll
            for (int c = 0; c < CH; c += CV) {
                lds_vec(ntr + c0 + c, e + c);
                lds_vec(yp + c0 + c, yb + c);
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) a[c & 3] += e[c] * yb[c];
        }
        // FP16: L's entries are stored divided by their row scale; forward passes
        // multiply the row's sums by it, backward passes keep it folded into the
        // solution window (which then holds y times the scale)
        const CT sums = fsum + ((a[0] + a[1]) + (a[2] + a[3]));
        const CT c = (kHalf && !rev) ? vin - sc * sums : vin - sums;
        bcast[r] = c;
        CT acc[4] = {c * dinv, CT(0), CT(0), CT(0)};
#pragma unroll
        for (int m0 = 0; m0 < BR; m0 += CH) {
            CT g[CH], cb[CH];
#pragma unroll
            for (int m = 0; m < CH; m += CV) {
                lds_vec(ntr + BR + m0 + m, g + m);
                lds_vec(bcast + m0 + m, cb + m);
            }
#pragma unroll
            for (int m = 0; m < CH; ++m) acc[m & 3] += g[m] * cb[m];
        }
        const CT y = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        finish_block(j, y, (kHalf && rev) ? y * sc : y);
    }

    // FP16 with inverses (store wave): block j's float32 triangle inverse, packed
    // in its stage (row r at r (r - 1) / 2), into the triangle columns of the
    // solver's row buffer; the solver reads it at the next step
    __device__ __forceinline__ void copy_tri(int j) {
        const RAS_LDS float* gp = reinterpret_cast<const RAS_LDS float*>(stage(j) + stage_bytes);
        RAS_LDS CT* dst = nt + (j & 1) * BR * NTS + BR;
        // lane: column m, rows 2 i + (lane >= 32); all reads in flight, then the writes
        // (no branches: every read index stays inside the packed block, and entries on
        // or above the diagonal go to the row's unread padding column)
        const int m = lane & (BR - 1), hi = lane >> 5;
        CT val[BR / 2];
#pragma unroll
        for (int i = 0; i < BR / 2; ++i) {
            const int r = 2 * i + hi;
            val[i] = gp[(r * (r - 1)) / 2 + m];
        }
#pragma unroll
        for (int i = 0; i < BR / 2; ++i) {
            const int r = 2 * i + hi;
            dst[r * NTS + (m < r ? m : BR)] = val[i];
        }
    }

    __device__ __forceinline__ void store_block(int j) {
        const int t = j * BR + lane;
        if (lane < BR && t < n) v[row_index(t)] = lds_opaque(yout + (j & 1) * BR + lane);
    }

    __device__ __forceinline__ void run() {
        const int tid = threadIdx.x;
        for (int i = tid; i <= winm + kSlabWinTail; i += kBandThreads) win[i] = CT(0);
        for (int i = tid; i < 2 * BR * NTS; i += kBandThreads) nt[i] = CT(0);
        __syncthreads();
        uprev = CT(0);
        const bool loader = wave == 4 || wave == 6;
        const int lk = wave == 4 ? 0 : 1;
        const int far = wave >= 1 && wave <= 3 ? wave - 1 : wave == 5 ? 3 : -1;
        if (loader) {
            for (int j = 0; j < D; ++j) load_block(lk, j);
            wait_vm<(D - 1) * C::QW>();  // block 0 has landed
        }
        lds_barrier();
        // step j: solver on block j - 1, far work on block j, loads of block
        // j + D (into the stage block j - 1 used), stores of block j - 2.  Every
        // role runs its own copy of the step loop (the same steps, one barrier
        // each): values a role keeps across steps are then live in its loop only,
        // not in every wave's, which keeps the register file free of the other
        // roles' loop invariants.
        if (wave == 0) {
            for (int j = 0; j <= nblk + 1; ++j) {
                if (j >= 1 && j <= nblk) {
                    if (tri_inv) solve_block_inv(j - 1);
                    else solve_block(j - 1);
                }
                lds_barrier();
            }
        } else if (far >= 0) {
            for (int j = 0; j <= nblk + 1; ++j) {
                if (j < nblk) far_work(far * 64 + lane, j);
                lds_barrier();
            }
        } else if (loader) {
            for (int j = 0; j <= nblk + 1; ++j) {
                load_block(lk, j + D);
                wait_vm<(D - 1) * C::QW>();  // block j + 1 has landed
                lds_barrier();
            }
        } else {
            for (int j = 0; j <= nblk + 1; ++j) {
                if (j >= 2) store_block(j - 2);
                if constexpr (kHalf)
                    if (tri_inv && j < nblk) copy_tri(j);
                lds_barrier();
            }
        }
        if (loader || wave == 7) wait_vm<0>();
        __syncthreads();
    }
};

// One pass, out of line: one copy serves both passes, and the pass state is
// a local here (registers), its pressure separate from the update around it.
template <class ST>
__device__ __attribute__((noinline)) void slab_run(RAS_GLOBAL const unsigned char* slab,
                                                   RAS_GLOBAL typename StorageTraits<ST>::CT* invd,
                                                   RAS_GLOBAL float* scale, RAS_GLOBAL const unsigned char* gtri,
                                                   RAS_GLOBAL typename StorageTraits<ST>::CT* v,
                                                   RAS_LDS unsigned char* lds, int stage_bytes, int n, int w, int winm,
                                                   bool rev, bool tri_inv) {
    using C = SlabCfg<ST>;
    using CT = typename C::CT;
    SlabPass<ST> ps;
    ps.slab = slab;
    ps.invd = invd;
    ps.scale = scale;
    ps.gtri = gtri;
    ps.v = v;
    ps.stages = lds;
    ps.win = (RAS_LDS CT*)(lds + C::S * (stage_bytes + C::GB + SlabPass<ST>::kRowBytes));
    ps.nt = ps.win + (winm + 1 + kSlabWinTail);
    ps.rowd = ps.nt + 2 * C::BR * C::NTS;
    ps.part = ps.rowd + 2 * 3 * C::BR;
    ps.yout = ps.part + 2 * kSlabParts * C::BR;
    ps.bcast = ps.yout + 2 * C::BR;
    ps.stage_bytes = stage_bytes;
    ps.n = n;
    ps.w = w;
    ps.winm = winm;
    ps.nblk = (n + C::BR - 1) / C::BR;
    ps.qlast = max((w * C::BR * C::SZ + 1023) / 1024 - 1, 0);  // last 1 KB piece of a block
    ps.rev = rev;
    ps.tri_inv = tri_inv;
    ps.lane = threadIdx.x & 63;
    ps.wave = uni(static_cast<int>(threadIdx.x >> 6));
    ps.run();
}

template <class ST>
__device__ __forceinline__ void slab_solve(const SubU& s, RAS_GLOBAL typename StorageTraits<ST>::CT* v,
                                           unsigned char* lds, int winm, int stage_bytes, bool tri_inv,
                                           const float* gf, const float* gb) {
    using CT = typename StorageTraits<ST>::CT;
    RAS_GLOBAL CT* invd = gptr(static_cast<const CT*>(s.invd));
    RAS_LDS unsigned char* l = (RAS_LDS unsigned char*)(lds);
    // FP16 subdomains without inverses stream a dummy piece from their own band (valid memory)
    RAS_GLOBAL const unsigned char* g0 =
        gf ? gptr(reinterpret_cast<const unsigned char*>(gf)) : gptr(static_cast<const unsigned char*>(s.band_f));
    RAS_GLOBAL const unsigned char* g1 =
        gb ? gptr(reinterpret_cast<const unsigned char*>(gb)) : gptr(static_cast<const unsigned char*>(s.band_b));
    slab_run<ST>(gptr(static_cast<const unsigned char*>(s.band_f)), invd, s.scale, g0, v, l, stage_bytes, s.n, s.w,
                 winm, false, tri_inv);
    slab_run<ST>(gptr(static_cast<const unsigned char*>(s.band_b)), invd, s.scale, g1, v, l, stage_bytes, s.n, s.w,
                 winm, true, tri_inv);
}

// One triangular pass over a sparse factor (Sec. 3.3.1's sparse direct
// solve) as a sequence of steps whose records read only values written in
// earlier steps: a record is one dot product of its entries with the vector y
// (in LDS) and writes one slot (a row of y, or a partial result of a dense
// block kept beyond the rows until the block's second step).  The host deals
// each step's records out to groups of lanes and lays each wave's share out
// as a stream of rounds (one item per lane, see kSparseWaves): entries
// accumulate into the lane's sum, a terminator round has each terminating
// group add its lanes' sums and write the total, and a marker round ends the
// wave's part of a step with a workgroup barrier.  No load of the stream
// depends on y, so each wave keeps kSparseLead rounds of loads in flight
// across steps; the barrier drains only the LDS counter.
__device__ __forceinline__ uint32_t low_bits(double v) {
    return static_cast<uint32_t>(__builtin_bit_cast(uint64_t, v));
}
__device__ __forceinline__ uint32_t low_bits(float v) { return __builtin_bit_cast(uint32_t, v); }

template <class ST>
__device__ __attribute__((noinline)) void sparse_run(RAS_GLOBAL const int32_t* wave_tab, RAS_GLOBAL const uint32_t* col,
                                                     RAS_GLOBAL const ST* val,
                                                     RAS_LDS typename StorageTraits<ST>::CT* y) {
    using CT = typename StorageTraits<ST>::CT;
    constexpr int D = kSparseLead;
    static_assert(kBandThreads == 64 * kSparseWaves, "one wave stream per wave of the workgroup");
    static_assert(D % 2 == 0, "column words hold two rounds");
    const int wave = uni(static_cast<int>(threadIdx.x) >> 6);
    const int lane = static_cast<int>(threadIdx.x) & 63;
    const int64_t base = uni(wave_tab[2 * wave]);
    const int R = uni(wave_tab[2 * wave + 1]);
    // the LDS address of y as an opaque scalar, so that it is not looked up again
    // after every barrier
    uint32_t yb = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(y));
    asm volatile("" : "+s"(yb));
    RAS_LDS CT* yy = reinterpret_cast<RAS_LDS CT*>(static_cast<uintptr_t>(yb));
    // base is even: the wave's column words start at base / 2
    RAS_GLOBAL const uint32_t* pc = col + (base / 2) * 64 + lane;
    RAS_GLOBAL const ST* pv = val + base * 64 + lane;
    uint32_t rc[D / 2];
    CT rv[D];
    // first rounds in the loop's own order (column word, then the two values),
    // so that the memory waits of the loop hold on entry as in steady state
#pragma unroll
    for (int j = 0; j < D / 2; ++j) {
        rc[j] = pc[j * 64];
        rv[2 * j] = static_cast<CT>(pv[(2 * j) * 64]);
        rv[2 * j + 1] = static_cast<CT>(pv[(2 * j + 1) * 64]);
        asm volatile("" ::: "memory");
    }
    // column of ring slot j (two rounds per word)
    auto col_at = [&](int j) { return static_cast<int>(j & 1 ? rc[j / 2] >> 16 : rc[j / 2] & 0xffffu); };
    CT acc = CT(0);
    // y of the next round is read one round ahead of its use: after this round's
    // barrier and before this round's write, which is legal because no record
    // reads a slot written in its own step
    CT ynext;
    {
        const int c0 = col_at(0);
        ynext = yy[R > 0 && c0 < kSparseTerm ? c0 : 0];
    }
    // R is a multiple of D: no bound check inside a group of D rounds; the loads
    // of the next group use immediate offsets from pointers advanced once per group
    for (int r0 = 0; r0 < R; r0 += D) {
        RAS_GLOBAL const uint32_t* pcn = pc + (D / 2) * 64;
        RAS_GLOBAL const ST* pvn = pv + D * 64;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int c = col_at(i);
            const CT v = rv[i];
            if (uni(c) == kSparseMark) {
                lds_barrier();
                acc = CT(0);
            }
            const CT yv = ynext;
            {
                // the last round of the group reads ahead into the next group, which
                // exists only below R (beyond it the arrays hold other waves' items)
                const int cn = col_at((i + 1) % D);
                ynext = yy[(i + 1 < D || r0 + D < R) && cn < kSparseTerm ? cn : 0];
            }
            const bool term = c == kSparseTerm;
            const bool add = c < kSparseTerm;
            acc = add ? acc + v * yv : acc;
            const uint64_t tm = __ballot(term);
            if (tm) {
                // groups of 2^g lanes end records together: sum over the group; the
                // terminator's value carries the slot and g
                const uint32_t pay = low_bits(v);
                const int g = (__builtin_amdgcn_readlane(static_cast<int>(pay), __builtin_ctzll(tm)) >>
                               kSparseGroupShift) & 7;
                CT t = acc;
                for (int k = 0; k < g; ++k) t += __shfl_xor(t, 1 << k);
                if (term && (lane & ((1 << g) - 1)) == 0) yy[pay & 0xffffffu] = t;
                acc = term ? CT(0) : acc;
            }
            if (i & 1) rc[i / 2] = pcn[(i / 2) * 64];
            rv[i] = static_cast<CT>(pvn[i * 64]);
        }
        pc = pcn;
        pv = pvn;
    }
}

// Both passes on the vector y in LDS (its first n slots hold the right-hand
// side on entry and the solution on return; every pass ends with a workgroup
// barrier, so the solution is visible to all threads on return).
template <class ST>
__device__ __forceinline__ void sparse_solve(const SubDev* sd, RAS_LDS typename StorageTraits<ST>::CT* y) {
    __syncthreads();
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass)
        sparse_run<ST>(gptr(sd->sp_wave[pass]), gptr(sd->sp_col[pass]), gptr(static_cast<const ST*>(sd->sp_val[pass])),
                       y);
}

template <class ST, bool ASYNC>
struct BandUpdate {
    using CT = typename StorageTraits<ST>::CT;
    static constexpr int B = kBandThreads;
    int max_w;        // widest row-major band of the launch (unpipelined pass stage)
    int winm;         // solution window size - 1
    int stage_bytes;  // slab pass: bytes of one factor block stage

    __device__ __forceinline__ void operator()(const Params& P, TeamCtx& tc, const ItemDev& item,
                                               RAS_GLOBAL double* xin, RAS_GLOBAL double* xout, double& own2,
                                               double& loc2, double& b2) {
        (void)tc;
        extern __shared__ __align__(16) unsigned char smem[];
        __shared__ double red3[3 * (B / 64)];
        __shared__ CT gsum[kBandRows];
        const SubU s = load_sub(P.subs + item.sub);
        const int slab = uni(P.subs[item.sub].slab);
        const int tri_inv = uni(P.subs[item.sub].tri_inv);
        const int sparse = uni(P.subs[item.sub].sparse);
        const InstU in = load_inst(P.insts + item.inst);
        const int tid = threadIdx.x;
        const int n = s.n;
        RAS_GLOBAL CT* v = gptr(static_cast<CT*>(in.scratch)) + s.row_off;
        own2 = 0.0;
        loc2 = 0.0;
        b2 = 0.0;
        RAS_GLOBAL double* xs = nullptr;
        if constexpr (ASYNC) {
            xs = in.snap + s.snap_off;
            take_snapshot(s, xin, xs, 0, n + s.n_ext, B);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        RAS_GLOBAL double* xr = ASYNC ? xs : xin;
        // the sparse solve keeps its vector in LDS: the residual goes there directly
        RAS_LDS CT* yl = (RAS_LDS CT*)(smem);
        const bool to_lds = sparse && sizeof(ST) != 2;
        if (s.K == 5 && to_lds) {
            residual_rows<5, 4, ASYNC>(s, in.b, xr, yl, n, B, own2, loc2, b2);
        } else if (s.K == 7 && to_lds) {
            residual_rows<7, 4, ASYNC>(s, in.b, xr, yl, n, B, own2, loc2, b2);
        } else if (s.K == 5) {
            residual_rows<5, 4, ASYNC>(s, in.b, xr, v, n, B, own2, loc2, b2);
        } else if (s.K == 7) {
            residual_rows<7, 4, ASYNC>(s, in.b, xr, v, n, B, own2, loc2, b2);
        } else {
            for (int i = tid; i < n; i += B) {
                bool owned;
                double bg;
                double ri;
                if constexpr (ASYNC)
                    ri = row_residual_snap<0>(s, in.b, xs, i, owned, bg);
                else
                    ri = row_residual<0, false>(s, in.b, xin, i, owned, bg);
                loc2 += ri * ri;
                b2 += bg * bg;
                if (owned) own2 += ri * ri;
                if (to_lds)
                    yl[i] = static_cast<CT>(ri);
                else
                    v[i] = static_cast<CT>(ri);
            }
        }
        // the loaders read v back through global-to-LDS loads
        __builtin_amdgcn_s_waitcnt(0);
        block_sum3<B>(own2, loc2, b2, red3);
        if (tid == 0) tc.st_res = wall_clock64();
        if (sparse) {
            if constexpr (sizeof(ST) != 2) sparse_solve<ST>(P.subs + item.sub, yl);
        } else if (slab) {
            slab_solve<ST>(s, v, smem, winm, stage_bytes, tri_inv != 0, P.subs[item.sub].tri_g[0],
                           P.subs[item.sub].tri_g[1]);
        } else {
            RAS_GLOBAL ST* Lf = gptr(static_cast<const ST*>(s.band_f));
            RAS_GLOBAL ST* Lr = gptr(static_cast<const ST*>(s.band_b));
            RAS_GLOBAL CT* iv = gptr(static_cast<const CT*>(s.invd));
            CT* win = reinterpret_cast<CT*>(smem);   // [winm + 1]
            CT* stage = win + (winm + 1);             // [kBandRows][max_w + 1]
            band_pass<ST>(Lf, s.scale, false, iv, n, s.w, v, stage, win, winm, gsum);
            band_pass<ST>(Lr, s.scale, true, iv, n, s.w, v, stage, win, winm, gsum);
        }
        if (tid == 0) tc.st_solve = wall_clock64();
        // restricted prolongation, four rows per thread at a time (loads first)
        constexpr int UP = 4;
        for (int i0 = tid; i0 < n; i0 += UP * B) {
            int32_t e[UP];
            double xo[UP];
            CT dv[UP];
#pragma unroll
            for (int u = 0; u < UP; ++u) {
                const int i = min(i0 + u * B, n - 1);
                e[u] = i0 + u * B < n ? s.omega[i] : -1;
                dv[u] = to_lds ? yl[i] : v[i];
                if constexpr (ASYNC) xo[u] = ldg_dev(xs + i);
            }
            if constexpr (!ASYNC) {
#pragma unroll
                for (int u = 0; u < UP; ++u) xo[u] = e[u] >= 0 ? xin[e[u]] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < UP; ++u)
                if (e[u] >= 0) stx<ASYNC>(xout + e[u], xo[u] + static_cast<double>(dv[u]));
        }
    }
};

// ------------------------------------------------------------------------------ drivers
template <int B>
__device__ double instance_owned_sum(const Params& P, const InstDev& in, int parity, double* red) {
    double s = 0.0;
    for (int k = threadIdx.x; k < in.item_count; k += B) s += P.res2_own[parity * P.n_items + in.item_begin + k];
    return block_sum<B>(s, red);
}

__device__ __forceinline__ ItemDev load_item(const Params& P, int it) {
    ItemDev item = P.items[it];
    item.inst = uni(item.inst);
    item.sub = uni(item.sub);
    return item;
}

// Synchronous sweeps: phase 1 updates every active item of the team from x^k
// into the other buffer and records its owned residual^2; after the grid
// barrier every workgroup assembles ||b - A x^k||^2 of its systems (same order
// everywhere, hence the same decision everywhere) and stops a system at the
// first k with relative residual < tol, returning x^k.
template <int B, class U>
__device__ __forceinline__ void run_sync(const Params& P, U& upd, TeamCtx& tc, double* red, int8_t* done) {
    const int tid = threadIdx.x;
    const int wg = blockIdx.x;
    const int ib = P.team_ptr[tc.team], ie = P.team_ptr[tc.team + 1];
    for (int j = tid; j < ie - ib; j += B) done[j] = 0;
    __syncthreads();
    for (int64_t s = P.sweep0;; ++s) {
        const int par = static_cast<int>(s & 1);
        for (int j = ib; j < ie; ++j) {
            if (done[j - ib]) continue;
            const int it = uni(P.team_items[j]);
            const ItemDev item = load_item(P, it);
            const InstU iu = load_inst(P.insts + item.inst);
            RAS_GLOBAL double* xc = par ? iu.x1 : iu.x0;
            RAS_GLOBAL double* xn = par ? iu.x0 : iu.x1;
            double own2, loc2, b2;
            const int64_t t_upd = wall_clock64();
            upd(P, tc, item, xc, xn, own2, loc2, b2);
            if (tid == 0 && tc.member == 0) {
                P.res2_own[par * P.n_items + it] = own2;
                P.solves[it] += 1;
                if (P.phase) {
                    int64_t* ph = P.phase + 4 * static_cast<int64_t>(it);
                    ph[0] += tc.st_res - t_upd;
                    ph[1] += tc.st_solve - tc.st_res;
                    ph[2] += wall_clock64() - tc.st_solve;
                }
            }
        }
        const int64_t t_bar = wall_clock64();
        grid_barrier(P.bar, static_cast<uint32_t>(P.n_wg));
        // uniform exit: every system's stop decision of an earlier sweep is visible now
        int running = 0;
        for (int k = tid; k < P.n_insts; k += B) running |= (P.ist[k].stopped_at < 0 || P.ist[k].stopped_at >= s);
        if (!__syncthreads_or(running)) break;
        const int64_t abort_at = P.bar->abort_at;
        int last_inst = -1;
        bool last_stop = false;
        for (int j = ib; j < ie; ++j) {
            if (done[j - ib]) continue;
            const int it = uni(P.team_items[j]);
            const ItemDev item = load_item(P, it);
            if (item.inst != last_inst) {
                const InstDev& in = P.insts[item.inst];
                const double sum = instance_owned_sum<B>(P, in, par, red);
                const double rel = sqrt(sum / in.bnorm2);
                last_stop = !(rel >= sqrt(in.tol2)) || s >= in.max_sweeps || abort_at <= s;
                last_inst = item.inst;
                if (tid == 0 && wg == in.leader && it == in.item_begin) {
                    InstState* st = P.ist + item.inst;
                    if (s < in.hist_cap) {
                        in.hist[s] = rel;
                        in.hist_t[s] = static_cast<double>(wall_clock64() - st->t0);
                        st->hist_len = s + 1;
                    }
                    if (last_stop) {
                        st->sweeps = s;
                        st->result_buf = par;
                        st->stopped_at = s;
                    }
                }
            }
            if (last_stop && tid == 0) done[j - ib] = 1;
        }
        if (wg == 0 && tid == 0 && P.max_ticks > 0 && abort_at > s + 1 &&
            wall_clock64() - P.ist[0].t0 > P.max_ticks)
            P.bar->abort_at = s + 1;
        // barrier wait and the convergence check, charged to the team's first item
        if (P.phase && tid == 0 && tc.member == 0)
            P.phase[4 * static_cast<int64_t>(P.team_items[ib]) + 3] += wall_clock64() - t_bar;
        __syncthreads();
    }
}

// Paced read (asynchronous mode): a subdomain about to read its neighbours
// waits, for at most `budget` wall-clock ticks, until every neighbour has
// published at least as many updates as it has itself.  Evenly loaded
// subdomains then read each other's latest update instead of the one before
// it; a slow neighbour costs at most the budget.  Every thread of the
// workgroup takes the same exits (both tests are block-wide votes).
template <int B>
__device__ __forceinline__ void paced_read_wait(const Params& P, const ItemDev& item, const InstDev& in, int it,
                                                int64_t budget) {
    const SubDev* sd = P.subs + item.sub;
    const int nn = uni(sd->n_nbr);
    const int32_t* nb = sd->nbr;
    const uint32_t mine = ld_rlx(P.version + it);
    const int64_t t0 = wall_clock64();
    for (;;) {
        int behind = 0;
        for (int k = threadIdx.x; k < nn; k += B) behind |= ld_rlx(P.version + in.item_begin + nb[k]) < mine;
        if (!__syncthreads_or(behind)) break;
        if (__syncthreads_or(wall_clock64() - t0 >= budget)) break;
        __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Asynchronous iteration: no grid barrier.  Decisions that steer team-wide
// control flow are taken by member 0 and broadcast to the team.
template <int B, class U>
__device__ __forceinline__ void run_async(const Params& P, U& upd, TeamCtx& tc, double* red, int8_t* done) {
    const int tid = threadIdx.x;
    const int wg = blockIdx.x;
    const int ib = P.team_ptr[tc.team], ie = P.team_ptr[tc.team + 1];
    __shared__ int flag;
    for (int j = tid; j < ie - ib; j += B) done[j] = 0;
    __syncthreads();
    int64_t last_dur = 0;  // wall-clock ticks of this workgroup's previous update (0: none yet)
    uint32_t ctl_visits = 0;  // item visits since the launch (host control words are polled on some)
    bool stalled = false;     // the previous visit found its subdomain paused
    for (;;) {
        bool any = false;
        for (int j = ib; j < ie; ++j) {
            if (done[j - ib]) continue;
            const int it = uni(P.team_items[j]);
            const ItemDev item = load_item(P, it);
            const InstDev& in = P.insts[item.inst];
            InstState* st = P.ist + item.inst;
            const int64_t t_item = wall_clock64();
            if (P.pace > 0.0 && tc.member == 0 && last_dur > 0)
                paced_read_wait<B>(P, item, in, it, static_cast<int64_t>(P.pace * static_cast<double>(last_dur)));
            const int64_t t_upd = wall_clock64();
            // 1: this item is finished; 2: the host has paused its subdomain
            int v0 = 0;
            if (tc.member == 0 && tid == 0) {
                // both host words in one round trip over the host link, on every 8th
                // visit and on every visit after a stall (a round trip costs about as
                // much as 1 % of a typical update)
                int32_t cz = 0, pz = 0;
                if (in.ctl && ((ctl_visits++ & 7) == 0 || stalled)) {
                    cz = __hip_atomic_load(in.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    pz = __hip_atomic_load(in.ctl + 1 + (it - in.item_begin), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                if (cz != 0) st_rlx(&st->stop, 2);  // cancelled by the host: ends like a time limit
                v0 = (ld_rlx(&st->stop) != 0) || (P.solves[it] >= in.max_sweeps) ||
                     (P.detect == 1 && ld_rlx(P.gflag + it) != 0);
                if (!v0 && pz != 0) v0 = 2;
            }
            const int state = team_bcast(tc, v0, &flag);
            stalled = state == 2;
            if (state == 1) {
                if (tid == 0) done[j - ib] = 1;
                __syncthreads();
                continue;
            }
            if (state == 2) {
                // a stalled subdomain: no update; the time limit still applies
                any = true;
                if (wg == in.leader && it == in.item_begin && tid == 0 && P.max_ticks > 0 &&
                    wall_clock64() - st->t0 > P.max_ticks)
                    st_rlx(&st->stop, 2);
                __syncthreads();
                continue;
            }
            any = true;
            double own2, loc2, b2;
            const InstU iu = load_inst(P.insts + item.inst);
            upd(P, tc, item, iu.x0, iu.x0, own2, loc2, b2);
            // The update wrote x[owned] = x[owned] + delta, delta computed from the
            // owned values this workgroup read in its residual.  The next residual
            // must read these stores, not older values still in flight (a
            // workgroup barrier does not wait for outstanding stores), or the
            // next correction would be added to a newer value than it was
            // computed from, i.e. counted twice.
            __builtin_amdgcn_s_waitcnt(0);
            team_barrier(tc);  // every member's part of x is written (and fenced) before the publish
            if (tid == 0 && tc.member == 0) {
                st_rlx(P.res2_own + it, own2);
                // the local criterion (eq. local_conv); the estimate detector only needs to
                // know that the subdomain has updated since the launch
                st_rlx(P.conv + it, static_cast<int32_t>(P.detect == 2 || loc2 < in.tol2 * b2));
                P.solves[it] += 1;
                __hip_atomic_fetch_add(P.version + it, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            const int64_t t_pub = wall_clock64();
            last_dur = t_pub - t_upd;
            if (P.detect == 1 && tc.member == 0) {
                // decentralized detection (Sec. 2.2, Sec. 3.3.2, after Bahi et al.): a
                // subdomain raises its global flag once it and every neighbour report
                // local convergence, or as soon as a neighbour's flag is up (flooding);
                // a flagged subdomain stops updating.
                const SubDev* sd = P.subs + item.sub;
                const int nn = uni(sd->n_nbr);
                const int32_t* nb = sd->nbr;
                int ok = 1, anyg = 0;
                for (int k = tid; k < nn; k += B) {
                    const int q = in.item_begin + nb[k];
                    ok &= ld_rlx(P.conv + q) != 0;
                    anyg |= ld_rlx(P.gflag + q) != 0;
                }
                ok = __syncthreads_and(ok);
                anyg = __syncthreads_or(anyg);
                if (tid == 0 && ((ok && loc2 < in.tol2 * b2) || anyg)) st_rlx(P.gflag + it, 1);
            }
            if (wg == in.leader && it == in.item_begin) {
                // centralized detector (Sec. 2.2): all local criteria + owned-residual estimate
                // (estimate detector: every subdomain updated + owned-residual estimate)
                int allc = 1;
                double sum = 0.0;
                for (int k = tid; k < in.item_count; k += B) {
                    allc &= ld_rlx(P.conv + in.item_begin + k);
                    sum += ld_rlx(P.res2_own + in.item_begin + k);
                }
                allc = __syncthreads_and(allc);
                sum = block_sum<B>(sum, red);
                if (tid == 0) {
                    const int64_t now = wall_clock64();
                    const int64_t h = st->hist_len;
                    if (h < in.hist_cap) {
                        in.hist[h] = sqrt(sum / in.bnorm2);
                        in.hist_t[h] = static_cast<double>(now - st->t0);
                        st->hist_len = h + 1;
                    }
                    st->sweeps += 1;
                    int32_t stop = 0;
                    if (!(sum == sum) || sum > 1e300) stop = 4;
                    else if (P.detect != 1 && allc && sum < in.tol2 * in.bnorm2) stop = 1;
                    else if (P.max_ticks > 0 && now - st->t0 > P.max_ticks) stop = 2;
                    if (stop) st_rlx(&st->stop, stop);
                }
            }
            if (P.phase && tid == 0 && tc.member == 0) {
                // residual (snapshot included), local solve, prolongation and publish,
                // other: paced wait before the read and detection after the publish
                int64_t* ph = P.phase + 4 * static_cast<int64_t>(it);
                ph[0] += tc.st_res - t_upd;
                ph[1] += tc.st_solve - tc.st_res;
                ph[2] += t_pub - tc.st_solve;
                ph[3] += (t_upd - t_item) + (wall_clock64() - t_pub);
            }
            __syncthreads();
        }
        if (!__syncthreads_or(any)) break;
    }
}

// ------------------------------------------------------------------------------ kernels
template <class CT, int KT, int R, bool ASYNC>
__global__ void __launch_bounds__(kCgThreads) cg_kernel(Params P) {
    __shared__ double red[kCgThreads / 64];
    __shared__ int8_t done[kMaxItemsPerWg];
    TeamCtx tc = make_team(P);
    CgUpdate<CT, KT, R, ASYNC> upd;
    if constexpr (ASYNC)
        run_async<kCgThreads>(P, upd, tc, red, done);
    else
        run_sync<kCgThreads>(P, upd, tc, red, done);
}

template <class ST, bool ASYNC>
__global__ void __launch_bounds__(kBandThreads) band_kernel(Params P, int max_w, int winm, int stage_bytes) {
    __shared__ double red[kBandThreads / 64];
    __shared__ int8_t done[kMaxItemsPerWg];
    TeamCtx tc = make_team(P);
    BandUpdate<ST, ASYNC> upd{max_w, winm, stage_bytes};
    if constexpr (ASYNC)
        run_async<kBandThreads>(P, upd, tc, red, done);
    else
        run_sync<kBandThreads>(P, upd, tc, red, done);
}

// ||b||^2 per instance and the exact residual ||b - A x||^2 (verification,
// Sec. 3.3.2), two-pass deterministic reductions.
constexpr int kRedThreads = 256;

__global__ void __launch_bounds__(kRedThreads)
    residual_partials(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                      const double* __restrict__ va, const double* __restrict__ b, const double* __restrict__ x,
                      double* __restrict__ part_r, double* __restrict__ part_b) {
    __shared__ double red[kRedThreads / 64];
    double sr = 0.0, sb = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRedThreads) {
        CompAcc ca{b[i], 0.0};
        if (x != nullptr)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) comp_sub(ca, va[e], x[ci[e]]);
        const double acc = comp_value(ca);
        sr += acc * acc;
        sb += b[i] * b[i];
    }
    sr = block_sum<kRedThreads>(sr, red);
    sb = block_sum<kRedThreads>(sb, red);
    if (threadIdx.x == 0) {
        part_r[blockIdx.x] = sr;
        part_b[blockIdx.x] = sb;
    }
}

__global__ void __launch_bounds__(kRedThreads)
    finish_partials(int nparts, const double* __restrict__ part_r, const double* __restrict__ part_b,
                    double* __restrict__ out /* [2]: r2, b2 */) {
    __shared__ double red[kRedThreads / 64];
    double sr = 0.0, sb = 0.0;
    for (int k = threadIdx.x; k < nparts; k += kRedThreads) {
        sr += part_r[k];
        sb += part_b[k];
    }
    sr = block_sum<kRedThreads>(sr, red);
    sb = block_sum<kRedThreads>(sb, red);
    if (threadIdx.x == 0) {
        out[0] = sr;
        out[1] = sb;
    }
}

__global__ void copy_vec(int64_t n, const double* __restrict__ src, double* __restrict__ dst) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        dst[i] = src[i];
}

__global__ void stamp_start(InstState* ist, int n) {
    const int64_t now = wall_clock64();
    for (int k = threadIdx.x; k < n; k += blockDim.x) ist[k].t0 = now;
}

// ------------------------------------------------------------------------------ host launchers
namespace {
template <class K>
hipError_t launch(K kern, dim3 grid, dim3 block, size_t lds, hipStream_t st, bool coop, void** args) {
    if (lds > 0) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    if (coop) return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), grid, block, args, lds, st);
    return hipLaunchKernel(reinterpret_cast<const void*>(kern), grid, block, args, lds, st);
}

template <class CT, int KT, bool ASYNC>
const void* cg_kernel_r(int r) {
    switch (r) {
        case 1: return reinterpret_cast<const void*>(cg_kernel<CT, KT, 1, ASYNC>);
        case 2: return reinterpret_cast<const void*>(cg_kernel<CT, KT, 2, ASYNC>);
        case 4: return reinterpret_cast<const void*>(cg_kernel<CT, KT, 4, ASYNC>);
        case 6: return reinterpret_cast<const void*>(cg_kernel<CT, KT, 6, ASYNC>);
        case 8: return reinterpret_cast<const void*>(cg_kernel<CT, KT, 8, ASYNC>);
        case 10: return reinterpret_cast<const void*>(cg_kernel<CT, KT, 10, ASYNC>);
        case 12: return reinterpret_cast<const void*>(cg_kernel<CT, KT, 12, ASYNC>);
        case 16: return reinterpret_cast<const void*>(cg_kernel<CT, KT, 16, ASYNC>);
        case 20: return reinterpret_cast<const void*>(cg_kernel<CT, KT, 20, ASYNC>);
        default: return nullptr;
    }
}

template <class CT, bool ASYNC>
const void* cg_kernel_for(int kt, int r) {
    if (kt == 5) return cg_kernel_r<CT, 5, ASYNC>(r);
    if (kt == 7) return cg_kernel_r<CT, 7, ASYNC>(r);
    return cg_kernel_r<CT, 0, ASYNC>(r);
}

template <class ST>
const void* band_kernel_for(bool async) {
    return async ? reinterpret_cast<const void*>(band_kernel<ST, true>)
                 : reinterpret_cast<const void*>(band_kernel<ST, false>);
}
}  // namespace

int cg_rows_class(int rows_per_member) {
    const int r = (rows_per_member + kCgThreads - 1) / kCgThreads;
    for (int c : {1, 2, 4, 6, 8, 10, 12, 16, 20})
        if (r <= c) return c;
    return -1;
}

const void* select_kernel(int solver, int storage, bool async, int ell_width, int rclass) {
    if (solver == 1) {  // CG
        if (storage == 0)
            return async ? cg_kernel_for<double, true>(ell_width, rclass) : cg_kernel_for<double, false>(ell_width, rclass);
        return async ? cg_kernel_for<float, true>(ell_width, rclass) : cg_kernel_for<float, false>(ell_width, rclass);
    }
    (void)rclass;
    if (storage == 0) return band_kernel_for<double>(async);
    if (storage == 1) return band_kernel_for<float>(async);
    return band_kernel_for<_Float16>(async);
}

hipError_t launch_solver(const void* kern, int solver, const Params& P, const int* band_args, size_t lds,
                         hipStream_t st, bool coop) {
    Params p = P;
    if (lds > 0) {
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    const dim3 grid(P.n_wg), block(solver == 1 ? kCgThreads : kBandThreads);
    if (solver == 1) {
        void* args[] = {&p};
        return coop ? hipLaunchCooperativeKernel(kern, grid, block, args, lds, st)
                    : hipLaunchKernel(kern, grid, block, args, lds, st);
    }
    int a0 = band_args[0], a1 = band_args[1], a2 = band_args[2];
    void* args[] = {&p, &a0, &a1, &a2};
    return coop ? hipLaunchCooperativeKernel(kern, grid, block, args, lds, st)
                : hipLaunchKernel(kern, grid, block, args, lds, st);
}

hipError_t occupancy(const void* kern, int solver, size_t lds, int* per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kern, solver == 1 ? kCgThreads : kBandThreads, lds);
}

hipError_t launch_residual(int64_t n, const int64_t* rp, const int32_t* ci, const double* va, const double* b,
                           const double* x, double* parts, int nparts, double* out, hipStream_t st) {
    residual_partials<<<nparts, kRedThreads, 0, st>>>(n, rp, ci, va, b, x, parts, parts + nparts);
    finish_partials<<<1, kRedThreads, 0, st>>>(nparts, parts, parts + nparts, out);
    return hipGetLastError();
}

hipError_t launch_copy(int64_t n, const double* src, double* dst, hipStream_t st) {
    copy_vec<<<1024, 256, 0, st>>>(n, src, dst);
    return hipGetLastError();
}

hipError_t launch_stamp(InstState* ist, int n, hipStream_t st) {
    stamp_start<<<1, 256, 0, st>>>(ist, n);
    return hipGetLastError();
}

// ---- banded Cholesky factorisation on the device --------------------------------------
// One workgroup per subdomain.  Right-looking: for each column j, the pivot
// L_jj = sqrt(a_jj), the column below it scaled by 1 / L_jj, then the rank-one
// update of the w x w window of rows j+1 .. j+w that the column reaches.  The
// band stays in global memory (each window is L2-resident); three workgroup
// barriers per column order the steps.
constexpr int kFactorThreads = 512;

__global__ void __launch_bounds__(kFactorThreads) band_factor_kernel(const FactorJob* __restrict__ jobs) {
    const FactorJob jb = jobs[blockIdx.x];
    const int n = jb.n, w = jb.w, ld = w + 1;
    const int tid = threadIdx.x;
    double* __restrict__ L = jb.L;
    __shared__ double colv[kMaxFactorW + 1];
    __shared__ int bad;
    for (int64_t e = tid; e < static_cast<int64_t>(n) * ld; e += kFactorThreads) L[e] = 0.0;
    if (tid == 0) bad = -1;
    __syncthreads();
    // A_p's lower band from the ELL rows; padding slots carry value 0 at the
    // row's own column, so entries are accumulated, never overwritten
    // (Robin transmission: the diagonal is lowered by a fraction of the row's
    // coupling to the external columns, slots >= n)
    for (int i = tid; i < n; i += kFactorThreads) {
        double out = 0.0;
        for (int k = 0; k < jb.K; ++k) {
            const int64_t slot = static_cast<int64_t>(k) * jb.n_pad + i;
            const int c = jb.ell_lcol[slot];
            if (c >= n) out += fabs(jb.ell_val[slot]);
            else if (c <= i && c >= i - w) L[static_cast<int64_t>(i) * ld + (c - i + w)] += jb.ell_val[slot];
        }
        L[static_cast<int64_t>(i) * ld + w] -= jb.robin_shift * out;
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            const double d = L[static_cast<int64_t>(j) * ld + w];
            if (!(d > 0.0) || !__builtin_isfinite(d)) {
                bad = j;
            } else {
                const double piv = sqrt(d);
                L[static_cast<int64_t>(j) * ld + w] = piv;
                colv[0] = 1.0 / piv;
            }
        }
        __syncthreads();
        if (bad >= 0) break;
        const int m = min(w, n - 1 - j);  // rows below the pivot inside the band
        const double inv = colv[0];
        for (int a = tid; a < m; a += kFactorThreads) {
            const int i = j + 1 + a;
            double* e = L + static_cast<int64_t>(i) * ld + (j - i + w);
            const double v = *e * inv;
            *e = v;
            colv[1 + a] = v;
        }
        __syncthreads();
        for (int q = tid; q < m * m; q += kFactorThreads) {
            const int a = q / m, c = q - a * m;
            if (c <= a) {
                const int i = j + 1 + a, k = j + 1 + c;
                L[static_cast<int64_t>(i) * ld + (k - i + w)] -= colv[1 + a] * colv[1 + c];
            }
        }
        __syncthreads();
    }
    if (tid == 0) *jb.fail = bad;
}

// float64 -> float16 bits, round to nearest even, in one rounding
__device__ __forceinline__ uint16_t f64_to_f16_bits(double d) {
    const uint64_t b = __builtin_bit_cast(uint64_t, d);
    const uint16_t sign = static_cast<uint16_t>((b >> 48) & 0x8000u);
    const int64_t ex = static_cast<int64_t>((b >> 52) & 0x7ff);
    const uint64_t man = b & ((1ull << 52) - 1);
    if (ex == 0x7ff) return static_cast<uint16_t>(sign | 0x7c00u | (man ? 0x200u : 0u));
    if (ex == 0) return sign;
    const int e = static_cast<int>(ex) - 1023;
    const uint64_t m = man | (1ull << 52);
    if (e > 15) return static_cast<uint16_t>(sign | 0x7c00u);
    if (e >= -14) {
        uint64_t q = m >> 42;
        const uint64_t rem = m & ((1ull << 42) - 1), half = 1ull << 41;
        if (rem > half || (rem == half && (q & 1))) ++q;
        int he = e + 15;
        if (q == 2048) {
            q = 1024;
            ++he;
        }
        if (he >= 31) return static_cast<uint16_t>(sign | 0x7c00u);
        return static_cast<uint16_t>(sign | (he << 10) | (q & 0x3ffu));
    }
    const int sh = 28 - e;
    if (sh > 63) return sign;
    uint64_t q = m >> sh;
    const uint64_t rem = m & ((1ull << sh) - 1), half = 1ull << (sh - 1);
    if (rem > half || (rem == half && (q & 1))) ++q;
    return static_cast<uint16_t>(sign | q);
}

// FP16_ROWSCALED: s_i = float32(max_o |L_io|) (1 for an all-zero row)
__global__ void band_scale_kernel(const FactorJob* __restrict__ jobs) {
    const FactorJob jb = jobs[blockIdx.y];
    const int ld = jb.w + 1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < jb.n; i += gridDim.x * blockDim.x) {
        double mx = 0.0;
        for (int o = 0; o < ld; ++o) mx = fmax(mx, fabs(jb.L[static_cast<int64_t>(i) * ld + o]));
        float sc = static_cast<float>(mx);
        if (!(sc > 0.0f)) sc = 1.0f;
        jb.scale[i] = sc;
    }
}

// The factor as the triangular solves read it: entry (t, o) of L and of the
// reversed transpose (row (n-1-t) + w - o of L at offset o) in the storage type,
// at the slab position ((t / BR) w + o) BR + t % BR (o < w; the diagonal is kept
// as its reciprocal in invd) or the row-major position t (w+1) + o.
template <int ST>
__global__ void band_layout_kernel(const FactorJob* __restrict__ jobs) {
    const FactorJob jb = jobs[blockIdx.y];
    const int n = jb.n, w = jb.w, ld = w + 1;
    const int olim = jb.slab ? w : ld;
    const int64_t total = static_cast<int64_t>(n) * olim;
    const double* L = jb.L;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int t = static_cast<int>(e / olim), o = static_cast<int>(e - static_cast<int64_t>(t) * olim);
        const int r = (n - 1 - t) + w - o;  // row of L read by the reversed transpose
        const int64_t di = jb.slab ? (static_cast<int64_t>(t / kBandRows) * w + o) * kBandRows + t % kBandRows
                                   : static_cast<int64_t>(t) * ld + o;
        const double lf = L[static_cast<int64_t>(t) * ld + o];
        const double lb = r < n ? L[static_cast<int64_t>(r) * ld + o] : 0.0;
        if constexpr (ST == RAS_STORAGE_FP64) {
            static_cast<double*>(jb.band_f)[di] = lf;
            static_cast<double*>(jb.band_b)[di] = lb;
        } else if constexpr (ST == RAS_STORAGE_FP32) {
            static_cast<float*>(jb.band_f)[di] = static_cast<float>(lf);
            static_cast<float*>(jb.band_b)[di] = static_cast<float>(lb);
        } else {
            static_cast<uint16_t*>(jb.band_f)[di] = f64_to_f16_bits(lf / static_cast<double>(jb.scale[t]));
            static_cast<uint16_t*>(jb.band_b)[di] =
                r < n ? f64_to_f16_bits(lb / static_cast<double>(jb.scale[r])) : static_cast<uint16_t>(0);
        }
        if (o == 0) {
            // reciprocal of the diagonal as the triangular solves see it
            const double dg = L[static_cast<int64_t>(t) * ld + w];
            if constexpr (ST == RAS_STORAGE_FP64) {
                static_cast<double*>(jb.invd)[t] = 1.0 / dg;
            } else if constexpr (ST == RAS_STORAGE_FP32) {
                static_cast<float*>(jb.invd)[t] =
                    static_cast<float>(1.0 / static_cast<double>(static_cast<float>(dg)));
            } else {
                const uint16_t hb = f64_to_f16_bits(dg / static_cast<double>(jb.scale[t]));
                const float deq = static_cast<float>(__builtin_bit_cast(_Float16, hb)) * jb.scale[t];
                static_cast<float*>(jb.invd)[t] = static_cast<float>(1.0 / static_cast<double>(deq));
            }
        }
    }
}

// FP64 / FP32 slab factors: the triangle slots of every 32-row block (of L for
// the forward pass, of its reversed transpose for the backward pass) receive the
// strictly lower part of the inverse G of the block's diagonal triangle T,
// computed in float64 (FP32: from T rounded to float32, the factor the solves
// use), so the solver applies the triangle as y = G c.  One workgroup per block,
// a thread per column of G (forward substitution on the unit vector).
template <int ST>
__global__ void __launch_bounds__(64) block_inverse_kernel(const FactorJob* __restrict__ jobs) {
    const FactorJob jb = jobs[blockIdx.z];
    if (!jb.tri_inv) return;
    constexpr int BR = kBandRows;
    const int n = jb.n, w = jb.w, ld = w + 1;
    const int nblk = (n + BR - 1) / BR;
    const bool rev = blockIdx.y == 1;
    __shared__ double T[BR][BR + 1];
    __shared__ double G[BR][BR + 1];
    for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int t0 = blk * BR;
        for (int e = threadIdx.x; e < BR * BR; e += 64) {
            const int r = e / BR, c = e - (e / BR) * BR;
            double v = r == c ? 1.0 : 0.0;  // rows past n: identity
            if (c <= r && t0 + r < n) {
                // entry (t0 + r, t0 + c) of L, or of its reversed transpose
                // (= L[n-1-(t0+c)][n-1-(t0+r)]); both at band offset c - r + w;
                // as the solves see it (FP32: rounded; FP16: quantised, then dequantised)
                const int64_t i = rev ? static_cast<int64_t>(n - 1 - t0 - c) : static_cast<int64_t>(t0 + r);
                v = jb.L[i * ld + (c - r + w)];
                if constexpr (ST == RAS_STORAGE_FP32) v = static_cast<double>(static_cast<float>(v));
                if constexpr (ST == RAS_STORAGE_FP16_ROWSCALED) {
                    const float s = jb.scale[i];
                    const uint16_t hb = f64_to_f16_bits(v / static_cast<double>(s));
                    v = static_cast<double>(static_cast<float>(__builtin_bit_cast(_Float16, hb)) * s);
                }
            }
            T[r][c] = v;
        }
        __syncthreads();
        if (threadIdx.x < BR) {
            const int m = threadIdx.x;
            for (int r = 0; r < BR; ++r) {
                if (r < m) {
                    G[r][m] = 0.0;
                    continue;
                }
                double s = r == m ? 1.0 : 0.0;
                for (int k = m; k < r; ++k) s -= T[r][k] * G[k][m];
                G[r][m] = s / T[r][r];
            }
        }
        __syncthreads();
        void* dst = rev ? jb.band_b : jb.band_f;
        float* gdst = jb.tri_g[rev ? 1 : 0];
        for (int e = threadIdx.x; e < BR * BR; e += 64) {
            const int r = e / BR, c = e - (e / BR) * BR;
            if constexpr (ST == RAS_STORAGE_FP16_ROWSCALED) {
                // packed float32 rows (row r at r (r - 1) / 2), zero past n
                if (c < r) gdst[static_cast<int64_t>(blk) * kTriPackFloats + (r * (r - 1)) / 2 + c] =
                    t0 + r < n ? static_cast<float>(G[r][c]) : 0.0f;
            } else if (c < r && t0 + r < n) {
                const int64_t di = (static_cast<int64_t>(blk) * w + (w - r + c)) * BR + r;
                if constexpr (ST == RAS_STORAGE_FP64) static_cast<double*>(dst)[di] = G[r][c];
                else static_cast<float*>(dst)[di] = static_cast<float>(G[r][c]);
            }
        }
        __syncthreads();
    }
}

hipError_t launch_band_factor(const FactorJob* jobs, int njobs, int storage, int max_n, hipStream_t st) {
    band_factor_kernel<<<njobs, kFactorThreads, 0, st>>>(jobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(std::max(1, std::min(64, (max_n + 255) / 256)), njobs);
    if (storage == RAS_STORAGE_FP16_ROWSCALED) {
        band_scale_kernel<<<grid, 256, 0, st>>>(jobs);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const dim3 lgrid(256, njobs);
    if (storage == RAS_STORAGE_FP64) band_layout_kernel<RAS_STORAGE_FP64><<<lgrid, 256, 0, st>>>(jobs);
    else if (storage == RAS_STORAGE_FP32) band_layout_kernel<RAS_STORAGE_FP32><<<lgrid, 256, 0, st>>>(jobs);
    else band_layout_kernel<RAS_STORAGE_FP16_ROWSCALED><<<lgrid, 256, 0, st>>>(jobs);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 igrid(std::max(1, std::min(256, (max_n + kBandRows - 1) / kBandRows)), 2, njobs);
    if (storage == RAS_STORAGE_FP64) block_inverse_kernel<RAS_STORAGE_FP64><<<igrid, 64, 0, st>>>(jobs);
    else if (storage == RAS_STORAGE_FP32) block_inverse_kernel<RAS_STORAGE_FP32><<<igrid, 64, 0, st>>>(jobs);
    else block_inverse_kernel<RAS_STORAGE_FP16_ROWSCALED><<<igrid, 64, 0, st>>>(jobs);
    return hipGetLastError();
}

// ---- fixed workspace of the solve that allocates nothing ---------------------------
// Every device that loads this code object holds one copy of the array until
// the process ends.  Host code never uses the array's name as an address: the
// device address of each device's copy comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is handed
// to kernels and copies.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void** ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (addr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace ras
