// Host-side setup: validation, partitioning, overlap, local factorisation.
// Built with -ffp-contract=off so the partitioner's float64 arithmetic is
// plain IEEE (no fused multiply-add), which keeps its index sets identical to
// any other IEEE implementation of the same formulas.
#include "plan.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

namespace ras {

int worker_count() {
    unsigned hc = std::thread::hardware_concurrency();
    int n = hc == 0 ? 1 : static_cast<int>(hc);
    return std::min(n, 16);
}

// ------------------------------------------------------------------------------ CSR checks
void validate_csr(const ras_csr& A) {
    if (A.n < 1 || A.n > INT32_MAX) throw Error{RAS_E_ARG, "n must be in [1, 2^31)"};
    if (!A.row_ptr || !A.col || !A.val) throw Error{RAS_E_ARG, "null CSR array"};
    if (A.row_ptr[0] != 0) throw Error{RAS_E_PATTERN, "row_ptr[0] != 0"};
    for (int64_t i = 0; i < A.n; ++i) {
        int64_t a = A.row_ptr[i], b = A.row_ptr[i + 1];
        if (b < a) throw Error{RAS_E_PATTERN, "row_ptr not monotone at row " + std::to_string(i)};
        for (int64_t e = a; e < b; ++e) {
            int32_t c = A.col[e];
            if (c < 0 || c >= A.n) throw Error{RAS_E_PATTERN, "column out of range in row " + std::to_string(i)};
            if (e > a && A.col[e - 1] >= c)
                throw Error{RAS_E_PATTERN, "columns not sorted/unique in row " + std::to_string(i)};
            if (!std::isfinite(A.val[e])) throw Error{RAS_E_ARG, "non-finite value in row " + std::to_string(i)};
        }
    }
    // symmetric pattern: every (i, j) has a stored (j, i)
    for (int64_t i = 0; i < A.n; ++i) {
        for (int64_t e = A.row_ptr[i]; e < A.row_ptr[i + 1]; ++e) {
            int32_t j = A.col[e];
            const int32_t* lo = A.col + A.row_ptr[j];
            const int32_t* hi = A.col + A.row_ptr[j + 1];
            if (!std::binary_search(lo, hi, static_cast<int32_t>(i)))
                throw Error{RAS_E_PATTERN, "pattern not symmetric at (" + std::to_string(i) + "," +
                                               std::to_string(j) + ")"};
        }
    }
}

// ------------------------------------------------------------------------------ partitions
uint64_t splitmix64_next(uint64_t& state) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static std::vector<int32_t> axis_slabs(int32_t extent, int32_t parts) {
    std::vector<int32_t> s(extent);
    for (int32_t q = 0; q < parts; ++q) {
        int64_t lo = static_cast<int64_t>(q) * extent / parts;
        int64_t hi = static_cast<int64_t>(q + 1) * extent / parts;
        for (int64_t i = lo; i < hi; ++i) s[i] = q;
    }
    return s;
}

static void rcb(const int32_t nx, const int32_t ny, const int32_t nz, int32_t P, uint64_t seed, double jitter,
                std::vector<int32_t>& owner) {
    const int64_t n = static_cast<int64_t>(nx) * ny * nz;
    std::vector<double> w(P);
    uint64_t st = seed;
    for (int32_t q = 0; q < P; ++q) {
        uint64_t z = splitmix64_next(st);
        double u = static_cast<double>(z >> 11) * 0x1.0p-53;
        w[q] = 1.0 + jitter * (2.0 * u - 1.0);
    }
    std::vector<int32_t> pts(n);
    for (int64_t g = 0; g < n; ++g) pts[g] = static_cast<int32_t>(g);
    auto coord = [&](int32_t g, int axis) -> int32_t {
        if (axis == 0) return g % nx;
        if (axis == 1) return (g / nx) % ny;
        return g / (nx * ny);
    };
    struct Task {
        int64_t begin, end;
        int32_t p0, m;
    };
    std::vector<Task> stack{{0, n, 0, P}};
    while (!stack.empty()) {
        Task t = stack.back();
        stack.pop_back();
        if (t.m == 1) {
            for (int64_t e = t.begin; e < t.end; ++e) owner[pts[e]] = t.p0;
            continue;
        }
        const int32_t ml = t.m / 2;
        int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
        for (int64_t e = t.begin; e < t.end; ++e)
            for (int a = 0; a < 3; ++a) {
                int32_t c = coord(pts[e], a);
                lo[a] = std::min(lo[a], c);
                hi[a] = std::max(hi[a], c);
            }
        int axis = 0;
        for (int a = 1; a < 3; ++a)
            if (hi[a] - lo[a] > hi[axis] - lo[axis]) axis = a;
        std::sort(pts.begin() + t.begin, pts.begin() + t.end, [&](int32_t a, int32_t b) {
            int32_t ca = coord(a, axis), cb = coord(b, axis);
            return ca != cb ? ca < cb : a < b;
        });
        double Wl = 0.0;
        for (int32_t q = t.p0; q < t.p0 + ml; ++q) Wl += w[q];
        double W = Wl;
        for (int32_t q = t.p0 + ml; q < t.p0 + t.m; ++q) W += w[q];
        const int64_t S = t.end - t.begin;
        double prod = static_cast<double>(S) * Wl;
        double ratio = prod / W;
        int64_t cut = static_cast<int64_t>(std::floor(ratio + 0.5));
        cut = std::min<int64_t>(std::max<int64_t>(cut, ml), S - (t.m - ml));
        stack.push_back({t.begin, t.begin + cut, t.p0, ml});
        stack.push_back({t.begin + cut, t.end, t.p0 + ml, t.m - ml});
    }
}

std::vector<int32_t> make_owner(const ras_csr& A, const ras_partition& part, int32_t* P_out) {
    const int64_t n = A.n;
    std::vector<int32_t> owner(n, -1);
    auto need_grid = [&]() {
        int64_t prod = static_cast<int64_t>(part.grid[0]) * part.grid[1] * part.grid[2];
        if (part.grid[0] < 1 || part.grid[1] < 1 || part.grid[2] < 1 || prod != n)
            throw Error{RAS_E_ARG, "grid[0]*grid[1]*grid[2] must equal n"};
    };
    int32_t P = 0;
    switch (part.kind) {
        case RAS_PART_REGULAR_1D: {
            P = part.parts[0];
            if (P < 1 || P > n) throw Error{RAS_E_ARG, "REGULAR_1D needs 1 <= parts[0] <= n"};
            for (int32_t p = 0; p < P; ++p) {
                int64_t lo = static_cast<int64_t>(p) * n / P, hi = static_cast<int64_t>(p + 1) * n / P;
                for (int64_t g = lo; g < hi; ++g) owner[g] = p;
            }
            break;
        }
        case RAS_PART_REGULAR_2D:
        case RAS_PART_REGULAR_3D: {
            need_grid();
            int32_t px = part.parts[0], py = part.parts[1];
            int32_t pz = part.kind == RAS_PART_REGULAR_3D ? part.parts[2] : 1;
            if (px < 1 || py < 1 || pz < 1 || px > part.grid[0] || py > part.grid[1] || pz > part.grid[2])
                throw Error{RAS_E_ARG, "regular partition needs 1 <= parts[a] <= grid[a]"};
            auto sx = axis_slabs(part.grid[0], px), sy = axis_slabs(part.grid[1], py),
                 sz = axis_slabs(part.grid[2], pz);
            const int32_t nx = part.grid[0], ny = part.grid[1];
            for (int64_t g = 0; g < n; ++g) {
                int32_t i = static_cast<int32_t>(g % nx), j = static_cast<int32_t>((g / nx) % ny),
                        k = static_cast<int32_t>(g / (static_cast<int64_t>(nx) * ny));
                owner[g] = sx[i] + px * (sy[j] + py * sz[k]);
            }
            P = px * py * pz;
            break;
        }
        case RAS_PART_RCB: {
            need_grid();
            P = part.parts[0];
            if (P < 1 || P > n) throw Error{RAS_E_ARG, "RCB needs 1 <= parts[0] <= n"};
            if (!(part.jitter >= 0.0 && part.jitter < 1.0)) throw Error{RAS_E_ARG, "RCB jitter must be in [0, 1)"};
            rcb(part.grid[0], part.grid[1], part.grid[2], P, part.seed, part.jitter, owner);
            break;
        }
        case RAS_PART_EXPLICIT: {
            P = part.parts[0];
            if (!part.owner || P < 1 || P > n) throw Error{RAS_E_ARG, "EXPLICIT needs owner[] and 1 <= parts[0] <= n"};
            std::vector<uint8_t> seen(P, 0);
            for (int64_t g = 0; g < n; ++g) {
                int32_t o = part.owner[g];
                if (o < 0 || o >= P) throw Error{RAS_E_ARG, "EXPLICIT owner out of range at " + std::to_string(g)};
                owner[g] = o;
                seen[o] = 1;
            }
            for (int32_t p = 0; p < P; ++p)
                if (!seen[p]) throw Error{RAS_E_ARG, "EXPLICIT part " + std::to_string(p) + " is empty"};
            break;
        }
        default:
            throw Error{RAS_E_ARG, "unknown partition kind"};
    }
    *P_out = P;
    return owner;
}

// ------------------------------------------------------------------------------ overlap
void build_overlap(Plan& plan) {
    const int32_t P = plan.P;
    std::vector<std::vector<int32_t>> owned(P);
    for (int64_t g = 0; g < plan.n; ++g) owned[plan.owner[g]].push_back(static_cast<int32_t>(g));
    plan.subs.assign(P, Subdomain{});
    // one visited array per worker, keyed by subdomain id so it never needs clearing
    std::vector<std::vector<int32_t>> marks(worker_count());
    parallel_for(P, [&](int64_t p, int worker) {
        std::vector<int32_t>& vis = marks[worker];
        if (vis.empty()) vis.assign(plan.n, -1);
        Subdomain& sd = plan.subs[p];
        std::vector<int32_t> all = owned[p];
        for (int32_t g : all) vis[g] = static_cast<int32_t>(p);
        std::vector<int32_t> frontier = all, next;
        for (int32_t l = 0; l < plan.overlap; ++l) {
            next.clear();
            for (int32_t g : frontier)
                for (int64_t e = plan.row_ptr[g]; e < plan.row_ptr[g + 1]; ++e) {
                    int32_t c = plan.col[e];
                    if (vis[c] != p) {
                        vis[c] = static_cast<int32_t>(p);
                        next.push_back(c);
                    }
                }
            all.insert(all.end(), next.begin(), next.end());
            frontier.swap(next);
        }
        std::sort(all.begin(), all.end());
        sd.omega = std::move(all);
        sd.owned.resize(sd.omega.size());
        int32_t no = 0, width = 0, w = 0;
        for (size_t i = 0; i < sd.omega.size(); ++i) {
            int32_t g = sd.omega[i];
            sd.owned[i] = plan.owner[g] == p;
            no += sd.owned[i];
            width = std::max<int32_t>(width, static_cast<int32_t>(plan.row_ptr[g + 1] - plan.row_ptr[g]));
            // lower half-bandwidth over stored entries whose column lies in omega
            for (int64_t e = plan.row_ptr[g]; e < plan.row_ptr[g + 1]; ++e) {
                int32_t c = plan.col[e];
                if (c >= g) break;
                auto it = std::lower_bound(sd.omega.begin(), sd.omega.end(), c);
                if (it != sd.omega.end() && *it == c) {
                    w = std::max<int32_t>(w, static_cast<int32_t>(i - (it - sd.omega.begin())));
                    break;  // columns ascend: the first local one gives the widest reach
                }
            }
        }
        sd.n_owned = no;
        sd.ell_width = width;
        // the stored band keeps at least one sub-diagonal (zero for a diagonal
        // local matrix): the device layout writes each row's diagonal reciprocal
        // together with its first band entry, and sizes its stages by w
        sd.w = std::max<int32_t>(w, 1);
    });
}

std::vector<int32_t> external_set(const Plan& plan, const Subdomain& sd) {
    std::vector<int32_t> xe;
    for (int32_t g : sd.omega)
        for (int64_t e = plan.row_ptr[g]; e < plan.row_ptr[g + 1]; ++e) {
            const int32_t c = plan.col[e];
            if (!std::binary_search(sd.omega.begin(), sd.omega.end(), c)) xe.push_back(c);
        }
    std::sort(xe.begin(), xe.end());
    xe.erase(std::unique(xe.begin(), xe.end()), xe.end());
    return xe;
}

void comm_volume(const Plan& plan, int64_t* volume) {
    const int64_t P = plan.P;
    std::fill(volume, volume + P * P, int64_t{0});
    parallel_for(P, [&](int64_t p, int) {
        int64_t* row = volume + p * P;
        const Subdomain& sd = plan.subs[p];
        for (int32_t g : sd.omega)
            if (plan.owner[g] != p) ++row[plan.owner[g]];
        for (int32_t g : external_set(plan, sd)) ++row[plan.owner[g]];  // never owned by p
    });
}

// ------------------------------------------------------------------------------ factorisation
uint16_t f64_to_f16_rne(double d) {
    uint64_t b;
    std::memcpy(&b, &d, 8);
    const uint16_t sign = static_cast<uint16_t>((b >> 48) & 0x8000u);
    const int64_t ex = static_cast<int64_t>((b >> 52) & 0x7ff);
    const uint64_t man = b & ((1ull << 52) - 1);
    if (ex == 0x7ff) return static_cast<uint16_t>(sign | 0x7c00u | (man ? 0x200u : 0u));
    if (ex == 0) return sign;  // zero or float64 subnormal: rounds to a signed zero in float16
    const int e = static_cast<int>(ex) - 1023;
    const uint64_t m = man | (1ull << 52);  // value = m * 2^(e - 52)
    if (e > 15) return static_cast<uint16_t>(sign | 0x7c00u);
    if (e >= -14) {
        const int sh = 42;
        uint64_t q = m >> sh, rem = m & ((1ull << sh) - 1), half = 1ull << (sh - 1);
        if (rem > half || (rem == half && (q & 1))) ++q;
        int he = e + 15;
        if (q == 2048) {
            q = 1024;
            ++he;
        }
        if (he >= 31) return static_cast<uint16_t>(sign | 0x7c00u);
        return static_cast<uint16_t>(sign | (he << 10) | (q & 0x3ffu));
    }
    const int sh = 28 - e;  // value / 2^-24 = m * 2^(e + 24 - 52)
    if (sh > 63) return sign;
    uint64_t q = m >> sh, rem = m & ((1ull << sh) - 1), half = 1ull << (sh - 1);
    if (rem > half || (rem == half && (q & 1))) ++q;
    return static_cast<uint16_t>(sign | q);  // q == 1024 encodes the smallest normal
}

void factor_one(const Plan& plan, Subdomain& sd, int32_t p) {
    const int64_t n = static_cast<int64_t>(sd.omega.size());
    const int32_t w = sd.w;
    const int64_t ld = w + 1;
    sd.L.assign(n * ld, 0.0);
    double* L = sd.L.data();
    // scatter the lower band of A[omega, omega]; Robin transmission lowers the
    // diagonal by a fraction of the row's coupling to points outside omega
    const double shift = robin_shift_factor(plan.local);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t g = sd.omega[i];
        double out = 0.0;
        for (int64_t e = plan.row_ptr[g]; e < plan.row_ptr[g + 1]; ++e) {
            const int32_t c = plan.col[e];
            auto it = std::lower_bound(sd.omega.begin(), sd.omega.end(), c);
            if (it == sd.omega.end() || *it != c) {
                out += std::fabs(plan.val[e]);
                continue;
            }
            if (c > g) continue;
            const int64_t j = it - sd.omega.begin();
            L[i * ld + (j - i + w)] = plan.val[e];
        }
        L[i * ld + w] -= shift * out;
    }
    // row-oriented (Cholesky-Banachiewicz) band factorisation, in place
    for (int64_t i = 0; i < n; ++i) {
        double* Li = L + i * ld;
        const int64_t j0 = std::max<int64_t>(0, i - w);
        for (int64_t j = j0; j <= i; ++j) {
            const double* Lj = L + j * ld;
            const int64_t k0 = std::max<int64_t>(j0, j - w);
            double s = Li[j - i + w];
            for (int64_t k = k0; k < j; ++k) s -= Li[k - i + w] * Lj[k - j + w];
            if (j < i) {
                Li[j - i + w] = s / Lj[w];
            } else {
                if (!(s > 0.0) || !std::isfinite(s))
                    throw Error{RAS_E_NOT_SPD, "non-positive pivot in subdomain " + std::to_string(p) +
                                                   " at local row " + std::to_string(i)};
                Li[w] = std::sqrt(s);
            }
        }
    }
    if (plan.local.storage == RAS_STORAGE_FP16_ROWSCALED) {
        sd.Lh.assign(n * ld, 0);
        sd.scale.assign(n, 1.0f);
        for (int64_t i = 0; i < n; ++i) {
            double mx = 0.0;
            for (int64_t o = 0; o < ld; ++o) mx = std::max(mx, std::fabs(L[i * ld + o]));
            float s = static_cast<float>(mx);
            if (!(s > 0.0f)) s = 1.0f;
            sd.scale[i] = s;
            const double sd64 = static_cast<double>(s);
            for (int64_t o = 0; o < ld; ++o) sd.Lh[i * ld + o] = f64_to_f16_rne(L[i * ld + o] / sd64);
        }
    }
}

void factor_local(Plan& plan) {
    parallel_for(plan.P, [&](int64_t p, int) { factor_one(plan, plan.subs[p], static_cast<int32_t>(p)); });
}

}  // namespace ras
