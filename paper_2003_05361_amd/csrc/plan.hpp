// Host-side setup of the restricted additive Schwarz solver (no GPU code).
//
// Builds, from the global CSR matrix and a partition description, the
// per-subdomain data the device kernels consume: owned and overlapping index
// sets (Sec. 3.2.1, Sec. 2.1 Fig. 1), the rows of A on each overlapping set
// (Sec. 3.2.2) and, for the direct local solver, the float64 banded Cholesky
// factor of each local matrix (Sec. 3.3.1).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ras.h"

namespace ras {

struct Subdomain {
    std::vector<int32_t> omega;  // overlapping set, ascending global ids
    std::vector<uint8_t> owned;  // owned[i] != 0 iff omega[i] is owned by this subdomain
    int32_t n_owned = 0;
    int32_t ell_width = 0;       // max stored entries in a row of A over omega
    int32_t w = 0;               // lower half-bandwidth of A[omega, omega]
    std::vector<double> L;       // Cholesky: row-major lower band, L[i*(w+1) + (j-i+w)]
    std::vector<uint16_t> Lh;    // FP16_ROWSCALED: float16 bits of L / scale(row)
    std::vector<float> scale;    // FP16_ROWSCALED: per-row scale
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
uint16_t f64_to_f16_rne(double d);

uint64_t splitmix64_next(uint64_t& state);

int worker_count();

}  // namespace ras
