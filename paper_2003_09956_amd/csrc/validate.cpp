// Host-side argument checks and admission accounting (see validate.hpp).
#include "validate.hpp"

#include <cmath>
#include <cstring>
#include <unordered_set>

namespace modap_host {

namespace {

modap_status bad(const char **msg, modap_status st, const char *what) {
    if (msg) *msg = what;
    return st;
}

double element(int dt, const void *p, size_t idx) {
    if (dt == MODAP_F64) return static_cast<const double *>(p)[idx];
    if (dt == MODAP_F32) return static_cast<const float *>(p)[idx];
    const uint32_t u = (uint32_t)static_cast<const uint16_t *>(p)[idx] << 16;   // bfloat16: upper half of a binary32
    float f;
    std::memcpy(&f, &u, sizeof f);
    return f;
}

}  // namespace

size_t storage_bytes(int dt) { return dt == MODAP_F64 ? 8 : dt == MODAP_F32 ? 4 : 2; }

int64_t padded_length(int dt, int64_t n) {
    const int64_t v = 16 / (int64_t)storage_bytes(dt);
    return (n + v - 1) / v * v;
}

modap_status check_params(const modap_params *p, const char **msg) {
    if (!p) return bad(msg, MODAP_E_INVAL, "params is NULL");
    if (!(p->lambda > 0.0) || !std::isfinite(p->lambda)) return bad(msg, MODAP_E_INVAL, "lambda must be finite and > 0");
    if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return bad(msg, MODAP_E_INVAL, "eps must be finite and > 0");
    if (p->step != MODAP_STEP_FIXED && p->step != MODAP_STEP_AVG) return bad(msg, MODAP_E_INVAL, "unknown step rule");
    if (p->max_iters < 0) return bad(msg, MODAP_E_INVAL, "max_iters must be >= 0");
    if (p->profile < 0) return bad(msg, MODAP_E_INVAL, "profile must be >= 0");
    return MODAP_OK;
}

modap_status check_system(int64_t m, int64_t n, int64_t lda, const void *A, const double *b, int dt,
                          const char **msg) {
    if (m < 1 || n < 1) return bad(msg, MODAP_E_INVAL, "m and n must be >= 1");
    if (lda < n) return bad(msg, MODAP_E_INVAL, "lda < n");
    if (!A || !b) return bad(msg, MODAP_E_INVAL, "A and b are required");
    if (dt != MODAP_F64 && dt != MODAP_F32 && dt != MODAP_BF16) return bad(msg, MODAP_E_INVAL, "unknown storage type");
    return MODAP_OK;
}

bool all_finite(const double *p, int64_t count) {
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

modap_status check_rows(int64_t k, const int64_t *rows, const void *new_rows, const double *new_b, int64_t m,
                        const char **msg) {
    if (k < 0 || k > m) return bad(msg, MODAP_E_INVAL, "k out of range");
    if (k > 0 && (!rows || !new_rows || !new_b)) return bad(msg, MODAP_E_INVAL, "rows, new_rows and new_b are required");
    std::unordered_set<int64_t> seen;
    for (int64_t q = 0; q < k; ++q) {
        if (rows[q] < 0 || rows[q] >= m) return bad(msg, MODAP_E_INVAL, "row index out of range");
        if (!seen.insert(rows[q]).second) return bad(msg, MODAP_E_INVAL, "row indices must be distinct");
        if (!std::isfinite(new_b[q])) return bad(msg, MODAP_E_INVAL, "new_b has a non-finite entry");
    }
    return MODAP_OK;
}

modap_status check_new_rows(int dt, const void *new_rows, int64_t k, int64_t n, const char **msg) {
    for (int64_t q = 0; q < k; ++q) {
        double s2 = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double v = element(dt, new_rows, (size_t)(q * n + j));
            if (!std::isfinite(v)) return bad(msg, MODAP_E_ZERO_ROW, "replacement row has a non-finite entry");
            s2 += v * v;
        }
        if (!(s2 > 0.0)) return bad(msg, MODAP_E_ZERO_ROW, "replacement row is zero");
    }
    return MODAP_OK;
}

modap_status check_drift(int64_t T, const double *V, int64_t ldv, int64_t n, bool host, const char **msg) {
    if (T < 0) return bad(msg, MODAP_E_INVAL, "T < 0");
    if (T > 0 && V && ldv < n) return bad(msg, MODAP_E_INVAL, "ldv < n");
    if (T > 0 && V && host)
        for (int64_t s = 0; s < T; ++s)
            if (!all_finite(V + s * ldv, n)) return bad(msg, MODAP_E_INVAL, "drift has a non-finite entry");
    return MODAP_OK;
}

double request_footprint(int dt, int64_t m, int64_t n, int64_t T) {
    const double ldA = (double)padded_length(dt, n);
    const double acc = dt == MODAP_F64 ? 8.0 : 4.0;
    return (double)m * ldA * (double)storage_bytes(dt) + 32.0 * (double)m + 6.0 * 8.0 * ldA + 6.0 * acc * ldA +
           acc * ldA * (double)((m + 63) / 64) + 8.0 * ldA * (double)T + 65536.0;
}

bool admissible(double used, double footprint, double budget, int64_t live, int64_t max_live) {
    if (used + footprint > budget) return false;
    if (max_live > 0 && live >= max_live) return false;
    return true;
}

modap_status check_request(int64_t m, int64_t n, const void *A, const double *b, int64_t T, const double *V,
                           int64_t ldv, const char **msg) {
    if (m < 1 || n < 1 || !A || !b) return bad(msg, MODAP_E_INVAL, "bad sizes or NULL data");
    if (T < 0 || (T > 0 && (!V || ldv < n))) return bad(msg, MODAP_E_INVAL, "bad drift schedule");
    return MODAP_OK;
}

}  // namespace modap_host
