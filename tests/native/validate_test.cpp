// Test driver of the library's host-side checks and admission accounting
// (paper_2003_09956_amd/csrc/validate.cpp), built with the sanitizers by
// tests/test_sanitizers.py.  No device is needed.  Exits non-zero on the
// first failed check.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

#include "validate.hpp"

using namespace modap_host;

static int failures = 0;
#define EXPECT(cond)                                                          \
    do {                                                                      \
        if (!(cond)) {                                                        \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static modap_params good_params() {
    modap_params p{};
    p.lambda = 1.0;
    p.eps = 1e-6;
    p.eps_relative = 1;
    p.step = MODAP_STEP_FIXED;
    p.max_iters = 10;
    return p;
}

static void test_params() {
    const char *msg = nullptr;
    modap_params p = good_params();
    EXPECT(check_params(&p, &msg) == MODAP_OK);
    EXPECT(check_params(nullptr, &msg) == MODAP_E_INVAL && msg);
    const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();
    for (double lam : {0.0, -1.0, nan, inf}) {
        p = good_params();
        p.lambda = lam;
        EXPECT(check_params(&p, &msg) == MODAP_E_INVAL);
    }
    for (double eps : {0.0, -1e-9, nan, inf}) {
        p = good_params();
        p.eps = eps;
        EXPECT(check_params(&p, &msg) == MODAP_E_INVAL);
    }
    p = good_params();
    p.step = 7;
    EXPECT(check_params(&p, &msg) == MODAP_E_INVAL);
    p = good_params();
    p.max_iters = -1;
    EXPECT(check_params(&p, &msg) == MODAP_E_INVAL);
    p = good_params();
    p.profile = -2;
    EXPECT(check_params(&p, &msg) == MODAP_E_INVAL);
    p = good_params();
    p.max_iters = 0;                   // a check of x0 only
    p.step = MODAP_STEP_AVG;
    EXPECT(check_params(&p, &msg) == MODAP_OK);
}

static void test_system() {
    const char *msg = nullptr;
    double A[6] = {1, 2, 3, 4, 5, 6}, b[2] = {1, 1};
    EXPECT(check_system(2, 3, 3, A, b, MODAP_F64, &msg) == MODAP_OK);
    EXPECT(check_system(0, 3, 3, A, b, MODAP_F64, &msg) == MODAP_E_INVAL);
    EXPECT(check_system(2, 0, 3, A, b, MODAP_F64, &msg) == MODAP_E_INVAL);
    EXPECT(check_system(2, 3, 2, A, b, MODAP_F64, &msg) == MODAP_E_INVAL);       // lda < n
    EXPECT(check_system(2, 3, 3, nullptr, b, MODAP_F64, &msg) == MODAP_E_INVAL);
    EXPECT(check_system(2, 3, 3, A, nullptr, MODAP_F64, &msg) == MODAP_E_INVAL);
    EXPECT(check_system(2, 3, 3, A, b, 3, &msg) == MODAP_E_INVAL);              // unknown storage
    EXPECT(padded_length(MODAP_F64, 3) == 4 && padded_length(MODAP_F32, 5) == 8 && padded_length(MODAP_BF16, 9) == 16);
    EXPECT(padded_length(MODAP_BF16, 16) == 16 && padded_length(MODAP_F32, 1) == 4);
    double v[3] = {0.0, -1.0, 1e308};
    EXPECT(all_finite(v, 3));
    v[1] = std::numeric_limits<double>::infinity();
    EXPECT(!all_finite(v, 3) && all_finite(v, 1));
    EXPECT(all_finite(v, 0));
}

static void test_rows() {
    const char *msg = nullptr;
    const int64_t m = 10, n = 3;
    int64_t rows[4] = {0, 9, 4, 5};
    double nb[4] = {1, 2, 3, 4};
    std::vector<double> nr(4 * n, 1.0);
    EXPECT(check_rows(4, rows, nr.data(), nb, m, &msg) == MODAP_OK);
    EXPECT(check_rows(0, nullptr, nullptr, nullptr, m, &msg) == MODAP_OK);
    EXPECT(check_rows(-1, rows, nr.data(), nb, m, &msg) == MODAP_E_INVAL);
    EXPECT(check_rows(11, rows, nr.data(), nb, m, &msg) == MODAP_E_INVAL);
    EXPECT(check_rows(2, nullptr, nr.data(), nb, m, &msg) == MODAP_E_INVAL);
    int64_t dup[3] = {2, 7, 2};
    EXPECT(check_rows(3, dup, nr.data(), nb, m, &msg) == MODAP_E_INVAL && std::strstr(msg, "distinct"));
    int64_t out[2] = {3, 10};
    EXPECT(check_rows(2, out, nr.data(), nb, m, &msg) == MODAP_E_INVAL && std::strstr(msg, "range"));
    int64_t neg[1] = {-1};
    EXPECT(check_rows(1, neg, nr.data(), nb, m, &msg) == MODAP_E_INVAL);
    double badb[2] = {1, std::numeric_limits<double>::quiet_NaN()};
    EXPECT(check_rows(2, rows, nr.data(), badb, m, &msg) == MODAP_E_INVAL);
    // row contents, in each storage type
    EXPECT(check_new_rows(MODAP_F64, nr.data(), 4, n, &msg) == MODAP_OK);
    nr[n + 1] = std::numeric_limits<double>::infinity();
    EXPECT(check_new_rows(MODAP_F64, nr.data(), 4, n, &msg) == MODAP_E_ZERO_ROW);
    std::vector<double> z(2 * n, 0.0);
    z[0] = 1.0;
    EXPECT(check_new_rows(MODAP_F64, z.data(), 2, n, &msg) == MODAP_E_ZERO_ROW && std::strstr(msg, "zero"));
    std::vector<float> f(2 * n, 0.5f);
    EXPECT(check_new_rows(MODAP_F32, f.data(), 2, n, &msg) == MODAP_OK);
    f[5] = std::numeric_limits<float>::quiet_NaN();
    EXPECT(check_new_rows(MODAP_F32, f.data(), 2, n, &msg) == MODAP_E_ZERO_ROW);
    // bfloat16 bit patterns: 0x3f80 = 1.0, 0x0000 = 0, 0x7f80 = +inf, 0x7fc0 = NaN
    uint16_t h[6] = {0x3f80, 0, 0, 0, 0, 0};
    EXPECT(check_new_rows(MODAP_BF16, h, 1, n, &msg) == MODAP_OK);
    EXPECT(check_new_rows(MODAP_BF16, h, 2, n, &msg) == MODAP_E_ZERO_ROW);
    h[3] = 0x7f80;
    EXPECT(check_new_rows(MODAP_BF16, h, 2, n, &msg) == MODAP_E_ZERO_ROW);
    h[3] = 0x0001;                     // the smallest BF16 subnormal, 2^-133: its square 2^-266 is still > 0 in FP64
    EXPECT(check_new_rows(MODAP_BF16, h, 2, n, &msg) == MODAP_OK);
}

static void test_drift() {
    const char *msg = nullptr;
    const int64_t n = 3, ldv = 4;
    std::vector<double> V(5 * ldv, 0.25);
    EXPECT(check_drift(5, V.data(), ldv, n, true, &msg) == MODAP_OK);
    EXPECT(check_drift(0, nullptr, 0, n, true, &msg) == MODAP_OK);
    EXPECT(check_drift(-1, V.data(), ldv, n, true, &msg) == MODAP_E_INVAL);
    EXPECT(check_drift(5, V.data(), 2, n, true, &msg) == MODAP_E_INVAL);
    V[3] = std::numeric_limits<double>::quiet_NaN();     // padding column: never read
    EXPECT(check_drift(5, V.data(), ldv, n, true, &msg) == MODAP_OK);
    V[4 * ldv + 2] = std::numeric_limits<double>::infinity();
    EXPECT(check_drift(5, V.data(), ldv, n, true, &msg) == MODAP_E_INVAL);
    EXPECT(check_drift(5, V.data(), ldv, n, false, &msg) == MODAP_OK);   // device data: checked on the device
}

static void test_footprint_and_admission() {
    // the footprint holds at least A and grows with every size
    for (int dt : {MODAP_F64, MODAP_F32, MODAP_BF16}) {
        const double a = request_footprint(dt, 4000, 1000, 0);
        EXPECT(a >= 4000.0 * 1000.0 * (double)storage_bytes(dt));
        EXPECT(request_footprint(dt, 4001, 1000, 0) > a);
        EXPECT(request_footprint(dt, 4000, 1001, 0) >= a);
        EXPECT(request_footprint(dt, 4000, 1000, 3) > a);
        EXPECT(std::isfinite(request_footprint(dt, 1LL << 20, 1LL << 15, 100)));
    }
    EXPECT(request_footprint(MODAP_BF16, 100, 100, 0) < request_footprint(MODAP_F32, 100, 100, 0));
    // admission in arrival order within the budget and the live cap
    EXPECT(admissible(0.0, 10.0, 10.0, 0, 0));
    EXPECT(!admissible(0.5, 10.0, 10.0, 0, 0));
    EXPECT(!admissible(0.0, 1.0, 10.0, 3, 3));
    EXPECT(admissible(0.0, 1.0, 10.0, 2, 3));
    // a simulated queue: memory in use never exceeds the budget, every request
    // is admitted in order once enough has been released
    const double budget = 100.0;
    std::vector<double> fp = {40, 30, 50, 20, 90, 10, 100, 5};
    double used = 0.0;
    int64_t live = 0;
    size_t head = 0;
    std::vector<size_t> admitted_at;
    std::vector<double> live_fp;
    for (int round = 0; round < 100 && head < fp.size(); ++round) {
        while (head < fp.size() && admissible(used, fp[head], budget, live, 0)) {
            used += fp[head];
            live_fp.push_back(fp[head]);
            ++live;
            admitted_at.push_back(head++);
        }
        EXPECT(used <= budget);
        if (!live_fp.empty()) {        // the oldest live request finishes
            used -= live_fp.front();
            live_fp.erase(live_fp.begin());
            --live;
        }
    }
    EXPECT(head == fp.size());
    for (size_t i = 0; i < admitted_at.size(); ++i) EXPECT(admitted_at[i] == i);
}

static void test_request() {
    const char *msg = nullptr;
    double A[4] = {1, 0, 0, 1}, b[2] = {1, 1}, V[4] = {0, 0, 0, 0};
    EXPECT(check_request(2, 2, A, b, 0, nullptr, 0, &msg) == MODAP_OK);
    EXPECT(check_request(2, 2, A, b, 2, V, 2, &msg) == MODAP_OK);
    EXPECT(check_request(2, 2, A, b, 2, nullptr, 2, &msg) == MODAP_E_INVAL);
    EXPECT(check_request(2, 2, A, b, 2, V, 1, &msg) == MODAP_E_INVAL);
    EXPECT(check_request(2, 2, A, b, -1, V, 2, &msg) == MODAP_E_INVAL);
    EXPECT(check_request(0, 2, A, b, 0, nullptr, 0, &msg) == MODAP_E_INVAL);
    EXPECT(check_request(2, 2, nullptr, b, 0, nullptr, 0, &msg) == MODAP_E_INVAL);
}

int main() {
    test_params();
    test_system();
    test_rows();
    test_drift();
    test_footprint_and_admission();
    test_request();
    if (failures) {
        std::fprintf(stderr, "%d host checks failed\n", failures);
        return 1;
    }
    std::printf("all host checks passed\n");
    return 0;
}
