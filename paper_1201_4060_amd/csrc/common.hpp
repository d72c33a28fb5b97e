// Internal declarations of the bsi library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/bsi.h"

namespace bsi {

// ---------------------------------------------------------------- errors ---

void set_error(const std::string& msg);
void clear_error();

struct Error {
    bsi_status status;
    std::string msg;
};

// Throw-free helper: evaluate a HIP call, on failure record and return.
#define BSI_HIP(call)                                                            \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            ::bsi::set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
            return BSI_E_DEVICE;                                                 \
        }                                                                        \
    } while (0)

#define BSI_CHECK(cond, status, msg)   \
    do {                               \
        if (!(cond)) {                 \
            ::bsi::set_error(msg);     \
            return (status);           \
        }                              \
    } while (0)

#define BSI_TRY(expr)                  \
    do {                               \
        bsi_status s_ = (expr);        \
        if (s_ != BSI_OK) return s_;   \
    } while (0)

// ------------------------------------------------------- small utilities ---

template <typename T>
struct cplx {
    T x, y;
};

inline bool is_2a3b(int n) {
    if (n <= 0) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

inline size_t dtype_size(int dt) { return dt == BSI_F64 ? 8 : (dt == BSI_F32 ? 4 : 2); }

// ------------------------------------------ B-spline matrix constants -------
// M_(N)[r][c] (row r = stencil point, column c = power of t) from the general
// formula of Section 7, evaluated at compile time in integers:
//   (N-1)! M[r][c] = C(N-1, N-c') * sum_{s=r'}^{N} (-1)^(s-r') C(N, s-r') (N-s)^(N-c')
// with 1-based r' = r+1, c' = c+1 and 0^0 = 1.  M^(1) = M D (Section 2).

constexpr long long ipow_ll(long long b, int e) {
    long long r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}
constexpr long long binom_ll(int n, int k) {
    if (k < 0 || k > n) return 0;
    long long r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}
constexpr long long fact_ll(int n) {
    long long r = 1;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}
// (N-1)! * M_(N)[r][c], 0-based
constexpr long long bspline_numer(int N, int r, int c) {
    long long acc = 0;
    for (int s = r + 1; s <= N; ++s) {
        const int d = s - (r + 1);
        acc += ((d & 1) ? -1 : 1) * binom_ll(N, d) * ipow_ll(N - s, N - (c + 1));
    }
    return binom_ll(N - 1, N - (c + 1)) * acc;
}

template <int N>
struct BSpline {
    double M[N][N];
    double M1[N][N];
    constexpr BSpline() : M{}, M1{} {
        for (int r = 0; r < N; ++r)
            for (int c = 0; c < N; ++c) {
                M[r][c] = double(bspline_numer(N, r, c)) / double(fact_ll(N - 1));
                M1[r][c] = (c + 1 < N)
                               ? double((c + 1) * bspline_numer(N, r, c + 1)) / double(fact_ll(N - 1))
                               : 0.0;
            }
    }
};

// Lagrange interpolation through the N nearest grid values (Section 8), whose
// nodes in a cell's local coordinate are j - N/2 + 1 for stencil point j
// (Section 5 rule): row j = monomial coefficients of the j-th Lagrange basis
// polynomial, built at compile time as an integer numerator polynomial over an
// integer denominator (one rounding per coefficient).  M^(1) = M D.
template <int N>
struct LagrangeM {
    double M[N][N];
    double M1[N][N];
    constexpr LagrangeM() : M{}, M1{} {
        for (int j = 0; j < N; ++j) {
            long long poly[N + 1] = {};
            poly[0] = 1;
            long long den = 1;
            int deg = 0;
            for (int k = 0; k < N; ++k) {
                if (k == j) continue;
                const long long node = k - N / 2 + 1;
                for (int i = deg + 1; i > 0; --i) poly[i] = poly[i - 1] - node * poly[i];
                poly[0] = -node * poly[0];
                ++deg;
                den *= (j - k);
            }
            for (int i = 0; i < N; ++i) {
                M[j][i] = double(poly[i]) / double(den);
                M1[j][i] = (i + 1 < N) ? double((i + 1) * poly[i + 1]) / double(den) : 0.0;
            }
        }
    }
};

// Cubic Hermite interpolation (Section 2): the printed matrix for the data
// f = (u(0), u'(0), u(1), u'(1)) of a cell; M^(1) = M D.
struct HermiteM {
    double M[4][4];
    double M1[4][4];
    constexpr HermiteM() : M{{1, 0, -3, 2}, {0, 1, -2, 1}, {0, 0, 3, -2}, {0, 0, -1, 1}}, M1{} {
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) M1[r][c] = (c + 1 < 4) ? (c + 1) * M[r][c + 1] : 0.0;
    }
};

// B_M(s) at an integer s: the t = 0 column of M_(M) holds the integer samples
// of the centred B-spline (row j <-> s = M/2 - 1 - j).
inline double bspline_integer_sample(int M, int s) {
    const int row = M / 2 - 1 - s;
    if (row < 0 || row >= M) return 0.0;
    return double(bspline_numer(M, row, 0)) / double(fact_ll(M - 1));
}

// ---------------------------------------------------------------- objects ---

struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace bsi

struct bsi_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cus = 0;
    size_t lds_per_block = 0;
    std::mutex mu;
    // twiddle tables e^{+2 pi i m / len}, m < len, keyed by (len, is_double)
    std::map<std::pair<int, int>, void*> twiddles;
    // prefilter constant tables c(k), k < n, FP64, keyed by (n, order, variant, L-bits)
    std::map<std::tuple<int, int, int>, double*> ctabs;
    // per-stream scratch, grown on demand
    std::map<hipStream_t, bsi::Workspace> fft_ws;
    std::map<hipStream_t, bsi::Workspace> eval_ws;
    // tuned evaluation configurations keyed by (order, coef, ncomp, density class)
    std::map<std::tuple<int, int, int, int>, bsi_eval_config> tune_table;
    int live_fields = 0;
    // stage timing (hipEvent pairs recorded around kernel launches)
    bool timing = false;
    struct Pending {
        std::string stage;
        hipEvent_t start, stop;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    std::map<std::string, std::pair<double, int64_t>> stage_totals;
};

struct bsi_field {
    bsi_ctx* ctx = nullptr;
    bsi_field_desc desc{};
    int N = 4;
    int C = 1;
    int basis = BSI_BASIS_BSPLINE;
    int cs = 1;            // stored grid points per cell along an axis: 1, or 2 (Hermite: value, derivative)
    int n[3] = {0, 0, 0};
    int gn[3] = {0, 0, 0}; // periodic extent of the stored grid: cs * n
    int P[3] = {0, 0, 0};  // padded extents gn + N - 1 (Hermite: 2n + 2)
    int padlo = 1;         // ghost planes below index 0 (N/2 - 1; Hermite 0)
    int pitch2 = 0;        // elements between consecutive (p0, p1) rows: P2*C rounded up to 16 B
    double L[3] = {0, 0, 0};
    double inv_h[3] = {0, 0, 0};
    void* grid = nullptr;
    size_t grid_bytes = 0;
    unsigned long long* counters = nullptr;  // [0] = non-finite positions
    hipStream_t last_stream = nullptr;
};

namespace bsi {

// While an UntimedScope lives on a host thread, StageTimer records nothing
// (used by the entry point that must not create events or allocate).
bool untimed();
struct UntimedScope {
    UntimedScope();
    ~UntimedScope();
    UntimedScope(const UntimedScope&) = delete;
    UntimedScope& operator=(const UntimedScope&) = delete;
};

// Brackets the kernel launches of one stage with events when timing is on.
class StageTimer {
   public:
    StageTimer(bsi_ctx* ctx, const char* stage, hipStream_t s);
    ~StageTimer();
    StageTimer(const StageTimer&) = delete;
    StageTimer& operator=(const StageTimer&) = delete;

   private:
    bsi_ctx* ctx_;
    const char* stage_;
    hipStream_t s_;
    hipEvent_t start_ = nullptr;
};

hipStream_t pick_stream(bsi_ctx* ctx, void* s);
bsi_status get_workspace(std::map<hipStream_t, Workspace>& m, hipStream_t s, size_t bytes, void** out);
bsi_status get_twiddles(bsi_ctx* ctx, int len, bool dbl, const void** out);
bsi_status get_ctable(bsi_ctx* ctx, int n, int order, int variant, const double** out);

// host-side prefilter constants (symbol.cpp); variant DERIVATIVE_TABLE gives
// the factor 2 pi k'/n of a derivative along the axis (0 at the Nyquist index)
constexpr int DERIVATIVE_TABLE = 100;
void prefilter_table(int n, int order, int variant, double* out);

// launchers
bsi_status prefilter_run(bsi_field* f, const void* uhat, int prec, hipStream_t s);
bsi_status grid_from_dense(bsi_field* f, const double* dense, hipStream_t s);
bsi_status grid_to_dense(const bsi_field* f, double* dense, hipStream_t s);
bsi_status eval_run(bsi_field* f, const double* pos, int64_t P, void* u, void* grad,
                    const bsi_eval_config& cfg, hipStream_t s);
// evaluation with a caller-provided workspace of eval_ws_bytes() bytes; it is
// eval_bin_ws (positions only: binning and work items) then eval_gather_ws
// (the gather from that binning and the field's current grid)
size_t eval_ws_bytes(const bsi_field* f, int64_t P, const bsi_eval_config& cfg);
bsi_status eval_check_config(const bsi_eval_config& cfg);
bsi_status eval_run_ws(bsi_field* f, const double* pos, int64_t P, void* u, void* grad,
                       const bsi_eval_config& cfg, hipStream_t s, void* ws);
bsi_status eval_bin_ws(bsi_field* f, const double* pos, int64_t P, const bsi_eval_config& cfg, hipStream_t s,
                       void* ws);
bsi_status eval_gather_ws(bsi_field* f, const double* pos, int64_t P, void* u, void* grad,
                          const bsi_eval_config& cfg, hipStream_t s, void* ws);
bsi_status lookup_config(bsi_ctx* ctx, const bsi_field* f, int64_t P, bsi_eval_config* out);
bsi_status check_device_ptr_ex(const void* p, const char* what);
bsi_status debug_cells_run(bsi_field* f, const double* pos, int64_t P, int32_t* cell, double* t,
                           hipStream_t s);
// the evaluation's binning alone, results copied to caller buffers
size_t bin_bucket_count(const bsi_field* f, int tile);
// byte offsets of the binning's arrays in its workspace (grouping scratch
// first, 16-byte aligned), and the binning itself
struct BinLayout {
    size_t grp, pos, perm, hist, offs, bytes;
};
BinLayout bin_layout(const bsi_field* f, long P, int tile);
bsi_status bin_run(bsi_field* f, const double* pos, long P, int tile, void* scratch, uint32_t* perm,
                   double* pos_sorted, uint32_t* hist, uint32_t* offs, hipStream_t s);
// u, grad u and the six second derivatives per component (hessian.hip)
bsi_status hessian_run(bsi_field* f, const double* pos, int64_t P, void* u, void* grad, void* hess,
                       hipStream_t s);
// device address of the static evaluation scratch (static_eval.hip), once per device
bsi_status static_scratch_init(int device);
bsi_status debug_bins_run(bsi_field* f, const double* pos, int64_t P, int tile, uint32_t* hist, uint32_t* offs,
                          uint32_t* perm, double* pos_sorted, hipStream_t s);

}  // namespace bsi
