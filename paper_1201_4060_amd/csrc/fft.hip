// Prefilter on the GPU: symbol multiply + one inverse 3D real FFT (Section 7).
//
// Pass A  (axis 0)  reads the caller's half spectrum uhat[c][k0][k1][k2],
//                   multiplies it by c(k0) c(k1) c(k2) in FP64, casts to the
//                   working precision T and does the inverse complex FFT along
//                   k0, writing the work buffer (same layout).
// Pass B  (axis 1)  inverse complex FFT along k1, in place.
// Pass C  (axis 2)  complex-to-real inverse FFT of each k2 line (length n2/2
//                   complex FFT after the standard even/odd twist), cast to the
//                   storage type and written to the ghost-padded, component-
//                   interleaved coefficient grid.
//
// Every line transform is a Stockham autosort FFT held in LDS: each stage has
// every thread load its radix-R butterflies into registers, apply twiddles
// from a table of exp(+2 pi i m / len) (computed on the host in FP64), do the
// radix-R DFT and store to the self-sorted positions.  A workgroup transforms
// W adjacent lines of a strided axis so that each global row access covers W
// consecutive elements.
#include "common.hpp"

// LDS budget (KiB) of one strided-pass workgroup's line block: two blocks per
// CU (160 KB of LDS), so 32 lines of 256 FP32 points or 16 lines of 512
#ifndef BSI_FFT_LDS_KB
#define BSI_FFT_LDS_KB 80
#endif
// The first pass reads the caller's spectrum (FP64 pairs, planes of 2 MB and
// more apart for lines of 512 points and longer): there, blocks of 32 lines
// (one per CU) give 512-byte row segments instead of 256.
#ifndef BSI_FFT_LDS_KB_LONG_FIRST
#define BSI_FFT_LDS_KB_LONG_FIRST 150
#endif
template <int LEN, bool FIRST>
constexpr int strided_lds_kb() {
    return (FIRST && LEN >= 512) ? BSI_FFT_LDS_KB_LONG_FIRST : BSI_FFT_LDS_KB;
}
// LDS budget of the narrow instance (a single leftover column)
#define BSI_FFT_LDS_KB_NARROW 8
// XCD-contiguous block order (k_fft_axis): the first pass with two blocks per CU
template <int LEN, bool FIRST>
constexpr bool fft_remap() {
    return FIRST && strided_lds_kb<LEN, FIRST>() == BSI_FFT_LDS_KB;
}

namespace bsi {

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cmul_i(cplx<T> a) { return {-a.y, a.x}; }  // i * a

// Inverse (sign +) DFT of length R in registers.
template <typename T>
__device__ __forceinline__ void dft2(cplx<T>* v) {
    cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}
template <typename T>
__device__ __forceinline__ void dft3(cplx<T>* v) {
    const T h = T(0.86602540378443864676372317075294);  // sin(2 pi / 3)
    cplx<T> s = cadd(v[1], v[2]);
    cplx<T> d = csub(v[1], v[2]);
    cplx<T> m = {v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y};
    cplx<T> r = {-h * d.y, h * d.x};  // i * h * (v1 - v2)
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}
template <typename T>
__device__ __forceinline__ void dft4(cplx<T>* v) {
    cplx<T> s0 = cadd(v[0], v[2]), s1 = csub(v[0], v[2]);
    cplx<T> s2 = cadd(v[1], v[3]), s3 = cmul_i(csub(v[1], v[3]));
    v[0] = cadd(s0, s2);
    v[2] = csub(s0, s2);
    v[1] = cadd(s1, s3);
    v[3] = csub(s1, s3);
}
template <typename T>
__device__ __forceinline__ void dft8(cplx<T>* v) {
    const T r2 = T(0.70710678118654752440084436210485);
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4(e);
    dft4(o);
    o[1] = {r2 * (o[1].x - o[1].y), r2 * (o[1].x + o[1].y)};    // * e^{+i pi/4}
    o[2] = cmul_i(o[2]);                                         // * e^{+i pi/2}
    o[3] = {-r2 * (o[3].x + o[3].y), r2 * (o[3].x - o[3].y)};   // * e^{+3i pi/4}
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = cadd(e[q], o[q]);
        v[q + 4] = csub(e[q], o[q]);
    }
}
template <typename T, int R>
__device__ __forceinline__ void dft(cplx<T>* v) {
    if constexpr (R == 2) dft2(v);
    else if constexpr (R == 3) dft3(v);
    else if constexpr (R == 4) dft4(v);
    else dft8(v);
}

template <int REM>
struct Radix {
    static constexpr int value = (REM % 3 == 0) ? 3 : (REM % 8 == 0) ? 8 : (REM % 4 == 0) ? 4 : 2;
};

// Stockham stages NS.. of an inverse FFT of length LEN on one LDS line.
// tw[m * TWS] = exp(+2 pi i m / LEN).  All threads of the block must call this
// with the same template arguments (it contains block barriers).
template <typename T, int LEN, int TEAM, int NS, int TWS>
__device__ __forceinline__ void fft_stages(cplx<T>* buf, const cplx<T>* tw, int lane) {
    if constexpr (NS < LEN) {
        constexpr int R = Radix<LEN / NS>::value;
        constexpr int NB = LEN / R;
        constexpr int PER = (NB + TEAM - 1) / TEAM;
        constexpr int TSTEP = LEN / (NS * R);
        cplx<T> v[PER][R];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int j = lane + q * TEAM;
            if (PER * TEAM == NB || j < NB) {
                const int k = j % NS;
#pragma unroll
                for (int r = 0; r < R; ++r) v[q][r] = buf[j + r * NB];
                if constexpr (NS > 1) {
#pragma unroll
                    for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], tw[r * k * TSTEP * TWS]);
                }
                dft<T, R>(v[q]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int j = lane + q * TEAM;
            if (PER * TEAM == NB || j < NB) {
                const int k = j % NS;
                const int base = (j / NS) * NS * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) buf[base + r * NS] = v[q][r];
            }
        }
        __syncthreads();
        fft_stages<T, LEN, TEAM, NS * R, TWS>(buf, tw, lane);
    }
}

// Lines per workgroup for the strided passes, within BSI_FFT_LDS_KB of LDS.
// W lines per workgroup (longer contiguous row segments of the strided axis
// are better for HBM), TEAM threads per line; TEAM divides LEN so that each
// thread moves a fixed line and a fixed set of rows.  The line block plus the
// twiddle table stay within BSI_FFT_LDS_KB.
#ifndef BSI_FFT_WMAX
#define BSI_FFT_WMAX 32
#endif
#ifndef BSI_FFT_THREADS
#define BSI_FFT_THREADS 512
#endif
template <typename T, int LEN, int KB = BSI_FFT_LDS_KB>
struct StridedCfg {
    static constexpr int bytes = int(sizeof(cplx<T>));
    static constexpr int raw = (KB * 1024 - LEN * bytes) / ((LEN + 1) * bytes);
    static constexpr int W = raw >= 32 && BSI_FFT_WMAX >= 32 ? 32
                             : raw >= 16 && BSI_FFT_WMAX >= 16 ? 16
                             : raw >= 8 ? 8 : raw >= 4 ? 4 : 2;
    static constexpr int POW2 = LEN & (-LEN);  // largest power of two dividing LEN
    static constexpr int TEAM = (BSI_FFT_THREADS / W) < POW2 ? (BSI_FFT_THREADS / W) : POW2;
    static constexpr int THREADS = W * TEAM;
};

// Passes A and B.  Element (c, a, other, k2) of the [C][..][..][H] input sits
// at c*sComp + a*sAxis + other*sOther + k2 (output: the same with the
// output strides); the FFT runs along a.
// FIRST: input is the caller's spectrum (InT pairs), multiplied by the FP64
// symbol cAxis[a] * cOther[other] * c2[k2]; otherwise in-place on the work
// buffer (in == out).
// Columns [k2_begin, k2_end) of the half spectrum are transformed.  NARROW:
// an instance with few lines per workgroup, for a last column left over by
// the wide blocks (k2 = n2/2 when n2/2 is a multiple of their width).
template <typename T, typename InT, int LEN, bool FIRST, bool NARROW = false>
__global__ __launch_bounds__(BSI_FFT_THREADS) void k_fft_axis(const InT* in, cplx<T>* out, int k2_begin,
                                                  int k2_end, int gx, int gy,
                                                  long sAxis, long sOther, long sComp, long oAxis, long oOther,
                                                  long oComp, const double* cAxis,
                                                  const double* cOther, const double* c2,
                                                  const cplx<T>* twg, int quarter) {
    using Cfg = StridedCfg<T, LEN, NARROW ? BSI_FFT_LDS_KB_NARROW : strided_lds_kb<LEN, FIRST>()>;
    constexpr int W = Cfg::W;
    constexpr int LP = LEN + 1;
    __shared__ cplx<T> lines[W * LP];
    __shared__ cplx<T> tw[LEN];
    const int tid = threadIdx.x;
    // Block (column block bx, row set `other`, component bz).  Workgroups are
    // dispatched round-robin over the 8 XCDs; in the first pass with two
    // blocks per CU the grid is one-dimensional and each XCD is given one
    // contiguous range of logical blocks instead, so that the column blocks of
    // one row set run on one XCD and the cache lines they share in the
    // caller's (unaligned) rows are L2 hits.  Elsewhere the plain
    // three-dimensional grid measured as fast or faster.
    int bx, other, bz;
    if constexpr (!NARROW && fft_remap<LEN, FIRST>()) {
        const long nblocks = gridDim.x;
        const long q8 = nblocks / 8, r8 = nblocks % 8, x8 = blockIdx.x % 8;
        const long lb = x8 * q8 + (x8 < r8 ? x8 : r8) + blockIdx.x / 8;
        bx = int(lb % gx);
        other = int((lb / gx) % gy);
        bz = int(lb / (long(gx) * gy));
    } else {
        bx = blockIdx.x;
        other = blockIdx.y;
        bz = blockIdx.z;
    }
    const int k2_0 = k2_begin + bx * W;
    const long base = long(bz) * sComp + long(other) * sOther + k2_0;
    const long obase = long(bz) * oComp + long(other) * oOther + k2_0;

    for (int i = tid; i < LEN; i += Cfg::THREADS) tw[i] = twg[i];
    // Thread tid always handles line w = tid % W; it moves PER elements of that
    // line (rows a = q * RSTEP + tid / W), all loads issued before any store.
    constexpr int RSTEP = Cfg::TEAM;
    constexpr int PER = LEN / RSTEP;
    static_assert(LEN % RSTEP == 0, "line length must be a multiple of the row step");
    const int w = tid % W;
    const int a0 = tid / W;
    const bool valid = k2_0 + w < k2_end;
    const long lane_base = base + (valid ? w : 0) + long(a0) * sAxis;
    const long step = long(RSTEP) * sAxis;
    const long olane_base = obase + (valid ? w : 0) + long(a0) * oAxis;
    const long ostep = long(RSTEP) * oAxis;
    cplx<T> v[PER];
    if constexpr (FIRST) {
        const double cw = (valid ? c2[k2_0 + w] : 0.0);
        const double cO = cOther[other];
        double re[PER], im[PER], ca[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const long e = lane_base + q * step;
            re[q] = double(in[2 * e]);
            im[q] = double(in[2 * e + 1]);
            ca[q] = cAxis[q * RSTEP + a0];
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const double m = (ca[q] * cO) * cw;
            const double a = re[q] * m, b = im[q] * m;
            // times i^quarter (the i's of derivative factors; 0 otherwise)
            const double x = quarter == 0 ? a : quarter == 1 ? -b : quarter == 2 ? -a : b;
            const double y = quarter == 0 ? b : quarter == 1 ? a : quarter == 2 ? -b : -a;
            v[q] = {T(x), T(y)};
        }
    } else {
        const cplx<T>* src = reinterpret_cast<const cplx<T>*>(in);
#pragma unroll
        for (int q = 0; q < PER; ++q) v[q] = src[lane_base + q * step];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) lines[w * LP + q * RSTEP + a0] = v[q];
    __syncthreads();
    fft_stages<T, LEN, Cfg::TEAM, 1, 1>(lines + (tid / Cfg::TEAM) * LP, tw, tid % Cfg::TEAM);
#pragma unroll
    for (int q = 0; q < PER; ++q) v[q] = lines[w * LP + q * RSTEP + a0];
    if (valid) {
#pragma unroll
        for (int q = 0; q < PER; ++q) out[olane_base + q * ostep] = v[q];
    }
}

// ---- storage conversions -------------------------------------------------

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    // IEEE binary32 -> bfloat16, round to nearest, ties to even; NaN stays NaN.
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
template <typename O, typename T>
__device__ __forceinline__ O store_cast(T v) {
    if constexpr (sizeof(O) == 2) return f32_to_bf16_rne(float(v));
    else return O(v);
}
template <typename O>
__device__ __forceinline__ double load_widen(O v) {
    if constexpr (sizeof(O) == 2) return double(__uint_as_float(uint32_t(v) << 16));
    else return double(v);
}

// Pass C configuration: TEAM threads per length-M transform, LINES grid rows of
// C components per workgroup.
template <typename T, int M, int C>
struct C2rCfg {
    static constexpr int TEAM = M >= 512 ? 64 : M >= 256 ? 32 : M >= 128 ? 16 : 8;
    static constexpr int LINES0 = 256 / (C * TEAM);
    // keep the LDS rows (plus the 2M twiddles) within about 40 KB
    static constexpr int LBYTES = (40 * 1024 - 2 * M * int(sizeof(cplx<T>))) / (C * (M + 2) * int(sizeof(cplx<T>)));
    static constexpr int LINES1 = LINES0 < LBYTES ? LINES0 : LBYTES;
    static constexpr int LINES = LINES1 < 1 ? 1 : LINES1;
    static constexpr int THREADS = LINES * C * TEAM;
};

// Pass C.  work[c][g0][g1][k2] (k2 <= M, rows of Hp) -> grid[p0][p1][p2][c] with ghost
// planes: padded index p holds grid index (p - padlo) mod n on every axis.
// tw[m] = exp(+2 pi i m / (2M)), m < 2M.
// A Hermite field stores the transformed field at stride st = 2 with offset
// (a0, a1, a2) on every axis (the derivative orders); otherwise st = 1, a = 0.
template <typename T, typename OutT, int M, int C>
__global__ __launch_bounds__(256) void k_c2r(const cplx<T>* __restrict__ work, int Hp, OutT* __restrict__ grid,
                                             int n0, int n1, int P0, int P1, int P2, int pitch2,
                                             int padlo, const cplx<T>* __restrict__ twg, int st, int a0,
                                             int a1, int a2) {
    using Cfg = C2rCfg<T, M, C>;
    constexpr int H = M + 1;
    constexpr int LP = M + 2;
    constexpr int NL = Cfg::LINES * C;  // transforms per block
    __shared__ cplx<T> zb[NL * LP];
    __shared__ cplx<T> tw[2 * M];
    const int tid = threadIdx.x;
    const long nlines = long(n0) * n1;
    const long line0 = long(blockIdx.x) * Cfg::LINES;
    const long compStride = nlines * Hp;

    for (int i = tid; i < 2 * M; i += Cfg::THREADS) tw[i] = twg[i];
    // load every (line, component) row of H complex values; all loads of a
    // thread are issued before its LDS stores
    constexpr int ITER = (NL * H + Cfg::THREADS - 1) / Cfg::THREADS;
    {
        cplx<T> v[ITER];
#pragma unroll
        for (int q = 0; q < ITER; ++q) {
            const int idx = q * Cfg::THREADS + tid;
            const int f = idx / H, k = idx - (idx / H) * H;
            const int l = f / C, c = f - (f / C) * C;
            const bool ok = idx < NL * H && line0 + l < nlines;
            v[q] = work[ok ? long(c) * compStride + (line0 + l) * Hp + k : 0];
        }
#pragma unroll
        for (int q = 0; q < ITER; ++q) {
            const int idx = q * Cfg::THREADS + tid;
            if (idx < NL * H) {
                const int f = idx / H, k = idx - (idx / H) * H;
                zb[f * LP + k] = v[q];
            }
        }
    }
    __syncthreads();
    // even/odd twist: Z[k] = (X[k] + conj X[M-k]) + i e^{2 pi i k/(2M)} (X[k] - conj X[M-k]),
    // with the imaginary parts of X[0] and X[M] dropped (real-FFT semantics).
    for (int idx = tid; idx < NL * (M / 2 + 1); idx += Cfg::THREADS) {
        const int f = idx / (M / 2 + 1), k = idx % (M / 2 + 1);
        cplx<T>* X = zb + f * LP;
        if (k == 0) {
            const T a = X[0].x, b = X[M].x;
            X[0] = {a + b, a - b};
        } else {
            const int kk = M - k;
            const cplx<T> A = X[k], B = X[kk];
            const cplx<T> Bc = {B.x, -B.y}, Ac = {A.x, -A.y};
            const cplx<T> z1 = cadd(cadd(A, Bc), cmul_i(cmul(tw[k], csub(A, Bc))));
            if (k < kk) {
                const cplx<T> z2 = cadd(cadd(B, Ac), cmul_i(cmul(tw[kk], csub(B, Ac))));
                X[kk] = z2;
            }
            X[k] = z1;
        }
    }
    __syncthreads();
    fft_stages<T, M, Cfg::TEAM, 1, 2>(zb + (tid / Cfg::TEAM) * LP, tw, tid % Cfg::TEAM);
    // scatter rows (with periodic ghost copies) to the interleaved grid
    const int rowElems = P2 * C;
    for (int l = 0; l < Cfg::LINES; ++l) {
        const long line = line0 + l;
        if (line >= nlines) break;
        const int g0 = int(line / n1), g1 = int(line % n1);
        // padded rows holding grid row g: st g + a + padlo, and one periodic
        // ghost copy (minus or plus st n) when that falls inside [0, P)
        const int p0a = st * g0 + a0 + padlo;
        const int p0b = (p0a - st * n0 >= 0) ? p0a - st * n0 : ((p0a + st * n0 < P0) ? p0a + st * n0 : -1);
        const int p1a = st * g1 + a1 + padlo;
        const int p1b = (p1a - st * n1 >= 0) ? p1a - st * n1 : ((p1a + st * n1 < P1) ? p1a + st * n1 : -1);
        OutT* r_aa = grid + (long(p0a) * P1 + p1a) * pitch2;
        OutT* r_ab = p1b >= 0 ? grid + (long(p0a) * P1 + p1b) * pitch2 : nullptr;
        OutT* r_ba = p0b >= 0 ? grid + (long(p0b) * P1 + p1a) * pitch2 : nullptr;
        OutT* r_bb = (p0b >= 0 && p1b >= 0) ? grid + (long(p0b) * P1 + p1b) * pitch2 : nullptr;
        for (int e = tid; e < rowElems; e += Cfg::THREADS) {
            const int p2 = e / C, c = e % C;
            int q2 = p2 - padlo - a2;
            if (st == 2) {
                if (q2 & 1) continue;   // another derivative field's entry
                q2 >>= 1;
            }
            int g2 = q2;
            if (g2 < 0) g2 += 2 * M;
            else if (g2 >= 2 * M) g2 -= 2 * M;
            const cplx<T> z = zb[(l * C + c) * LP + (g2 >> 1)];
            const OutT v = store_cast<OutT>((g2 & 1) ? z.y : z.x);
            r_aa[e] = v;
            if (r_ab) r_ab[e] = v;
            if (r_ba) r_ba[e] = v;
            if (r_bb) r_bb[e] = v;
        }
    }
}

// Pass C of a Hermite field pair: from one line X of the half spectrum (the
// axis-0/1 derivative factors already applied) the fields with axis-2
// derivative order 0 and 1 -- Y[k] = i d[k] X[k], d the derivative table of
// axis 2 -- each by the even/odd twist and a length-M FFT, written together:
// doubled grid entry 2 g + a2 (+ the offsets a0, a1 of axes 0 and 1) holds
// field a2 at grid point g, so whole rows are written.  dtab[k] = 2 pi k / n2
// for k < M, 0 at the Nyquist index M.
template <typename T, typename OutT, int M, int C>
__global__ __launch_bounds__(256) void k_c2r_dual(const cplx<T>* __restrict__ work, int Hp,
                                                  OutT* __restrict__ grid, int n0, int n1, int P0, int P1, int P2,
                                                  int pitch2, const cplx<T>* __restrict__ twg,
                                                  const double* __restrict__ dtab, int a0, int a1) {
    using Cfg = C2rCfg<T, M, 2 * C>;
    constexpr int H = M + 1;
    constexpr int LP = M + 2;
    constexpr int NL = Cfg::LINES * C;  // lines of X per block; the Y lines follow
    __shared__ cplx<T> zb[2 * NL * LP];
    __shared__ cplx<T> tw[2 * M];
    const int tid = threadIdx.x;
    const long nlines = long(n0) * n1;
    const long line0 = long(blockIdx.x) * Cfg::LINES;
    const long compStride = nlines * Hp;

    for (int i = tid; i < 2 * M; i += Cfg::THREADS) tw[i] = twg[i];
    constexpr int ITER = (NL * H + Cfg::THREADS - 1) / Cfg::THREADS;
    {
        cplx<T> v[ITER];
#pragma unroll
        for (int q = 0; q < ITER; ++q) {
            const int idx = q * Cfg::THREADS + tid;
            const int f = idx / H, k = idx - (idx / H) * H;
            const int l = f / C, c = f - (f / C) * C;
            const bool ok = idx < NL * H && line0 + l < nlines;
            v[q] = work[ok ? long(c) * compStride + (line0 + l) * Hp + k : 0];
        }
#pragma unroll
        for (int q = 0; q < ITER; ++q) {
            const int idx = q * Cfg::THREADS + tid;
            if (idx < NL * H) {
                const int f = idx / H, k = idx - (idx / H) * H;
                const T d = T(dtab[k]);
                zb[f * LP + k] = v[q];
                zb[(NL + f) * LP + k] = {-d * v[q].y, d * v[q].x};  // i d X
            }
        }
    }
    __syncthreads();
    // even/odd twist of every line (as k_c2r)
    for (int idx = tid; idx < 2 * NL * (M / 2 + 1); idx += Cfg::THREADS) {
        const int f = idx / (M / 2 + 1), k = idx % (M / 2 + 1);
        cplx<T>* X = zb + f * LP;
        if (k == 0) {
            const T a = X[0].x, b = X[M].x;
            X[0] = {a + b, a - b};
        } else {
            const int kk = M - k;
            const cplx<T> A = X[k], B = X[kk];
            const cplx<T> Bc = {B.x, -B.y}, Ac = {A.x, -A.y};
            const cplx<T> z1 = cadd(cadd(A, Bc), cmul_i(cmul(tw[k], csub(A, Bc))));
            if (k < kk) {
                const cplx<T> z2 = cadd(cadd(B, Ac), cmul_i(cmul(tw[kk], csub(B, Ac))));
                X[kk] = z2;
            }
            X[k] = z1;
        }
    }
    __syncthreads();
    fft_stages<T, M, Cfg::TEAM, 1, 2>(zb + (tid / Cfg::TEAM) * LP, tw, tid % Cfg::TEAM);
    // rows of the doubled grid: st = 2 with offsets (a0, a1); both parities of
    // axis 2; one periodic ghost copy per axis where it falls inside [0, P)
    const int rowElems = P2 * C;
    for (int l = 0; l < Cfg::LINES; ++l) {
        const long line = line0 + l;
        if (line >= nlines) break;
        const int g0 = int(line / n1), g1 = int(line % n1);
        const int p0a = 2 * g0 + a0;
        const int p0b = (p0a + 2 * n0 < P0) ? p0a + 2 * n0 : -1;
        const int p1a = 2 * g1 + a1;
        const int p1b = (p1a + 2 * n1 < P1) ? p1a + 2 * n1 : -1;
        OutT* r_aa = grid + (long(p0a) * P1 + p1a) * pitch2;
        OutT* r_ab = p1b >= 0 ? grid + (long(p0a) * P1 + p1b) * pitch2 : nullptr;
        OutT* r_ba = p0b >= 0 ? grid + (long(p0b) * P1 + p1a) * pitch2 : nullptr;
        OutT* r_bb = (p0b >= 0 && p1b >= 0) ? grid + (long(p0b) * P1 + p1b) * pitch2 : nullptr;
        for (int e = tid; e < rowElems; e += Cfg::THREADS) {
            const int p2 = e / C, c = e % C;
            const int a2 = p2 & 1;
            int g2 = p2 >> 1;
            if (g2 >= 2 * M) g2 -= 2 * M;
            const cplx<T> z = zb[((a2 ? NL : 0) + l * C + c) * LP + (g2 >> 1)];
            const OutT v = store_cast<OutT>((g2 & 1) ? z.y : z.x);
            r_aa[e] = v;
            if (r_ab) r_ab[e] = v;
            if (r_ba) r_ba[e] = v;
            if (r_bb) r_bb[e] = v;
        }
    }
}

// Dense FP64 [C][n0][n1][n2] <-> padded interleaved grid.
template <typename O>
__global__ void k_from_dense(const double* __restrict__ dense, O* __restrict__ grid, int C, int n0,
                             int n1, int n2, int P0, int P1, int P2, int pitch2, int padlo) {
    const long total = long(P0) * P1 * P2 * C;
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < total;
         i += long(gridDim.x) * blockDim.x) {
        const int c = int(i % C);
        long r = i / C;
        const int p2 = int(r % P2);
        r /= P2;
        const int p1 = int(r % P1);
        const int p0 = int(r / P1);
        int g0 = p0 - padlo, g1 = p1 - padlo, g2 = p2 - padlo;
        g0 += (g0 < 0) ? n0 : (g0 >= n0 ? -n0 : 0);
        g1 += (g1 < 0) ? n1 : (g1 >= n1 ? -n1 : 0);
        g2 += (g2 < 0) ? n2 : (g2 >= n2 ? -n2 : 0);
        grid[(long(p0) * P1 + p1) * pitch2 + long(p2) * C + c] =
            store_cast<O>(dense[((long(c) * n0 + g0) * n1 + g1) * n2 + g2]);
    }
}
template <typename O>
__global__ void k_to_dense(const O* __restrict__ grid, double* __restrict__ dense, int C, int n0,
                           int n1, int n2, int P1, int pitch2, int padlo) {
    const long total = long(C) * n0 * n1 * n2;
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < total;
         i += long(gridDim.x) * blockDim.x) {
        long r = i;
        const int g2 = int(r % n2);
        r /= n2;
        const int g1 = int(r % n1);
        r /= n1;
        const int g0 = int(r % n0);
        const int c = int(r / n0);
        dense[i] = load_widen<O>(
            grid[(long(g0 + padlo) * P1 + (g1 + padlo)) * pitch2 + long(g2 + padlo) * C + c]);
    }
}

// ------------------------------------------------------------- launchers ---

namespace {

template <typename T, typename InT, bool FIRST>
bsi_status launch_axis(int len, dim3 grid, const InT* in, cplx<T>* out, int H, long sAxis, long sOther,
                       long sComp, long oAxis, long oOther, long oComp, const double* cAxis,
                       const double* cOther, const double* c2,
                       const cplx<T>* tw, hipStream_t s, int* Wout, int quarter = 0) {
// In the first pass, a last block of wide lines holding a single column (k2 =
// n2/2 when n2/2 is a multiple of the width) is replaced by a narrow launch for
// that column (512^3 x3 FP32: 1273 -> 1136 + 52 us; in pass B the narrow
// launch costs what it saves).
#define BSI_AXIS_CASE(L)                                                                           \
    case L: {                                                                                      \
        using Cfg = StridedCfg<T, L, strided_lds_kb<L, FIRST>()>;                                  \
        using CfgN = StridedCfg<T, L, BSI_FFT_LDS_KB_NARROW>;                                      \
        *Wout = Cfg::W;                                                                            \
        const int full = FIRST && H - 1 >= Cfg::W && (H - 1) % Cfg::W == 0 ? H - 1 : H;           \
        const int gx = (full + Cfg::W - 1) / Cfg::W;                                               \
        const dim3 g = fft_remap<L, FIRST>() ? dim3(unsigned(gx) * grid.y * grid.z)              \
                                              : dim3(unsigned(gx), grid.y, grid.z);              \
        hipLaunchKernelGGL((k_fft_axis<T, InT, L, FIRST>), g, dim3(Cfg::THREADS), 0, s, in, out, 0, full, gx, \
                           int(grid.y), sAxis, sOther, sComp, oAxis, oOther, oComp, cAxis, cOther, c2, tw, \
                           quarter);                                                              \
        if (full < H)                                                                              \
            hipLaunchKernelGGL((k_fft_axis<T, InT, L, FIRST, true>), dim3(1u, grid.y, grid.z),     \
                               dim3(CfgN::THREADS), 0, s, in, out, full, H, 1, int(grid.y), sAxis, sOther, \
                               sComp, oAxis, oOther, oComp, cAxis, cOther, c2, tw, quarter);       \
        break;                                                                                     \
    }
    switch (len) {
        BSI_AXIS_CASE(8)
        BSI_AXIS_CASE(12)
        BSI_AXIS_CASE(16)
        BSI_AXIS_CASE(24)
        BSI_AXIS_CASE(32)
        BSI_AXIS_CASE(48)
        BSI_AXIS_CASE(64)
        BSI_AXIS_CASE(96)
        BSI_AXIS_CASE(128)
        BSI_AXIS_CASE(192)
        BSI_AXIS_CASE(256)
        BSI_AXIS_CASE(384)
        BSI_AXIS_CASE(512)
        BSI_AXIS_CASE(768)
        BSI_AXIS_CASE(1024)
        default:
            set_error("unsupported FFT length " + std::to_string(len));
            return BSI_E_UNSUPPORTED;
    }
#undef BSI_AXIS_CASE
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

template <typename T, typename OutT, int C>
bsi_status launch_c2r(int M, const cplx<T>* work, int Hp, OutT* grid, int n0, int n1, int P0, int P1, int P2,
                      int pitch2, int padlo, const cplx<T>* tw, hipStream_t s, int st = 1, int a0 = 0,
                      int a1 = 0, int a2 = 0) {
    const long nlines = long(n0) * n1;
#define BSI_C2R_CASE(MM)                                                                           \
    case MM: {                                                                                     \
        using Cfg = C2rCfg<T, MM, C>;                                                                 \
        const unsigned nb = unsigned((nlines + Cfg::LINES - 1) / Cfg::LINES);                      \
        hipLaunchKernelGGL((k_c2r<T, OutT, MM, C>), dim3(nb), dim3(Cfg::THREADS), 0, s, work, Hp, grid, \
                           n0, n1, P0, P1, P2, pitch2, padlo, tw, st, a0, a1, a2);                \
        break;                                                                                     \
    }
    switch (M) {
        BSI_C2R_CASE(4)
        BSI_C2R_CASE(6)
        BSI_C2R_CASE(8)
        BSI_C2R_CASE(12)
        BSI_C2R_CASE(16)
        BSI_C2R_CASE(24)
        BSI_C2R_CASE(32)
        BSI_C2R_CASE(48)
        BSI_C2R_CASE(64)
        BSI_C2R_CASE(96)
        BSI_C2R_CASE(128)
        BSI_C2R_CASE(192)
        BSI_C2R_CASE(256)
        BSI_C2R_CASE(384)
        BSI_C2R_CASE(512)
        default:
            set_error("unsupported real FFT length " + std::to_string(2 * M));
            return BSI_E_UNSUPPORTED;
    }
#undef BSI_C2R_CASE
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

template <typename T, typename OutT, int C>
bsi_status launch_c2r_dual(int M, const cplx<T>* work, int Hp, OutT* grid, int n0, int n1, int P0, int P1,
                           int P2, int pitch2, const cplx<T>* tw, const double* dtab, int a0, int a1,
                           hipStream_t s) {
    const long nlines = long(n0) * n1;
#define BSI_C2RD_CASE(MM)                                                                          \
    case MM: {                                                                                     \
        using Cfg = C2rCfg<T, MM, 2 * C>;                                                          \
        const unsigned nb = unsigned((nlines + Cfg::LINES - 1) / Cfg::LINES);                      \
        hipLaunchKernelGGL((k_c2r_dual<T, OutT, MM, C>), dim3(nb), dim3(Cfg::THREADS), 0, s, work, Hp, grid, \
                           n0, n1, P0, P1, P2, pitch2, tw, dtab, a0, a1);                          \
        break;                                                                                     \
    }
    switch (M) {
        BSI_C2RD_CASE(4)
        BSI_C2RD_CASE(6)
        BSI_C2RD_CASE(8)
        BSI_C2RD_CASE(12)
        BSI_C2RD_CASE(16)
        BSI_C2RD_CASE(24)
        BSI_C2RD_CASE(32)
        BSI_C2RD_CASE(48)
        BSI_C2RD_CASE(64)
        BSI_C2RD_CASE(96)
        BSI_C2RD_CASE(128)
        BSI_C2RD_CASE(192)
        BSI_C2RD_CASE(256)
        BSI_C2RD_CASE(384)
        BSI_C2RD_CASE(512)
        default:
            set_error("unsupported real FFT length " + std::to_string(2 * M));
            return BSI_E_UNSUPPORTED;
    }
#undef BSI_C2RD_CASE
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

template <typename T, typename InT, typename OutT>
bsi_status prefilter_pass(bsi_field* f, const InT* uhat, OutT* grid, cplx<T>* work, int H, int Hp, long sComp,
                          long wComp, const double* const* ct, const int* a, int st, int quarter,
                          const void* tw0, const void* tw1, const void* tw2, hipStream_t s,
                          const double* dual_tab = nullptr);

template <typename T, typename InT, typename OutT>
bsi_status prefilter_typed(bsi_field* f, const InT* uhat, OutT* grid, hipStream_t s) {
    bsi_ctx* ctx = f->ctx;
    const int n0 = f->n[0], n1 = f->n[1], n2 = f->n[2], C = f->C;
    const int H = n2 / 2 + 1;
    // work rows padded to whole 128-byte lines, so that the W-column row
    // segments of the strided passes do not straddle an extra line
    constexpr int LINE = 128 / int(sizeof(cplx<T>));
    const int Hp = (H + LINE - 1) / LINE * LINE;
    const size_t elems = size_t(C) * n0 * n1 * Hp;
    void* wsp = nullptr;
    BSI_TRY(get_workspace(ctx->fft_ws, s, elems * sizeof(cplx<T>), &wsp));
    cplx<T>* work = static_cast<cplx<T>*>(wsp);
    const void *tw0, *tw1, *tw2;
    const bool dbl = sizeof(T) == 8;
    BSI_TRY(get_twiddles(ctx, n0, dbl, &tw0));
    BSI_TRY(get_twiddles(ctx, n1, dbl, &tw1));
    BSI_TRY(get_twiddles(ctx, n2, dbl, &tw2));
    const long sComp = long(n0) * n1 * H;    // caller's spectrum
    const long wComp = long(n0) * n1 * Hp;   // work buffer
    // one inverse FFT per stored field: the prefiltered (or plain) field, or
    // for Hermite the 8 derivative fields d^(a0+a1+a2) u / ds0^a0 ds1^a1 ds2^a2,
    // where the two fields of each (a0, a1) share the axis-0 and axis-1 passes
    // and one pass C writes both (k_c2r_dual)
    const bool herm = f->basis == BSI_BASIS_HERMITE;
    const int nn[3] = {n0, n1, n2};
    if (!herm) {
        const int a[3] = {0, 0, 0};
        const double* ct[3];
        for (int d = 0; d < 3; ++d) BSI_TRY(get_ctable(ctx, nn[d], f->N, f->desc.prefilter, &ct[d]));
        return prefilter_pass<T, InT, OutT>(f, uhat, grid, work, H, Hp, sComp, wComp, ct, a, 1, 0, tw0, tw1, tw2,
                                            s);
    }
    const double* dtab2 = nullptr;
    BSI_TRY(get_ctable(ctx, n2, f->N, DERIVATIVE_TABLE, &dtab2));
    for (int pr = 0; pr < 4; ++pr) {
        const int a[3] = {(pr >> 1) & 1, pr & 1, 0};
        const double* ct[3];
        for (int d = 0; d < 2; ++d)
            BSI_TRY(get_ctable(ctx, nn[d], f->N, a[d] ? DERIVATIVE_TABLE : BSI_PREFILTER_NONE, &ct[d]));
        BSI_TRY(get_ctable(ctx, n2, f->N, BSI_PREFILTER_NONE, &ct[2]));
        BSI_TRY((prefilter_pass<T, InT, OutT>(f, uhat, grid, work, H, Hp, sComp, wComp, ct, a, 2,
                                              (a[0] + a[1]) & 3, tw0, tw1, tw2, s, dtab2)));
    }
    return BSI_OK;
}

// The three passes of one inverse FFT: symbol tables ct[d] per axis, the
// product times i^quarter, written at stride st with offsets a[] (see k_c2r);
// with dual_tab, pass C writes the Hermite pair of axis-2 orders 0 and 1
// (k_c2r_dual, dual_tab the axis-2 derivative table).
template <typename T, typename InT, typename OutT>
bsi_status prefilter_pass(bsi_field* f, const InT* uhat, OutT* grid, cplx<T>* work, int H, int Hp, long sComp,
                          long wComp, const double* const* ct, const int* a, int st, int quarter,
                          const void* tw0, const void* tw1, const void* tw2, hipStream_t s,
                          const double* dual_tab) {
    bsi_ctx* ctx = f->ctx;
    const int n0 = f->n[0], n1 = f->n[1], n2 = f->n[2], C = f->C;
    const double *c0 = ct[0], *c1 = ct[1], *c2 = ct[2];
    int W = 0;
    // pass A: axis 0 (stride n1*H in, n1*Hp out), other = k1 (stride H in, Hp out)
    {
    StageTimer tm(ctx, "fft_axis0", s);
    BSI_TRY((launch_axis<T, InT, true>(n0, dim3(1, n1, C), uhat, work, H, long(n1) * H, long(H), sComp,
                                       long(n1) * Hp, long(Hp), wComp, c0, c1, c2,
                                       static_cast<const cplx<T>*>(tw0), s, &W, quarter)));
    }
    // pass B: axis 1 (stride Hp), other = k0 (stride n1*Hp), in place
    {
    StageTimer tm(ctx, "fft_axis1", s);
    BSI_TRY((launch_axis<T, T, false>(n1, dim3(1, n0, C), reinterpret_cast<const T*>(work), work, H,
                                      long(Hp), long(n1) * Hp, wComp, long(Hp), long(n1) * Hp, wComp, nullptr,
                                      nullptr, nullptr, static_cast<const cplx<T>*>(tw1), s, &W)));
    }
    // pass C: c2r along axis 2
    const int M = n2 / 2;
    StageTimer tm(ctx, "fft_c2r", s);
    if (dual_tab) {
        const cplx<T>* t2 = static_cast<const cplx<T>*>(tw2);
        if (C == 1)
            return launch_c2r_dual<T, OutT, 1>(M, work, Hp, grid, n0, n1, f->P[0], f->P[1], f->P[2], f->pitch2, t2,
                                               dual_tab, a[0], a[1], s);
        return launch_c2r_dual<T, OutT, 3>(M, work, Hp, grid, n0, n1, f->P[0], f->P[1], f->P[2], f->pitch2, t2,
                                           dual_tab, a[0], a[1], s);
    }
    if (C == 1)
        return launch_c2r<T, OutT, 1>(M, work, Hp, grid, n0, n1, f->P[0], f->P[1], f->P[2], f->pitch2, f->padlo,
                                      static_cast<const cplx<T>*>(tw2), s, st, a[0], a[1], a[2]);
    return launch_c2r<T, OutT, 3>(M, work, Hp, grid, n0, n1, f->P[0], f->P[1], f->P[2], f->pitch2, f->padlo,
                                  static_cast<const cplx<T>*>(tw2), s, st, a[0], a[1], a[2]);
}

}  // namespace

bsi_status prefilter_run(bsi_field* f, const void* uhat, int prec, hipStream_t s) {
    const int coef = f->desc.coef;
    if (coef == BSI_F64) {
        if (prec == BSI_F64)
            return prefilter_typed<double, double, double>(f, static_cast<const double*>(uhat),
                                                           static_cast<double*>(f->grid), s);
        return prefilter_typed<double, float, double>(f, static_cast<const float*>(uhat),
                                                      static_cast<double*>(f->grid), s);
    }
    if (coef == BSI_F32) {
        if (prec == BSI_F64)
            return prefilter_typed<float, double, float>(f, static_cast<const double*>(uhat),
                                                         static_cast<float*>(f->grid), s);
        return prefilter_typed<float, float, float>(f, static_cast<const float*>(uhat),
                                                    static_cast<float*>(f->grid), s);
    }
    if (prec == BSI_F64)
        return prefilter_typed<float, double, uint16_t>(f, static_cast<const double*>(uhat),
                                                        static_cast<uint16_t*>(f->grid), s);
    return prefilter_typed<float, float, uint16_t>(f, static_cast<const float*>(uhat),
                                                   static_cast<uint16_t*>(f->grid), s);
}

bsi_status grid_from_dense(bsi_field* f, const double* dense, hipStream_t s) {
    const long total = long(f->P[0]) * f->P[1] * f->P[2] * f->C;
    const unsigned nb = unsigned(std::min<long>((total + 255) / 256, 65535L * 8));
    if (f->desc.coef == BSI_F64)
        hipLaunchKernelGGL(k_from_dense<double>, dim3(nb), dim3(256), 0, s, dense,
                           static_cast<double*>(f->grid), f->C, f->gn[0], f->gn[1], f->gn[2], f->P[0],
                           f->P[1], f->P[2], f->pitch2, f->padlo);
    else if (f->desc.coef == BSI_F32)
        hipLaunchKernelGGL(k_from_dense<float>, dim3(nb), dim3(256), 0, s, dense,
                           static_cast<float*>(f->grid), f->C, f->gn[0], f->gn[1], f->gn[2], f->P[0],
                           f->P[1], f->P[2], f->pitch2, f->padlo);
    else
        hipLaunchKernelGGL(k_from_dense<uint16_t>, dim3(nb), dim3(256), 0, s, dense,
                           static_cast<uint16_t*>(f->grid), f->C, f->gn[0], f->gn[1], f->gn[2], f->P[0],
                           f->P[1], f->P[2], f->pitch2, f->padlo);
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

bsi_status grid_to_dense(const bsi_field* f, double* dense, hipStream_t s) {
    const long total = long(f->C) * f->gn[0] * f->gn[1] * f->gn[2];
    const unsigned nb = unsigned(std::min<long>((total + 255) / 256, 65535L * 8));
    if (f->desc.coef == BSI_F64)
        hipLaunchKernelGGL(k_to_dense<double>, dim3(nb), dim3(256), 0, s,
                           static_cast<const double*>(f->grid), dense, f->C, f->gn[0], f->gn[1], f->gn[2],
                           f->P[1], f->pitch2, f->padlo);
    else if (f->desc.coef == BSI_F32)
        hipLaunchKernelGGL(k_to_dense<float>, dim3(nb), dim3(256), 0, s,
                           static_cast<const float*>(f->grid), dense, f->C, f->gn[0], f->gn[1], f->gn[2],
                           f->P[1], f->pitch2, f->padlo);
    else
        hipLaunchKernelGGL(k_to_dense<uint16_t>, dim3(nb), dim3(256), 0, s,
                           static_cast<const uint16_t*>(f->grid), dense, f->C, f->gn[0], f->gn[1],
                           f->gn[2], f->P[1], f->pitch2, f->padlo);
    BSI_HIP(hipGetLastError());
    return BSI_OK;
}

}  // namespace bsi
