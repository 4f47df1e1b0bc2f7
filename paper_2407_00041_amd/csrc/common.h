// Internal definitions shared by the HIP sources of the library (not part of
// the C ABI).  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/wdirac.h"

namespace wd {

// ---------------------------------------------------------------------------
// error state (thread-local message, status codes of the C ABI)
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
// verbosity from the WDIRAC_LOG environment variable (read once): 0 silent, 1 errors, 2 progress
int log_level();
#define WD_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::wd::fail(WDIRAC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// lattice geometry: dims = {nT, nZ, nY, nX}, site = ((t*nZ + z)*nY + y)*nX + x
struct Geom {
    int n[4];       // nT, nZ, nY, nX
    int V;          // volume (< 2^31 / 12 is enforced at create)
    int stride[4];  // site stride of one step in direction mu: nZ*nY*nX, nY*nX, nX, 1
};

Geom make_geom(const int dims[4]);

// ---------------------------------------------------------------------------
// complex arithmetic in the compute type T (float or double)
template <typename T> struct cx {
    T r, i;
};
template <typename T> __device__ __forceinline__ cx<T> mk(T r, T i) { return {r, i}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
// a * b
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
// conj(a) * b
template <typename T> __device__ __forceinline__ cx<T> cjmul(cx<T> a, cx<T> b) {
    return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
// acc + a * b
template <typename T> __device__ __forceinline__ cx<T> cfma(cx<T> acc, cx<T> a, cx<T> b) {
    acc.r = fma(a.r, b.r, acc.r);
    acc.r = fma(-a.i, b.i, acc.r);
    acc.i = fma(a.r, b.i, acc.i);
    acc.i = fma(a.i, b.r, acc.i);
    return acc;
}
// acc + conj(a) * b
template <typename T> __device__ __forceinline__ cx<T> cjfma(cx<T> acc, cx<T> a, cx<T> b) {
    acc.r = fma(a.r, b.r, acc.r);
    acc.r = fma(a.i, b.i, acc.r);
    acc.i = fma(a.r, b.i, acc.i);
    acc.i = fma(-a.i, b.r, acc.i);
    return acc;
}
template <typename T> __device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.i, a.r}; }
template <typename T> __device__ __forceinline__ cx<T> times_mi(cx<T> a) { return {a.i, -a.r}; }

// ---------------------------------------------------------------------------
// storage precisions of the native layouts (see wdirac.h)
enum class Prec : int { F64 = WDIRAC_F64, F32 = WDIRAC_F32, F16S = WDIRAC_F16S };

// bytes of one right-hand side of a native field (16-byte aligned)
inline size_t field_rhs_bytes(int prec, long long V) {
    switch (prec) {
    case WDIRAC_F64: return (size_t)V * 192;
    case WDIRAC_F32: return (size_t)V * 96;
    case WDIRAC_F16S: return ((size_t)V * 52 + 15) / 16 * 16;
    default: return 0;
    }
}

// Operator data (links and clover, internal to the handle) are stored
// site-tiled: entry e of site s at ((s / 64) * ne + e) * 64 + s % 64 with ne
// entries per site, so one site tile's entries are contiguous and a
// wavefront's loads of any entry hit one 64-site run; arrays are sized for V
// rounded up to a multiple of 64.
constexpr int kOpTile = 64;
__host__ __device__ __forceinline__ size_t op_idx(int e, int ne, int s) {
    return ((size_t)(s >> 6) * ne + e) * kOpTile + (s & (kOpTile - 1));
}
inline long long op_sites(long long V) { return (V + kOpTile - 1) / kOpTile * kOpTile; }

// device-resident operator data at one precision
struct OpData {
    // entries per site (site-tiled, op_idx):
    const void *links = nullptr;   // rows = 3: 4 x 9 (F64 double2, F32 float2, F16 half2);
                                   // rows = 2: F64 4 x 6 double2, F32 4 x 3 float4, F16 4 x 3 (4 x half)
    const void *clover = nullptr;  // packed: F64 2 x 18 double2; F32 2 x 9 float4; F16 2 x 9 (4 x half)
                                   // compact: F64 2 x 14 double2; F32 2 x 7 float4; F16 2 x 7 (4 x half)
    int rows = 3;                  // link rows stored (2: the third is conj(row0 x row1))
    int clover_compact = 0;        // 1: compact clover blocks (H, A_01) with the diagonal constant below
    double diag = 0;               // 4 + m0 (compact clover only)
};

// wavefront-level constants
constexpr int kWave = 64;

// Work-group index -> logical tile index, so that the tiles handled by one XCD
// are contiguous along the lattice (the hardware deals work-groups to the 8
// XCDs round-robin, and each XCD has its own L2).
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
    constexpr int kXcd = 8;
    int q = nblocks / kXcd, r = nblocks % kXcd;
    int k = b % kXcd, j = b / kXcd;
    return k * q + (k < r ? k : r) + j;
}

}  // namespace wd

struct dirac_op {
    wd::Geom g;
    double m0 = 0, csw = 0;
    unsigned flags = 0;
    bool clover_from_links = false;
    int device = 0;
    // device buffers (owned)
    void *links64 = nullptr, *clover64 = nullptr;
    void *links32 = nullptr, *clover32 = nullptr;
    void *links16 = nullptr, *clover16 = nullptr;
    double *links_force = nullptr;  // FP64 links of the force kernel, site tiles [V/64][4][9][64] complex
    // inverse site-local term A(x)^{-1} (even-odd flag only): packed clover layout
    void *cinv64 = nullptr, *cinv32 = nullptr, *cinv16 = nullptr;
    int link_rows = 3;
    bool clover_compact = false;
    wd::OpData data(int prec) const {
        wd::OpData d;
        d.rows = link_rows;
        d.clover_compact = clover_compact ? 1 : 0;
        d.diag = 4.0 + m0;
        if (prec == WDIRAC_F64) { d.links = links64; d.clover = clover64; }
        if (prec == WDIRAC_F32) { d.links = links32; d.clover = clover32; }
        if (prec == WDIRAC_F16S) { d.links = links16; d.clover = clover16; }
        return d;
    }
    const void *cinv(int prec) const {
        return prec == WDIRAC_F64 ? cinv64 : prec == WDIRAC_F32 ? cinv32 : prec == WDIRAC_F16S ? cinv16 : nullptr;
    }
};
