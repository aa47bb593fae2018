// GPU construction of the adaptive quadtree over the points and their images, and of the
// U/V/W/X interaction lists (Algorithm 1, tree step: one tree over the target points and the
// image sources).
//
// Tree rules (fixed here because the paper leaves them open):
//  * root square [x_lo, x_lo + S] x [-S/2, S/2], x_lo = min x, S = max(max x - x_lo, 2 max y):
//    symmetric about y = 0, so the lower half is the exact mirror of the upper half and an image
//    box is fully described by its upper twin;
//  * 30-bit integer cells, ix = floor((x - x_lo) * 2^30 / S), iy = 2^29 + floor(y * 2^30 / S)
//    (clamped), Morton keys with x in the even bits; points sorted by (key, input index);
//  * the root always splits; a box at level l >= 1 splits iff it holds more than leaf_size points
//    and l < max_level; boxes are numbered by (level, Morton prefix);
//  * two boxes are adjacent iff their closed integer spans meet in x and in y;
//  * for an upper target box b, with c over upper and image boxes:
//      V(b) = { c : same level, not adjacent to b, parent(c) adjacent to parent(b) }
//      U(b) = { leaf c adjacent to b }                                   (b a leaf)
//      W(b) = { c : finer than b, not adjacent to b, parent(c) adjacent to b }  (b a leaf)
//      X(b) = { leaf c coarser than b, not adjacent to b, adjacent to parent(b) }
//    entries 2 * box + image, ascending.
//
// A forest of independent instances (batched plans) is one tree whose keys carry the instance
// index above the Morton bits: each instance has its own root square and quantisation (27-bit
// cells, so that 9 instance bits fit), boxes are numbered by (level, instance, Morton prefix), and
// lists never cross instances.  A single instance uses 30-bit cells and no instance bits.
//
// The GPU build enumerates these sets structurally (colleagues of b and of its ancestors, and a
// depth-first walk down the colleagues' subtrees); a reference build elsewhere tests the
// defining predicates directly, and the two are compared bit for bit.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>

#include "internal.hpp"

namespace fmmhp {

// ---------------------------------------------------------------------------------------------
// Arena
// ---------------------------------------------------------------------------------------------
fmmhp_status Arena::alloc(void **p, size_t nbytes, const char *what) {
    *p = nullptr;
    if (getenv("FMMHP_TEST_FAIL_ALLOC")) {
        long k = atol(getenv("FMMHP_TEST_FAIL_ALLOC"));
        if (k > 0 && (long)ptrs.size() + 1 == k) {
            set_error("allocation of %s (%zu bytes) failed (test hook)", what, nbytes);
            return FMMHP_ENOMEM;
        }
    }
    hipError_t e = hipMalloc(p, nbytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("hipMalloc of %s (%zu bytes) failed: %s", what, nbytes, hipGetErrorString(e));
        return FMMHP_ENOMEM;
    }
    ptrs.push_back(*p);
    bytes += (int64_t)nbytes;
    return FMMHP_OK;
}

void Arena::release() {
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
}

// RAII scratch for build-time temporaries (stream-ordered).
struct Scratch {
    hipStream_t s;
    std::vector<void *> ptrs;
    explicit Scratch(hipStream_t st) : s(st) {}
    ~Scratch() {
        for (void *p : ptrs) (void)hipFreeAsync(p, s);
    }
    template <class T>
    fmmhp_status get(T **p, size_t n, const char *what) {
        void *q = nullptr;
        hipError_t e = hipMallocAsync(&q, (n ? n : 1) * sizeof(T), s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMallocAsync of %s failed: %s", what, hipGetErrorString(e));
            return FMMHP_ENOMEM;
        }
        ptrs.push_back(q);
        *p = (T *)q;
        return FMMHP_OK;
    }
};

static inline unsigned nblocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// ---------------------------------------------------------------------------------------------
// Exclusive scan of int32 (out has n + 1 entries; out[n] = total)
// ---------------------------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;

__global__ __launch_bounds__(kScanThreads) void k_scan_tile(const int32_t *__restrict__ in,
                                                            int32_t *__restrict__ out,
                                                            int32_t *__restrict__ sums, int64_t n) {
    __shared__ int32_t s[kScanThreads];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)t * kScanPer;
    int32_t v[kScanPer];
    int32_t tot = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        tot += v[k];
    }
    s[t] = tot;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int32_t a = (t >= off) ? s[t - off] : 0;
        __syncthreads();
        s[t] += a;
        __syncthreads();
    }
    int32_t run = s[t] - tot;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (t == kScanThreads - 1) sums[blockIdx.x] = s[t];
}

__global__ void k_scan_add(int32_t *__restrict__ out, const int32_t *__restrict__ offs, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += offs[i / kScanTile];
    if (i == 0) out[n] = offs[(n + kScanTile - 1) / kScanTile];
}

__global__ void k_scan_single_total(int32_t *__restrict__ out, const int32_t *__restrict__ sums) {
    out[0] = 0;
    out[1] = sums[0];
}

static fmmhp_status exclusive_scan(const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
    if (n <= 0) {
        // out[0] = 0
        int32_t zero = 0;
        FMMHP_HIP(hipMemcpyAsync(out, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
        FMMHP_HIP(hipStreamSynchronize(s));
        return FMMHP_OK;
    }
    Scratch sc(s);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    int32_t *sums = nullptr, *soffs = nullptr;
    FMMHP_CHECK(sc.get(&sums, nb, "scan sums"));
    FMMHP_CHECK(sc.get(&soffs, nb + 1, "scan offsets"));
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, sums, n);
    FMMHP_HIP(hipGetLastError());
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_single_total, dim3(1), dim3(1), 0, s, soffs, sums);
    } else {
        FMMHP_CHECK(exclusive_scan(sums, soffs, nb, s));
    }
    hipLaunchKernelGGL(k_scan_add, dim3(nblocks(n, 256)), dim3(256), 0, s, out, soffs, n);
    FMMHP_HIP(hipGetLastError());
    return FMMHP_OK;
}

// ---------------------------------------------------------------------------------------------
// Root square, validation, keys
// ---------------------------------------------------------------------------------------------
struct BBox {
    double xmin, xmax, ymax;
    int bad;        // non-finite coordinate, or y <= 0 (a source) or y < 0 (a target-only point)
    int img_bad;    // image arrays not equal to (x, -y)
    int pad;
};

// Points are processed in chunks that never straddle two instances.
struct Chunk {
    int64_t start, end;
    int32_t inst, pad;
};
constexpr int64_t kChunk = 4096;

// Points from src_end on are target-only (no charge): y = 0 is allowed for them.
__global__ __launch_bounds__(256) void k_bbox(const double *__restrict__ x, const double *__restrict__ y,
                                              const double *__restrict__ ix, const double *__restrict__ iy,
                                              int64_t src_end, const Chunk *__restrict__ chunks,
                                              BBox *__restrict__ part) {
    __shared__ double s0[256], s1[256], s2[256];
    __shared__ int s3[256], s4[256];
    const Chunk ch = chunks[blockIdx.x];
    double xmin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
    int bad = 0, ibad = 0;
    for (int64_t i = ch.start + threadIdx.x; i < ch.end; i += 256) {
        const double a = x[i], b = y[i];
        if (!isfinite(a) || !isfinite(b)) bad |= 1;
        else if (!(b > 0.0) && !(i >= src_end && b == 0.0)) bad |= 2;
        xmin = fmin(xmin, a);
        xmax = fmax(xmax, a);
        ymax = fmax(ymax, b);
        if (ix) {
            // bitwise (x, -y)
            const uint64_t ux = __double_as_longlong(a), uix = __double_as_longlong(ix[i]);
            const uint64_t uy = __double_as_longlong(-b), uiy = __double_as_longlong(iy[i]);
            if (ux != uix || uy != uiy) ibad = 1;
        }
    }
    const int t = threadIdx.x;
    s0[t] = xmin; s1[t] = xmax; s2[t] = ymax; s3[t] = bad; s4[t] = ibad;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            s0[t] = fmin(s0[t], s0[t + off]);
            s1[t] = fmax(s1[t], s1[t + off]);
            s2[t] = fmax(s2[t], s2[t + off]);
            s3[t] |= s3[t + off];
            s4[t] |= s4[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        part[blockIdx.x].xmin = s0[0];
        part[blockIdx.x].xmax = s1[0];
        part[blockIdx.x].ymax = s2[0];
        part[blockIdx.x].bad = s3[0];
        part[blockIdx.x].img_bad = s4[0];
    }
}

__host__ __device__ inline uint64_t interleave2(uint64_t ix, uint64_t iy, int bits) {
    uint64_t k = 0;
    for (int b = 0; b < bits; ++b) {
        k |= ((ix >> b) & 1ull) << (2 * b);
        k |= ((iy >> b) & 1ull) << (2 * b + 1);
    }
    return k;
}

__device__ inline uint64_t spread30(uint64_t v) {
    // spread the low 32 bits of v to the even bit positions
    v &= 0xffffffffull;
    v = (v | (v << 16)) & 0x0000ffff0000ffffull;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffull;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

__device__ inline uint64_t compact30(uint64_t v) {
    v &= 0x5555555555555555ull;
    v = (v | (v >> 1)) & 0x3333333333333333ull;
    v = (v | (v >> 2)) & 0x0f0f0f0f0f0f0f0full;
    v = (v | (v >> 4)) & 0x00ff00ff00ff00ffull;
    v = (v | (v >> 8)) & 0x0000ffff0000ffffull;
    v = (v | (v >> 16)) & 0x00000000ffffffffull;
    return v;
}

// key = instance << 2L | Morton(ix, iy); kChunk / 256 blocks of 256 threads per chunk.
__global__ void k_keys(const double *__restrict__ x, const double *__restrict__ y, const Chunk *__restrict__ chunks,
                       const double *__restrict__ xlo, const double *__restrict__ scale, int lb,
                       uint64_t *__restrict__ keys, int32_t *__restrict__ idx) {
    constexpr int kPer = (int)(kChunk / 256);  // blocks per chunk
    const Chunk ch = chunks[blockIdx.x / kPer];
    const int64_t i = ch.start + (int64_t)(blockIdx.x % kPer) * 256 + threadIdx.x;
    if (i >= ch.end) return;
    const int64_t full = 1ll << lb, half = 1ll << (lb - 1);
    // (x - x_lo) * scale: a subtraction then a multiplication, each correctly rounded
    const double fx = floor(__dmul_rn(__dsub_rn(x[i], xlo[ch.inst]), scale[ch.inst]));
    const double fy = floor(__dmul_rn(y[i], scale[ch.inst]));
    const int64_t ix = fx < 0.0 ? 0 : (fx > (double)(full - 1) ? full - 1 : (int64_t)fx);
    const int64_t iu = fy < 0.0 ? 0 : (fy > (double)(half - 1) ? half - 1 : (int64_t)fy);
    keys[i] = ((uint64_t)ch.inst << (2 * lb)) | spread30((uint64_t)ix) | (spread30((uint64_t)(half + iu)) << 1);
    idx[i] = (int32_t)i;
}

// ---------------------------------------------------------------------------------------------
// Stable LSD radix sort of (uint64 key, int32 value), 8-bit digits
// ---------------------------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;

__global__ __launch_bounds__(256) void k_digit_totals(const uint64_t *__restrict__ keys, int64_t n,
                                                      int32_t *__restrict__ tot /* [8][256] */) {
    __shared__ int32_t h[8][256];
    for (int k = threadIdx.x; k < 8 * 256; k += 256) (&h[0][0])[k] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint64_t k = keys[i];
#pragma unroll
        for (int d = 0; d < 8; ++d) atomicAdd(&h[d][(k >> (8 * d)) & 255], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 8 * 256; k += 256) {
        const int32_t v = (&h[0][0])[k];
        if (v) atomicAdd(&tot[k], v);
    }
}

__global__ __launch_bounds__(256) void k_block_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                    int32_t *__restrict__ hist, int nblk) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__global__ __launch_bounds__(256) void k_scatter(const uint64_t *__restrict__ kin, const int32_t *__restrict__ vin,
                                                 uint64_t *__restrict__ kout, int32_t *__restrict__ vout,
                                                 int64_t n, int shift, const int32_t *__restrict__ offs,
                                                 int nblk) {
    __shared__ int32_t base[256];
    __shared__ int32_t wc[4][256];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    base[t] = offs[(int64_t)t * nblk + blockIdx.x];
    const int64_t tile = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        wc[0][t] = 0; wc[1][t] = 0; wc[2][t] = 0; wc[3][t] = 0;
        __syncthreads();
        const int64_t i = tile + r * kSortThreads + t;
        const bool valid = i < n;
        uint64_t key = 0;
        int32_t val = 0;
        int digit = 0;
        if (valid) {
            key = kin[i];
            val = vin[i];
            digit = (int)((key >> shift) & 255);
        }
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int bit = (digit >> b) & 1;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & lanemask_lt(lane));
        if (valid && rank == 0) wc[wave][digit] = __popcll(peers);
        __syncthreads();
        {
            int32_t run = base[t];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int32_t c = wc[w][t];
                wc[w][t] = run;
                run += c;
            }
            base[t] = run;
        }
        __syncthreads();
        if (valid) {
            const int32_t pos = wc[wave][digit] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

static fmmhp_status radix_sort(uint64_t *&keys, int32_t *&vals, uint64_t *keys_alt, int32_t *vals_alt,
                               int64_t n, hipStream_t s) {
    Scratch sc(s);
    int32_t *tot = nullptr;
    FMMHP_CHECK(sc.get(&tot, 8 * 256, "digit totals"));
    FMMHP_HIP(hipMemsetAsync(tot, 0, 8 * 256 * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_digit_totals, dim3(std::min<int64_t>(1024, nblocks(n, 256))), dim3(256), 0, s,
                       keys, n, tot);
    FMMHP_HIP(hipGetLastError());
    std::vector<int32_t> htot(8 * 256);
    FMMHP_HIP(hipMemcpyAsync(htot.data(), tot, htot.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FMMHP_HIP(hipStreamSynchronize(s));
    const int nblk = (int)nblocks(n, kSortTile);
    int32_t *hist = nullptr, *offs = nullptr;
    FMMHP_CHECK(sc.get(&hist, (size_t)256 * nblk, "radix histogram"));
    FMMHP_CHECK(sc.get(&offs, (size_t)256 * nblk + 1, "radix offsets"));
    uint64_t *ka = keys, *kb = keys_alt;
    int32_t *va = vals, *vb = vals_alt;
    for (int d = 0; d < 8; ++d) {
        bool trivial = false;
        for (int b = 0; b < 256; ++b)
            if (htot[d * 256 + b] == n) trivial = true;
        if (trivial) continue;  // every key has the same digit: the pass is the identity
        hipLaunchKernelGGL(k_block_hist, dim3(nblk), dim3(256), 0, s, ka, n, 8 * d, hist, nblk);
        FMMHP_HIP(hipGetLastError());
        FMMHP_CHECK(exclusive_scan(hist, offs, (int64_t)256 * nblk, s));
        hipLaunchKernelGGL(k_scatter, dim3(nblk), dim3(256), 0, s, ka, va, kb, vb, n, 8 * d, offs, nblk);
        FMMHP_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    keys = ka;
    vals = va;
    FMMHP_HIP(hipStreamSynchronize(s));
    return FMMHP_OK;
}

__global__ void k_gather_points(const double *__restrict__ x, const double *__restrict__ y,
                                const int32_t *__restrict__ perm, int64_t n, double *__restrict__ xs,
                                double *__restrict__ ys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t j = perm[i];
    xs[i] = x[j];
    ys[i] = y[j];
}

// ---------------------------------------------------------------------------------------------
// Boxes, level by level
// ---------------------------------------------------------------------------------------------
constexpr int32_t kInactive = -2;   // point's box at the previous level does not split
constexpr int32_t kRoot = -1;

__global__ void k_fill_i32(int32_t *__restrict__ a, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_level_flags(const uint64_t *__restrict__ keys, const int32_t *__restrict__ act, int64_t n,
                              int level, int lb, int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int f = 0;
    if (act[i] != kInactive) {
        if (i == 0 || act[i - 1] != act[i]) {
            f = 1;
        } else {
            const int sh = 2 * (lb - level);
            f = ((keys[i] ^ keys[i - 1]) >> sh) != 0;
        }
    }
    flag[i] = f;
}

__global__ void k_make_boxes(const uint64_t *__restrict__ keys, const int32_t *__restrict__ act,
                             const int32_t *__restrict__ flag, const int32_t *__restrict__ pos, int64_t n,
                             int level, int lb, int base, int32_t *__restrict__ b_level, int32_t *__restrict__ b_bx,
                             int32_t *__restrict__ b_by, int32_t *__restrict__ b_first,
                             int32_t *__restrict__ b_parent, uint64_t *__restrict__ b_prefix,
                             int32_t *__restrict__ b_inst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const int k = base + pos[i];
    const uint64_t pre = keys[i] >> (2 * (lb - level));  // instance << 2 level | Morton prefix
    const uint64_t cell = (1ull << level) - 1;
    b_level[k] = level;
    b_first[k] = (int32_t)i;
    b_parent[k] = act[i] >= 0 ? act[i] : -1;
    b_prefix[k] = pre;
    b_bx[k] = (int32_t)(compact30(pre) & cell);
    b_by[k] = (int32_t)(compact30(pre >> 1) & cell);
    b_inst[k] = (int32_t)(pre >> (2 * level));
}

__global__ void k_box_counts(int base, int nb, int64_t n, int leaf_size, int level, int max_level,
                             const int32_t *__restrict__ b_first, const int32_t *__restrict__ b_parent,
                             int32_t *__restrict__ b_count, int32_t *__restrict__ b_leaf,
                             int32_t *__restrict__ nsplit) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    const int k = base + j;
    const int64_t next = (j + 1 < nb) ? b_first[k + 1] : n;
    const int par = b_parent[k];
    const int64_t pend = par >= 0 ? (int64_t)b_first[par] + b_count[par] : n;
    const int32_t c = (int32_t)((next < pend ? next : pend) - b_first[k]);
    b_count[k] = c;
    const int split = (c > leaf_size) && (level < max_level);
    b_leaf[k] = !split;
    if (split) atomicAdd(nsplit, 1);
}

__global__ void k_update_act(const int32_t *__restrict__ flag, const int32_t *__restrict__ pos, int64_t n,
                             int base, const int32_t *__restrict__ b_leaf, int32_t *__restrict__ act,
                             int32_t *__restrict__ leaf_of) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || act[i] == kInactive) return;
    const int k = base + pos[i] + flag[i] - 1;
    if (b_leaf[k]) {
        leaf_of[i] = k;
        act[i] = kInactive;
    } else {
        act[i] = k;
    }
}

__global__ void k_children(int lo, int hi, const int32_t *__restrict__ b_parent, int32_t *__restrict__ child_first,
                           int32_t *__restrict__ nchild) {
    const int k = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= hi) return;
    const int p = b_parent[k];
    if (p < 0) return;
    if (k == lo || b_parent[k - 1] != p) child_first[p] = k;
    atomicAdd(&nchild[p], 1);
}

// ---------------------------------------------------------------------------------------------
// Interaction lists
// ---------------------------------------------------------------------------------------------
struct TreeView {
    const int32_t *level, *bx, *by, *parent, *leaf, *child_first, *nchild, *inst;
    const uint64_t *prefix;
    const int32_t *lev_start;  // device [32]
    int depth;
    int lb;                    // cell bits per axis
};

// Box reference: (index << 1) | image.  Returns -1 if (l, X, Y) (full-tree coordinates of the
// instance's tree) is empty.
__device__ inline int find_box(const TreeView &t, int inst, int l, int64_t X, int64_t Y) {
    if (l < 1 || l > t.depth) return -1;
    const int64_t side = 1ll << l;
    if (X < 0 || X >= side || Y < 0 || Y >= side) return -1;
    int img = 0;
    if (Y < (side >> 1)) {
        img = 1;
        Y = side - 1 - Y;
    }
    const uint64_t pre = ((uint64_t)inst << (2 * l)) | spread30((uint64_t)X) | (spread30((uint64_t)Y) << 1);
    int lo = t.lev_start[l], hi = t.lev_start[l + 1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (t.prefix[mid] < pre) lo = mid + 1;
        else hi = mid;
    }
    if (lo < t.lev_start[l + 1] && t.prefix[lo] == pre) return (lo << 1) | img;
    return -1;
}

struct Span {
    int64_t x0, x1, y0, y1;
};

__device__ inline Span ref_span(const TreeView &t, int ref) {
    const int k = ref >> 1;
    const int l = t.level[k];
    const int64_t w = 1ll << (t.lb - l);
    int64_t Y = t.by[k];
    if (ref & 1) Y = (1ll << l) - 1 - Y;
    Span s;
    s.x0 = (int64_t)t.bx[k] * w;
    s.x1 = s.x0 + w;
    s.y0 = Y * w;
    s.y1 = s.y0 + w;
    return s;
}

__device__ inline bool adjacent(const Span &a, const Span &b) {
    return a.x0 <= b.x1 && b.x0 <= a.x1 && a.y0 <= b.y1 && b.y0 <= a.y1;
}

constexpr int kStack = 256;

template <bool FILL>
__global__ void k_lists(TreeView t, int nbox, int32_t *__restrict__ cnt /* [4][nbox] */,
                        const int32_t *__restrict__ off0, const int32_t *__restrict__ off1,
                        const int32_t *__restrict__ off2, const int32_t *__restrict__ off3,
                        int32_t *__restrict__ ent0, int32_t *__restrict__ ent1, int32_t *__restrict__ ent2,
                        int32_t *__restrict__ ent3, int32_t *__restrict__ err) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    const int l = t.level[b];
    const int inst = t.inst[b];
    const int64_t bxf = t.bx[b], byf = t.by[b];
    const bool bleaf = t.leaf[b];
    const Span sb = ref_span(t, b << 1);
    int32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    int32_t *e0 = nullptr, *e1 = nullptr, *e2 = nullptr, *e3 = nullptr;
    if (FILL) {
        e0 = ent0 + off0[b];
        e1 = ent1 + off1[b];
        e2 = ent2 + off2[b];
        e3 = ent3 + off3[b];
    }
#define EMIT(list, val)                              \
    do {                                             \
        if (FILL) e##list[c##list] = (val);          \
        ++c##list;                                   \
    } while (0)

    // V: children of the colleagues of parent(b) that are not adjacent to b
    if (l >= 2) {
        const int64_t PX = bxf >> 1, PY = byf >> 1;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int r = find_box(t, inst, l - 1, PX + dx, PY + dy);
                if (r < 0) continue;
                const int k = r >> 1;
                if (t.leaf[k]) continue;
                const int img = r & 1;
                for (int c = t.child_first[k]; c < t.child_first[k] + t.nchild[k]; ++c) {
                    int64_t cy = t.by[c];
                    if (img) cy = (1ll << l) - 1 - cy;
                    const int64_t ddx = (int64_t)t.bx[c] - bxf, ddy = cy - byf;
                    if (ddx < -1 || ddx > 1 || ddy < -1 || ddy > 1) EMIT(1, (c << 1) | img);
                }
            }
    }
    // Coarser leaves: colleagues of ancestors.  U if adjacent to b (b a leaf), X if not adjacent
    // to b but adjacent to parent(b).
    if (l >= 2) {
        Span sp = ref_span(t, t.parent[b] << 1);
        for (int la = 1; la < l; ++la) {
            const int64_t AX = bxf >> (l - la), AY = byf >> (l - la);
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    const int r = find_box(t, inst, la, AX + dx, AY + dy);
                    if (r < 0 || !t.leaf[r >> 1]) continue;
                    const Span sc = ref_span(t, r);
                    if (adjacent(sc, sb)) {
                        if (bleaf) EMIT(0, r);
                    } else if (adjacent(sc, sp)) {
                        EMIT(3, r);
                    }
                }
        }
    }
    // Same level and finer: U and W for a leaf b, by walking down the colleagues' subtrees.
    if (bleaf) {
        int32_t stack[kStack];
        int sp_ = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int r = find_box(t, inst, l, bxf + dx, byf + dy);
                if (r < 0) continue;
                const int k = r >> 1;
                if (t.leaf[k]) {
                    EMIT(0, r);
                } else {
                    for (int c = t.child_first[k] + t.nchild[k] - 1; c >= t.child_first[k]; --c) {
                        if (sp_ < kStack) stack[sp_++] = (c << 1) | (r & 1);
                        else atomicOr(err, 1);
                    }
                }
            }
        while (sp_ > 0) {
            const int r = stack[--sp_];
            const int k = r >> 1;
            const Span sd = ref_span(t, r);
            if (adjacent(sd, sb)) {
                if (t.leaf[k]) {
                    EMIT(0, r);
                } else {
                    for (int c = t.child_first[k] + t.nchild[k] - 1; c >= t.child_first[k]; --c) {
                        if (sp_ < kStack) stack[sp_++] = (c << 1) | (r & 1);
                        else atomicOr(err, 1);
                    }
                }
            } else {
                EMIT(2, r);
            }
        }
    }
#undef EMIT
    if (!FILL) {
        cnt[b] = c0;
        cnt[nbox + b] = c1;
        cnt[2 * nbox + b] = c2;
        cnt[3 * nbox + b] = c3;
    } else {
        // canonical order: ascending entry value
        int32_t *es[4] = {e0, e1, e2, e3};
        const int32_t cs[4] = {c0, c1, c2, c3};
        for (int li = 0; li < 4; ++li) {
            int32_t *e = es[li];
            for (int i = 1; i < cs[li]; ++i) {
                const int32_t v = e[i];
                int j = i - 1;
                while (j >= 0 && e[j] > v) {
                    e[j + 1] = e[j];
                    --j;
                }
                e[j + 1] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Driver
// ---------------------------------------------------------------------------------------------
fmmhp_status build_tree(Arena &A, Tree &T, int n_inst, const int64_t *inst_off, const double *x, const double *y,
                        const double *img_x, const double *img_y, int64_t src_end, int leaf_size, int max_level,
                        hipStream_t s) {
    Scratch sc(s);
    const int64_t n = inst_off[n_inst];
    T.n = n;
    T.n_inst = n_inst;
    T.lbits = n_inst == 1 ? kLBits : kLBitsForest;
    T.inst_off.assign(inst_off, inst_off + n_inst + 1);
    // chunks of at most kChunk points within one instance
    std::vector<Chunk> hch;
    for (int k = 0; k < n_inst; ++k)
        for (int64_t a = inst_off[k]; a < inst_off[k + 1]; a += kChunk)
            hch.push_back(Chunk{a, std::min(inst_off[k + 1], a + kChunk), k, 0});
    const int nch = (int)hch.size();
    Chunk *chunks = nullptr;
    FMMHP_CHECK(sc.get(&chunks, nch, "point chunks"));
    FMMHP_HIP(hipMemcpyAsync(chunks, hch.data(), nch * sizeof(Chunk), hipMemcpyHostToDevice, s));
    // Root squares from device reductions
    BBox *part = nullptr;
    FMMHP_CHECK(sc.get(&part, nch, "bbox partials"));
    hipLaunchKernelGGL(k_bbox, dim3(nch), dim3(256), 0, s, x, y, img_x, img_y, src_end, chunks, part);
    FMMHP_HIP(hipGetLastError());
    std::vector<BBox> hp(nch);
    FMMHP_HIP(hipMemcpyAsync(hp.data(), part, nch * sizeof(BBox), hipMemcpyDeviceToHost, s));
    FMMHP_HIP(hipStreamSynchronize(s));
    std::vector<double> xmin(n_inst, INFINITY), xmax(n_inst, -INFINITY), ymax(n_inst, -INFINITY);
    int bad = 0, img_bad = 0;
    for (int c = 0; c < nch; ++c) {
        const BBox &b = hp[c];
        const int k = hch[c].inst;
        xmin[k] = std::min(xmin[k], b.xmin);
        xmax[k] = std::max(xmax[k], b.xmax);
        ymax[k] = std::max(ymax[k], b.ymax);
        bad |= b.bad;
        img_bad |= b.img_bad;
    }
    if (bad & 1) {
        set_error("a point coordinate is not finite");
        return FMMHP_EINVAL;
    }
    if (bad & 2) {
        set_error("a source has y <= 0 or a target has y < 0: sources lie in the open upper half plane, "
                  "targets in the closed one");
        return FMMHP_EDOMAIN;
    }
    if (img_bad) {
        set_error("image arrays are not the exact mirror (x, -y) of the points");
        return FMMHP_EDOMAIN;
    }
    T.inst_xlo.resize(n_inst);
    T.inst_S.resize(n_inst);
    T.inst_scale.resize(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        double S = xmax[k] - xmin[k];
        if (2.0 * ymax[k] > S) S = 2.0 * ymax[k];
        if (!(S > 0.0)) S = 1.0;
        T.inst_xlo[k] = xmin[k];
        T.inst_S[k] = S;
        T.inst_scale[k] = ldexp(1.0, T.lbits) / S;
    }
    T.x_lo = T.inst_xlo[0];
    T.S = T.inst_S[0];
    T.scale = T.inst_scale[0];
    double *d_xlo = nullptr, *d_scale = nullptr;
    FMMHP_CHECK(sc.get(&d_xlo, n_inst, "instance x_lo"));
    FMMHP_CHECK(sc.get(&d_scale, n_inst, "instance scale"));
    FMMHP_HIP(hipMemcpyAsync(d_xlo, T.inst_xlo.data(), n_inst * sizeof(double), hipMemcpyHostToDevice, s));
    FMMHP_HIP(hipMemcpyAsync(d_scale, T.inst_scale.data(), n_inst * sizeof(double), hipMemcpyHostToDevice, s));

    // keys and sort
    uint64_t *keys = nullptr, *keys2 = nullptr;
    int32_t *idx = nullptr, *idx2 = nullptr;
    FMMHP_CHECK(sc.get(&keys, n, "keys"));
    FMMHP_CHECK(sc.get(&keys2, n, "keys (alt)"));
    FMMHP_CHECK(sc.get(&idx, n, "indices"));
    FMMHP_CHECK(sc.get(&idx2, n, "indices (alt)"));
    hipLaunchKernelGGL(k_keys, dim3((unsigned)(kChunk / 256) * nch), dim3(256), 0, s, x, y, chunks, d_xlo, d_scale,
                       T.lbits, keys, idx);
    FMMHP_HIP(hipGetLastError());
    uint64_t *ks = keys;
    int32_t *vs = idx;
    FMMHP_CHECK(radix_sort(ks, vs, keys2, idx2, n, s));

    FMMHP_CHECK(A.alloc_n(&T.perm, n, "perm"));
    FMMHP_CHECK(A.alloc_n(&T.xs, n, "sorted x"));
    FMMHP_CHECK(A.alloc_n(&T.ys, n, "sorted y"));
    FMMHP_CHECK(A.alloc_n(&T.leaf_of, n, "leaf_of"));
    FMMHP_HIP(hipMemcpyAsync(T.perm, vs, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_gather_points, dim3(nblocks(n, 256)), dim3(256), 0, s, x, y, T.perm, n, T.xs, T.ys);
    FMMHP_HIP(hipGetLastError());

    // Boxes.  A tree over n points has fewer than n * max_level boxes; grow by levels instead:
    // each level has at most n boxes, so allocate per-level and copy into final arrays.
    int32_t *act = nullptr, *flag = nullptr, *pos = nullptr, *nsplit = nullptr;
    FMMHP_CHECK(sc.get(&act, n, "act"));
    FMMHP_CHECK(sc.get(&flag, n, "flags"));
    FMMHP_CHECK(sc.get(&pos, n + 1, "positions"));
    FMMHP_CHECK(sc.get(&nsplit, 1, "split counter"));
    hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(n, 256)), dim3(256), 0, s, act, n, kRoot);
    FMMHP_HIP(hipGetLastError());

    // box arrays grow in chunks: keep a capacity and reallocate (build time only)
    int cap = (int)std::min<int64_t>(std::max<int64_t>(1024, 2 * n / std::max(1, leaf_size) + 64), 0x7fffffff);
    int32_t *b_level = nullptr, *b_bx = nullptr, *b_by = nullptr, *b_first = nullptr, *b_count = nullptr,
            *b_parent = nullptr, *b_leaf = nullptr, *b_inst = nullptr;
    uint64_t *b_prefix = nullptr;
    auto alloc_boxes = [&](int c) -> fmmhp_status {
        FMMHP_CHECK(sc.get(&b_level, c, "box level"));
        FMMHP_CHECK(sc.get(&b_bx, c, "box bx"));
        FMMHP_CHECK(sc.get(&b_by, c, "box by"));
        FMMHP_CHECK(sc.get(&b_first, c, "box first"));
        FMMHP_CHECK(sc.get(&b_count, c, "box count"));
        FMMHP_CHECK(sc.get(&b_parent, c, "box parent"));
        FMMHP_CHECK(sc.get(&b_leaf, c, "box leaf"));
        FMMHP_CHECK(sc.get(&b_prefix, c, "box prefix"));
        FMMHP_CHECK(sc.get(&b_inst, c, "box instance"));
        return FMMHP_OK;
    };
    FMMHP_CHECK(alloc_boxes(cap));
    T.lev_start.assign(2, 0);  // lev_start[0] unused, lev_start[1] = 0
    int total = 0;
    int level = 0;
    for (level = 1; level <= max_level; ++level) {
        hipLaunchKernelGGL(k_level_flags, dim3(nblocks(n, 256)), dim3(256), 0, s, ks, act, n, level, T.lbits, flag);
        FMMHP_HIP(hipGetLastError());
        FMMHP_CHECK(exclusive_scan(flag, pos, n, s));
        int32_t nb = 0;
        FMMHP_HIP(hipMemcpyAsync(&nb, pos + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FMMHP_HIP(hipStreamSynchronize(s));
        if (nb == 0) break;
        if ((int64_t)total + nb > cap) {
            // grow: copy existing arrays
            int ncap = (int)std::min<int64_t>(0x7fffffff, std::max<int64_t>(2ll * cap, (int64_t)total + nb));
            int32_t *o_level = b_level, *o_bx = b_bx, *o_by = b_by, *o_first = b_first, *o_count = b_count,
                    *o_parent = b_parent, *o_leaf = b_leaf, *o_inst = b_inst;
            uint64_t *o_prefix = b_prefix;
            FMMHP_CHECK(alloc_boxes(ncap));
            const size_t b4 = (size_t)total * 4;
            FMMHP_HIP(hipMemcpyAsync(b_level, o_level, b4, hipMemcpyDeviceToDevice, s));
            FMMHP_HIP(hipMemcpyAsync(b_bx, o_bx, b4, hipMemcpyDeviceToDevice, s));
            FMMHP_HIP(hipMemcpyAsync(b_by, o_by, b4, hipMemcpyDeviceToDevice, s));
            FMMHP_HIP(hipMemcpyAsync(b_first, o_first, b4, hipMemcpyDeviceToDevice, s));
            FMMHP_HIP(hipMemcpyAsync(b_count, o_count, b4, hipMemcpyDeviceToDevice, s));
            FMMHP_HIP(hipMemcpyAsync(b_parent, o_parent, b4, hipMemcpyDeviceToDevice, s));
            FMMHP_HIP(hipMemcpyAsync(b_leaf, o_leaf, b4, hipMemcpyDeviceToDevice, s));
            FMMHP_HIP(hipMemcpyAsync(b_inst, o_inst, b4, hipMemcpyDeviceToDevice, s));
            FMMHP_HIP(hipMemcpyAsync(b_prefix, o_prefix, (size_t)total * 8, hipMemcpyDeviceToDevice, s));
            cap = ncap;
        }
        hipLaunchKernelGGL(k_make_boxes, dim3(nblocks(n, 256)), dim3(256), 0, s, ks, act, flag, pos, n, level,
                           T.lbits, total, b_level, b_bx, b_by, b_first, b_parent, b_prefix, b_inst);
        FMMHP_HIP(hipGetLastError());
        FMMHP_HIP(hipMemsetAsync(nsplit, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_box_counts, dim3(nblocks(nb, 256)), dim3(256), 0, s, total, nb, n, leaf_size, level,
                           max_level, b_first, b_parent, b_count, b_leaf, nsplit);
        FMMHP_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_update_act, dim3(nblocks(n, 256)), dim3(256), 0, s, flag, pos, n, total, b_leaf,
                           act, T.leaf_of);
        FMMHP_HIP(hipGetLastError());
        int32_t hsplit = 0;
        FMMHP_HIP(hipMemcpyAsync(&hsplit, nsplit, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FMMHP_HIP(hipStreamSynchronize(s));
        total += nb;
        T.lev_start.push_back(total);
        if (hsplit == 0) {
            ++level;
            break;
        }
    }
    T.depth = (int)T.lev_start.size() - 2;
    T.nbox = total;
    while ((int)T.lev_start.size() < 33) T.lev_start.push_back(total);

    // final box arrays
    const int nbx = T.nbox;
    FMMHP_CHECK(A.alloc_n(&T.level, nbx, "level"));
    FMMHP_CHECK(A.alloc_n(&T.bx, nbx, "bx"));
    FMMHP_CHECK(A.alloc_n(&T.by, nbx, "by"));
    FMMHP_CHECK(A.alloc_n(&T.first, nbx, "first"));
    FMMHP_CHECK(A.alloc_n(&T.count, nbx, "count"));
    FMMHP_CHECK(A.alloc_n(&T.parent, nbx, "parent"));
    FMMHP_CHECK(A.alloc_n(&T.leaf, nbx, "leaf"));
    FMMHP_CHECK(A.alloc_n(&T.child_first, nbx, "child_first"));
    FMMHP_CHECK(A.alloc_n(&T.nchild, nbx, "nchild"));
    FMMHP_CHECK(A.alloc_n(&T.prefix, nbx, "prefix"));
    FMMHP_CHECK(A.alloc_n(&T.inst, nbx, "box instance"));
    const size_t b4 = (size_t)nbx * 4;
    FMMHP_HIP(hipMemcpyAsync(T.level, b_level, b4, hipMemcpyDeviceToDevice, s));
    FMMHP_HIP(hipMemcpyAsync(T.bx, b_bx, b4, hipMemcpyDeviceToDevice, s));
    FMMHP_HIP(hipMemcpyAsync(T.by, b_by, b4, hipMemcpyDeviceToDevice, s));
    FMMHP_HIP(hipMemcpyAsync(T.first, b_first, b4, hipMemcpyDeviceToDevice, s));
    FMMHP_HIP(hipMemcpyAsync(T.count, b_count, b4, hipMemcpyDeviceToDevice, s));
    FMMHP_HIP(hipMemcpyAsync(T.parent, b_parent, b4, hipMemcpyDeviceToDevice, s));
    FMMHP_HIP(hipMemcpyAsync(T.leaf, b_leaf, b4, hipMemcpyDeviceToDevice, s));
    FMMHP_HIP(hipMemcpyAsync(T.prefix, b_prefix, (size_t)nbx * 8, hipMemcpyDeviceToDevice, s));
    FMMHP_HIP(hipMemcpyAsync(T.inst, b_inst, b4, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(nbx, 256)), dim3(256), 0, s, T.child_first, (int64_t)nbx, -1);
    hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(nbx, 256)), dim3(256), 0, s, T.nchild, (int64_t)nbx, 0);
    FMMHP_HIP(hipGetLastError());
    for (int l = 2; l <= T.depth; ++l) {
        const int lo = T.lev_start[l], hi = T.lev_start[l + 1];
        if (hi > lo)
            hipLaunchKernelGGL(k_children, dim3(nblocks(hi - lo, 256)), dim3(256), 0, s, lo, hi, T.parent,
                               T.child_first, T.nchild);
    }
    FMMHP_HIP(hipGetLastError());

    // lists
    int32_t *dlev = nullptr, *cnt = nullptr, *err = nullptr;
    FMMHP_CHECK(sc.get(&dlev, 33, "level starts"));
    FMMHP_HIP(hipMemcpyAsync(dlev, T.lev_start.data(), 33 * sizeof(int32_t), hipMemcpyHostToDevice, s));
    FMMHP_CHECK(sc.get(&cnt, (size_t)4 * nbx, "list counts"));
    FMMHP_CHECK(sc.get(&err, 1, "list error flag"));
    FMMHP_HIP(hipMemsetAsync(err, 0, sizeof(int32_t), s));
    TreeView tv{T.level, T.bx, T.by, T.parent, T.leaf, T.child_first, T.nchild, T.inst, T.prefix, dlev, T.depth,
                T.lbits};
    hipLaunchKernelGGL(k_lists<false>, dim3(nblocks(nbx, 128)), dim3(128), 0, s, tv, nbx, cnt,
                       (const int32_t *)nullptr, (const int32_t *)nullptr, (const int32_t *)nullptr,
                       (const int32_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr,
                       (int32_t *)nullptr, err);
    FMMHP_HIP(hipGetLastError());
    for (int li = 0; li < 4; ++li) {
        FMMHP_CHECK(A.alloc_n(&T.off[li], (size_t)nbx + 1, "list offsets"));
        FMMHP_CHECK(exclusive_scan(cnt + (size_t)li * nbx, T.off[li], nbx, s));
    }
    int32_t tot[4];
    for (int li = 0; li < 4; ++li)
        FMMHP_HIP(hipMemcpyAsync(&tot[li], T.off[li] + nbx, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    int32_t herr = 0;
    FMMHP_HIP(hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FMMHP_HIP(hipStreamSynchronize(s));
    if (herr) {
        set_error("interaction-list walk exceeded its stack of %d boxes", kStack);
        return FMMHP_EUNSUPPORTED;
    }
    for (int li = 0; li < 4; ++li) {
        if (tot[li] < 0) {
            set_error("interaction list %d exceeds 2^31 entries", li);
            return FMMHP_EUNSUPPORTED;
        }
        T.len[li] = tot[li];
        FMMHP_CHECK(A.alloc_n(&T.ent[li], (size_t)tot[li], "list entries"));
    }
    hipLaunchKernelGGL(k_lists<true>, dim3(nblocks(nbx, 128)), dim3(128), 0, s, tv, nbx, cnt, T.off[0], T.off[1],
                       T.off[2], T.off[3], T.ent[0], T.ent[1], T.ent[2], T.ent[3], err);
    FMMHP_HIP(hipGetLastError());
    // number of leaves
    std::vector<int32_t> hleaf(nbx);
    FMMHP_HIP(hipMemcpyAsync(hleaf.data(), T.leaf, b4, hipMemcpyDeviceToHost, s));
    FMMHP_HIP(hipStreamSynchronize(s));
    T.nleaf = 0;
    for (int k = 0; k < nbx; ++k) T.nleaf += hleaf[k] != 0;
    return FMMHP_OK;
}

}  // namespace fmmhp
