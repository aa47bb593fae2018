// Evaluation of phi = A q (Algorithm 2): upward pass, multipole-to-local translation, downward
// pass and leaf evaluation, for the free-space, image and reaction parts of the half-plane Robin
// Green's function.
//
// Representation.  For an upper box b with centre c_b and half side rho (level l, rho = S 2^-l / 2):
//  * multipole  w_n = sum_j q_j (-(z_j - c_b) / rho)^n / n!,  n = 0..p.  It carries the moments of
//    the box's points (mu_n = (-1)^n n! w_n); the mirror image box has moments conj(mu_n).  From it
//    follow the log-kernel multipole (a_0 = mu_0, a_k = -rho^k mu_k / k, textbook) and the paper's
//    reaction multipole of the image box, alpha_n = rho^n (-i)^n conj(mu_n) (eq. (MEcoefficients)).
//  * local      lambda_n = n! rho^n h_n, where the holomorphic local field of the box is
//    H(z) = sum_n h_n (z - c_b)^n.  With a complex impedance a second local G is kept.
//    The far field at a target is  2 Re H(z) (+ a rank-one surface term, below) for a real
//    impedance, and H(z) + conj(G(z)) for a complex one.
//
// Why H and G.  Phi_free + Phi_1 = -(1/2pi) Re u, u(z) = sum q log(z - z_j) - sum q log(z - conj z_j)
// (eqs. (1.2), (reactioncomp1)); Phi_2^+ (eq. (reactioncomp2)) is holomorphic in the target z, and
// Phi_2^-, the same algorithm on x-mirrored coordinates (Algorithm 2), is anti-holomorphic.  So
// phi = [ -u/(4pi) + Phi_2^+ ](z) + conj[ -u/(4pi) + conj(Phi_2^-) ](z) = H + conj(G).  For a real
// impedance and real charges I_0(-X, Y) = conj(I_0(X, Y)) + i exp(-Z (Y + iX)) (the residue the
// lossless contour picks up, eq. (aaa1.5)), hence Phi_2^- = conj(Phi_2^+) + i e^{-Z(y_i + i x_i)} s with
// s = sum_j q_j e^{-Z(y_j - i x_j)}: G = conj-mirror of H, and phi = 2 Re H + i e^{-Z(y_i+ix_i)} s.
//
// Multipole-to-local.  Every translation of this method is a Hankel contraction in these variables:
//   lambda_n += - sum_m T_{n+m} w_m  (+ L w_0 for n = 0),
// with, for an upper source at same-level offset Delta (t = 1 / (2 Delta)),
//   T_j = -(1/4pi) (j-1)! t^j (j >= 1), T_0 = 0,   L = -(1/4pi) log(-2 rho Delta)     (classic M2L)
// and for an image source (applied to conj(w)),
//   T_j = (1/4pi) (j-1)! t^j - j! i^j K_j,  K_j = rho^j I_j(X, Y),  L = (1/4pi) log(-2 rho Delta)
// which is the log M2L of the image box plus the paper's reaction M2L (eq. (truncatedM2Lcoef)):
//   beta_n = sum_m i^-n (n+m)!/(n! m!) I_{n+m}(x_c - x'_c, y_c - y'_c) alpha_m, re-expanded in
//   powers of (z - c_b) (the paper's local uses powers of (c_b - z), eq. (LEformula)).
// G uses conj(rho^j I_j(-X, Y)) in place of K_j.
//
// M2M and L2L (eqs. (metome), (truncatedL2L) and their log-kernel twins) are Toeplitz in these
// variables:  w^P_n = sum_{m<=n} (-eps)^{n-m}/(n-m)! 2^-m w^c_m,
//             lambda^c_m += 2^-m sum_{n>=m} eps^{n-m}/(n-m)! lambda^P_n,  eps = (c_child - c_parent)/rho_parent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <map>
#include <mutex>
#include <cmath>
#include <complex>
#include <thread>

#include "internal.hpp"
#include "special.hpp"

namespace fmmhp {

static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

struct Geo {
    double x_lo, S;
};

// Root square and impedance of each instance (one for a plain plan).
__device__ __forceinline__ Geo geo_of(const InstInfo *ii, int k) { return Geo{ii[k].x_lo, ii[k].S}; }

__device__ __forceinline__ double side_of(const Geo &g, int l) { return ldexp(g.S, -l); }
__device__ __forceinline__ cplx centre_of(const Geo &g, int l, int bx, int by) {
    const double s = side_of(g, l);
    return mk(g.x_lo + (bx + 0.5) * s, -0.5 * g.S + (by + 0.5) * s);
}

// I_0 with a short series when |P| <= 2 (the near field); the general routine otherwise.
__device__ __noinline__ cplx reaction_I0_general(double x, double y, cplx Z) { return reaction_I0(x, y, Z); }

__constant__ EiSeries kEiSeries;

// Ei(P) - gamma - log P = sum_{k=1..K} P^k / (k k!) by Horner, K chosen from |P| so that the first
// omitted term is below 1e-18 of the leading one: K = 12 for |P| <= 1/4, 20 for |P| <= 1, 30 for
// |P| <= 2.
__device__ __forceinline__ cplx ei_series_small(cplx P, double r2) {
    const int K = r2 <= 0.0625 ? 12 : (r2 <= 1.0 ? 20 : 30);
    cplx h = mk(kEiSeries.c[K], 0.0);
    for (int k = K - 1; k >= 1; --k) {
        cplx t = mk(kEiSeries.c[k], 0.0);
        cfma(t, h, P);
        h = t;
    }
    return h * P;
}

__device__ __forceinline__ cplx reaction_I0_near(double x, double y, cplx Z) {
    const cplx P = Z * mk(y, -x);
    const double r2 = abs2(P);
    if (r2 > 4.0) return reaction_I0_general(x, y, Z);
    const cplx ei = mk(kEulerGamma, 0.0) + clog_(P) + ei_series_small(P, r2);
    const cplx e = cexp_(-P);
    return kInv2Pi * (e * mk(-ei.re, kPi - ei.im));
}

__global__ void k_pack_xy(const double *__restrict__ xs, const double *__restrict__ ys, int64_t n,
                          double2 *__restrict__ xy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) xy[i] = make_double2(xs[i], ys[i]);
}

// ---------------------------------------------------------------------------------------------
// Charges into sorted order
// ---------------------------------------------------------------------------------------------
// U entry (box << 1 | image) -> (first point, count | image << 31) of the box
__global__ void k_u2(int64_t m, const int32_t *__restrict__ uent, const int32_t *__restrict__ first,
                     const int32_t *__restrict__ count, int2 *__restrict__ u2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int code = uent[i], c = code >> 1;
    u2[i] = make_int2(first[c], (int)((unsigned)count[c] | ((unsigned)(code & 1) << 31)));
}

// ---------------------------------------------------------------------------------------------
// nv charge vectors [nv][n] (caller order) -> qs[i * nv + v] (sorted, vectors interleaved)
__global__ void k_gather_q(const double *__restrict__ q, const int32_t *__restrict__ perm, int64_t n, int nv,
                           double *__restrict__ qs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i];
    for (int v = 0; v < nv; ++v) qs[i * nv + v] = q[(int64_t)v * n + o];
}

// ---------------------------------------------------------------------------------------------
// P2M: leaves.  kP2MSplit consecutive lanes share a leaf, each summing every kP2MSplit-th point;
// a butterfly over the lanes combines the partial sums (the same value, bitwise, in every lane).
// ---------------------------------------------------------------------------------------------
constexpr int kP2MSplit = 4;

//
// Dipole sources (DIP: density mu_j, normal n_j, potential mu_j n_j . grad_{r_j} G): the expansions
// of this method are real-linear in the per-source terms q_j f_n(z_j), f_n(z) = (-(z - c)/rho)^n/n!,
// and f_n is holomorphic, so n_j . grad f_n = nu_j f_n' with nu_j = n_x + i n_y; the multipole of a
// dipole is w_n = mu_j nu_j (-1/rho) f_{n-1}(z_j) (w_0 = 0), and every translation is unchanged.
template <int PB, bool DIP>
__global__ __launch_bounds__(256) void k_p2m(const InstInfo *__restrict__ ii, const int32_t *__restrict__ inst,
                                             const int32_t *__restrict__ leaves, int nleaf, int nbox, int nv,
                                             const int32_t *__restrict__ level, const int32_t *__restrict__ bx,
                                             const int32_t *__restrict__ by, const int32_t *__restrict__ first,
                                             const int32_t *__restrict__ count, const double *__restrict__ xs,
                                             const double *__restrict__ ys, const double *__restrict__ qs,
                                             const double2 *__restrict__ nrm, cplx *__restrict__ W) {
    __builtin_amdgcn_s_setprio(3);  // upward pass: the critical path
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = gt / kP2MSplit, part = gt % kP2MSplit;
    const bool ok = t < nleaf;  // no early exit: every lane of a leaf group takes part in the butterfly
    const int v = blockIdx.y;   // charge vector
    W += (int64_t)v * (PB + 1) * nbox;
    const int b = ok ? leaves[t] : 0;
    cplx w[PB + 1];
#pragma unroll
    for (int n = 0; n <= PB; ++n) w[n] = mk(0.0, 0.0);
    if (ok) {
        const int l = level[b];
        const Geo g = geo_of(ii, inst[b]);
        const cplx c = centre_of(g, l, bx[b], by[b]);
        const double irho = 2.0 / side_of(g, l);
        const int f = first[b], e = f + count[b];
        for (int j = f + part; j < e; j += kP2MSplit) {
            const cplx mz = mk((c.re - xs[j]) * irho, (c.im - ys[j]) * irho);  // -(z_j - c) / rho
            if (DIP) {
                const double2 nj = nrm[j];
                cplx term = (-irho * qs[(int64_t)j * nv + v]) * mk(nj.x, nj.y);  // mu nu (-1/rho) f_0
#pragma unroll
                for (int n = 1; n <= PB; ++n) {
                    w[n] += term;
                    term = term * mz * (1.0 / n);
                }
            } else {
                cplx term = mk(qs[(int64_t)j * nv + v], 0.0);
#pragma unroll
                for (int n = 0; n <= PB; ++n) {
                    w[n] += term;
                    term = term * mz * (1.0 / (n + 1));
                }
            }
        }
    }
#pragma unroll
    for (int n = 0; n <= PB; ++n)
        for (int off = 1; off < kP2MSplit; off <<= 1) {
            w[n].re += __shfl_xor(w[n].re, off);
            w[n].im += __shfl_xor(w[n].im, off);
        }
    if (ok) {
#pragma unroll
        for (int n = 0; n <= PB; ++n)
            if (n % kP2MSplit == part) W[(int64_t)n * nbox + b] = w[n];
    }
}

// ---------------------------------------------------------------------------------------------
// M2M.  (P2M and M2M raise their waves' issue priority: the upward pass is the critical path of
// an evaluation while the near field and the deep-level M2L run beside it on other streams.)
// A block takes kM2MParents consecutive boxes of a level; their children are a contiguous
// range of the next level, whose multipoles are staged in LDS once.  Thread (parent, n) then forms
// w^P_n = sum_children sum_{m<=n} (-eps)^{n-m}/(n-m)! 2^-m w^c_m.
// k_m2m runs one level; k_m2m_sub runs every level below a cut level, one block per subtree
// rooted at the cut (a subtree's boxes of one level are a contiguous range), deepest level first.
// ---------------------------------------------------------------------------------------------
constexpr int kM2MParents = 16;

// Coefficient n of a parent's multipole from its children's staged multipoles: children
// c0 .. c0 + nc - 1, child c's coefficient m (scaled by 2^-m) at sw[m * ld + c], its position in
// the parent quad[c].  Callers put n in the fastest-varying thread index: the lanes of a wave then
// read a few children (broadcast) and consecutive shift coefficients (no LDS bank conflicts).
template <int PB>
__device__ __forceinline__ cplx m2m_coef(const cplx *sE, const int *quad, const cplx *sw, int ld, int c0, int nc,
                                         int n) {
    cplx out = mk(0.0, 0.0);
    for (int c = c0; c < c0 + nc; ++c) {
        const cplx *Eq = sE + quad[c] * (PB + 1) + n;
#pragma unroll 4
        for (int m = 0; m <= n; ++m) cfma(out, Eq[-m], sw[m * ld + c]);
    }
    return out;
}

// Coefficient m of a child's local from its parent's staged local (coefficient n at sl[n * ld]):
// sum_{n>=m} Eq[n] sl[n * ld], Eq the child's shift row offset by -m.
template <int PB>
__device__ __forceinline__ cplx l2l_coef(const cplx *Eq, const cplx *sl, int ld, int m) {
    cplx s = mk(0.0, 0.0);
#pragma unroll 4
    for (int n = m; n <= PB; ++n) cfma(s, Eq[n], sl[n * ld]);
    return s;
}

template <int PB>
struct M2MShared {
    cplx sE[4 * (PB + 1)];
    int2 par[kM2MParents];                // (first staged child, number of children) per parent
    int quad[4 * kM2MParents];            // position of each staged child in its parent
    int range[2];
};

// Parents [p0, p1) of one level (p1 - p0 <= kM2MParents); called by every thread of the block
// with block-uniform bounds.  The children's multipoles, scaled by 2^-m, are staged in the LDS
// rows sw (row length ld >= 4 kM2MParents: coefficient m of staged child k at sw[m * ld + k]).
// Two dependent memory round trips (the parents' child ranges, then the children's multipoles and
// positions); ends with a barrier, so the multipoles written are visible to the whole block.
template <int PB>
__device__ __forceinline__ void m2m_parents(M2MShared<PB> &sh, cplx *sw, int ld, int p0, int p1, int nbox,
                            const int32_t *__restrict__ leaf,
                            const int32_t *__restrict__ child_first, const int32_t *__restrict__ nchild,
                            const int32_t *__restrict__ bx, const int32_t *__restrict__ by,
                            cplx *__restrict__ W) {
    static_assert(kM2MParents <= 64, "the child range is reduced over one wave");
    if (threadIdx.x < 64) {  // child range of the non-leaf parents, reduced over the first wave
        const int p = p0 + (int)threadIdx.x;
        int cf = 0, ncp = 0;
        if (p < p1 && !leaf[p]) {
            cf = child_first[p];
            ncp = nchild[p];
        }
        int clo = ncp > 0 ? cf : 0x7fffffff, chi = ncp > 0 ? cf + ncp : -1;
        for (int off = 32; off > 0; off >>= 1) {
            clo = min(clo, __shfl_xor(clo, off));
            chi = max(chi, __shfl_xor(chi, off));
        }
        if (threadIdx.x < kM2MParents) sh.par[threadIdx.x] = make_int2(cf - clo, ncp);
        if (threadIdx.x == 0) {
            sh.range[0] = clo;
            sh.range[1] = chi;
        }
    }
    __syncthreads();
    const int clo = sh.range[0], nc = sh.range[1] - sh.range[0];
    for (int idx = threadIdx.x; idx < (PB + 1) * nc; idx += blockDim.x) {
        const int m = idx / nc, k = idx - m * nc;
        sw[m * ld + k] = W[(int64_t)m * nbox + clo + k] * ldexp(1.0, -m);
    }
    for (int k = threadIdx.x; k < nc; k += blockDim.x) sh.quad[k] = (bx[clo + k] & 1) | ((by[clo + k] & 1) << 1);
    __syncthreads();
    for (int idx = threadIdx.x; idx < (p1 - p0) * (PB + 1); idx += blockDim.x) {
        const int pi = idx / (PB + 1), n = idx - pi * (PB + 1);
        const int2 pr = sh.par[pi];
        if (pr.y > 0) W[(int64_t)n * nbox + p0 + pi] = m2m_coef<PB>(sh.sE, sh.quad, sw, ld, pr.x, pr.y, n);
    }
    __syncthreads();
}

template <int PB>
__global__ __launch_bounds__(256) void k_m2m(int lo, int nb, int nbox, const int32_t *__restrict__ leaf,
                                             const int32_t *__restrict__ child_first,
                                             const int32_t *__restrict__ nchild, const int32_t *__restrict__ bx,
                                             const int32_t *__restrict__ by, const cplx *__restrict__ E,
                                             cplx *__restrict__ W) {
    __builtin_amdgcn_s_setprio(3);  // upward pass: the critical path
    __shared__ M2MShared<PB> sh;
    extern __shared__ cplx dyn_lds[];  // (PB + 1) x 4 kM2MParents
    W += (int64_t)blockIdx.y * (PB + 1) * nbox;  // charge vector
    for (int k = threadIdx.x; k < 4 * (PB + 1); k += blockDim.x) sh.sE[k] = E[k];
    const int p0 = lo + blockIdx.x * kM2MParents;
    m2m_parents<PB>(sh, dyn_lds, 4 * kM2MParents, p0, min(p0 + kM2MParents, lo + nb), nbox, leaf, child_first, nchild,
                    bx, by, W);
}

// Subtree passes.  rng: [n_roots][nlev] box ranges (begin, end) of each subtree at the levels
// cut + k.  The block's dynamic LDS holds ld rows slots (ld >= 4 kM2MParents); a subtree whose
// expansions fit keeps all of them in LDS between levels (one memory round trip to load them,
// then LDS only), a larger one runs the chunked one-level code level after level.
constexpr int kSubMaxLev = 32;
constexpr int kSubMaxSlots = 256;   // resident slots (the host keeps ld within this)

struct SubShared {
    int base[kSubMaxLev + 1];        // first resident slot of each level
    int first[kSubMaxLev];           // first box of each level
    int slot[kSubMaxSlots];          // leaf: -1; else slot of the first child (M2M) / of the parent (L2L)
    int nch[kSubMaxSlots];           // number of children (M2M)
    int quad[kSubMaxSlots];          // position of the box in its parent
};

// Fills ss.base and ss.first from the subtree's ranges; ends with a barrier.
__device__ __forceinline__ void sub_ranges(SubShared &ss, const int2 *__restrict__ R, int nlev) {
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < nlev; ++k) {
            const int2 r = R[k];
            ss.base[k] = tot;
            ss.first[k] = r.x;
            tot += r.y - r.x;
        }
        ss.base[nlev] = tot;
    }
    __syncthreads();
}

// Level of resident slot i.
__device__ __forceinline__ int sub_level_of(const SubShared &ss, int nlev, int i) {
    int k = 0;
    while (k + 1 < nlev && ss.base[k + 1] <= i) ++k;
    return k;
}

// M2M of the parents [c.x, c.y) of one level for each chunk c (at most kM2MParents parents): the
// subtrees too large for LDS, one launch per level, deepest first.
template <int PB>
__global__ __launch_bounds__(256) void k_m2m_chunks(const int2 *__restrict__ chunks, int nbox,
                                                    const int32_t *__restrict__ leaf,
                                                    const int32_t *__restrict__ child_first,
                                                    const int32_t *__restrict__ nchild, const int32_t *__restrict__ bx,
                                                    const int32_t *__restrict__ by, const cplx *__restrict__ E,
                                                    cplx *__restrict__ W) {
    __builtin_amdgcn_s_setprio(3);  // upward pass: the critical path
    __shared__ M2MShared<PB> sh;
    extern __shared__ cplx dyn_lds[];  // (PB + 1) x 4 kM2MParents
    W += (int64_t)blockIdx.y * (PB + 1) * nbox;  // charge vector
    for (int k = threadIdx.x; k < 4 * (PB + 1); k += blockDim.x) sh.sE[k] = E[k];
    const int2 c = chunks[blockIdx.x];
    m2m_parents<PB>(sh, dyn_lds, 4 * kM2MParents, c.x, c.y, nbox, leaf, child_first, nchild, bx, by, W);
}

// skip_big: a subtree whose expansions do not fit the block's LDS rows is left to k_m2m_chunks
// (otherwise the block runs it level by level itself).
template <int PB>
__global__ __launch_bounds__(256) void k_m2m_sub(int nlev, const int2 *__restrict__ rng, int ld, int skip_big, int nbox,
                                                 const int32_t *__restrict__ leaf,
                                                 const int32_t *__restrict__ child_first,
                                                 const int32_t *__restrict__ nchild, const int32_t *__restrict__ bx,
                                                 const int32_t *__restrict__ by, const cplx *__restrict__ E,
                                                 cplx *__restrict__ W) {
    __builtin_amdgcn_s_setprio(3);  // upward pass: the critical path
    __shared__ M2MShared<PB> sh;
    __shared__ SubShared ss;
    extern __shared__ cplx dyn_lds[];  // (PB + 1) x ld: slot i, coefficient m at [m * ld + i]
    cplx *sw = dyn_lds;
    W += (int64_t)blockIdx.y * (PB + 1) * nbox;  // charge vector
    for (int k = threadIdx.x; k < 4 * (PB + 1); k += blockDim.x) sh.sE[k] = E[k];
    const int2 *R = rng + (int64_t)blockIdx.x * nlev;
    sub_ranges(ss, R, nlev);
    const int tot = ss.base[nlev];
    if (tot > ld) {
        if (skip_big) return;
        for (int k = nlev - 2; k >= 0; --k) {
            const int2 r = R[k];
            for (int p0 = r.x; p0 < r.y; p0 += kM2MParents)
                m2m_parents<PB>(sh, sw, ld, p0, min(p0 + kM2MParents, r.y), nbox, leaf, child_first, nchild, bx, by,
                                W);
        }
        return;
    }
    // every box's structure and multipole (the non-leaf ones are recomputed below before use),
    // stored scaled by 2^-m as its parent consumes it
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        const int k = sub_level_of(ss, nlev, i);
        const int b = ss.first[k] + (i - ss.base[k]);
        const int lf = leaf[b];
        ss.slot[i] = lf ? -1 : ss.base[k + 1] + (child_first[b] - ss.first[k + 1]);
        ss.nch[i] = lf ? 0 : nchild[b];
        ss.quad[i] = (bx[b] & 1) | ((by[b] & 1) << 1);
    }
    for (int idx = threadIdx.x; idx < tot * (PB + 1); idx += blockDim.x) {
        const int m = idx / tot, i = idx - m * tot;
        const int k = sub_level_of(ss, nlev, i);
        const int b = ss.first[k] + (i - ss.base[k]);
        sw[m * ld + i] = W[(int64_t)m * nbox + b] * ldexp(1.0, -m);
    }
    __syncthreads();
    for (int k = nlev - 2; k >= 0; --k) {
        const int i0 = ss.base[k], np = ss.base[k + 1] - i0;
        for (int idx = threadIdx.x; idx < np * (PB + 1); idx += blockDim.x) {
            const int ip = idx / (PB + 1), n = idx - ip * (PB + 1), i = i0 + ip;
            const int c0 = ss.slot[i];
            if (c0 < 0) continue;
            const cplx out = m2m_coef<PB>(sh.sE, ss.quad, sw, ld, c0, ss.nch[i], n);
            W[(int64_t)n * nbox + ss.first[k] + (i - i0)] = out;
            sw[n * ld + i] = out * ldexp(1.0, -n);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// M2L over tiles of same-level, same-class target boxes; one wave per (tile, chunk of CH output
// coefficients).  Lanes are target boxes; the operator of an offset slot is the same for every
// lane, so its coefficients are read with scalar loads.  Operator rows are zero-padded to
// m2l_row(PB) entries so that every chunk runs the same branch-free inner loop.
// ---------------------------------------------------------------------------------------------
struct M2LArgs {
    int nbox;
    int tile0;               // first tile of this launch
    const int32_t *tiles, *tile_level, *tile_src_off, *tile_src;
    const int16_t *tile_slot;
    const uint64_t *tile_mask;
    const cplx *Tfree, *Lfree;
    const double *logside;   // [nbox] log(side) of each box
    const cplx *W;           // [nv][PB + 1][nbox]
    cplx *Lam;               // [nv][nloc][PB + 1][nbox]
    int nloc;
};

// One workgroup per tile of up to 64 same-level target boxes (lane = target), kM2LWaves waves;
// wave w owns output coefficients [w CH, w CH + CH).  The tile's distinct V sources have their
// multipoles staged in LDS, kM2LPhase coefficients at a time, and every (target, offset slot)
// pair reads its source from there.  The operator of a slot is the same for all lanes and is
// read with scalar loads.
template <int PB, int CH>
__global__ __launch_bounds__(64 * m2l_waves(PB)) void k_m2l(M2LArgs a) {
    constexpr int NTP = m2l_row(PB);
    constexpr int NPH = (PB + kM2LPhase) / kM2LPhase;
    __shared__ cplx sW[kM2LPhase * kM2LMaxSrc];
    const int tile = blockIdx.x + a.tile0;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n0 = wave * CH;
    const int lane = threadIdx.x & 63;
    const int b = a.tiles[tile * kTile + lane];
    const double ll = b >= 0 ? a.logside[b] * kInv4Pi : 0.0;
    const cplx *W = a.W + (int64_t)blockIdx.y * (PB + 1) * a.nbox;            // charge vector
    cplx *Lam = a.Lam + (int64_t)blockIdx.y * a.nloc * (PB + 1) * a.nbox;
    const int s0 = a.tile_src_off[tile];
    const int ns = a.tile_src_off[tile + 1] - s0;
    const uint64_t mask = a.tile_mask[tile];
    const int16_t *slot = a.tile_slot + (int64_t)tile * kNumSlots * kTile + lane;
    cplx acc[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) acc[k] = mk(0.0, 0.0);
    cplx acc0 = mk(0.0, 0.0);
#pragma unroll
    for (int ph = 0; ph < NPH; ++ph) {
        const int m0 = ph * kM2LPhase;
        const int mc = (PB + 1 - m0) < kM2LPhase ? (PB + 1 - m0) : kM2LPhase;
        __syncthreads();
        for (int idx = threadIdx.x; idx < mc * ns; idx += 64 * m2l_waves(PB)) {
            const int mm = idx / ns, sj = idx - mm * ns;
            sW[idx] = W[(int64_t)(m0 + mm) * a.nbox + a.tile_src[s0 + sj]];
        }
        __syncthreads();
        // the walk over the tile's slots loads the next slot's source index before this slot's
        // arithmetic, so that its memory latency is hidden
        uint64_t rest = mask;
        int o = rest ? __builtin_ctzll(rest) : 0;
        rest &= rest - 1;
        int li = mask ? slot[o * kTile] : -1;
        for (bool go = mask != 0; go;) {
            go = rest != 0;
            const int on = go ? __builtin_ctzll(rest) : o;  // the last slot reloads its own index
            rest &= rest - 1;
            const int lin = slot[on * kTile];
            const int oc = o, lc = li;
            o = on;
            li = lin;
            if (lc < 0) continue;
            const cplx *T = a.Tfree + oc * NTP + n0 + m0;
            const cplx *w = sW + lc;
#pragma unroll
            for (int mm = 0; mm < kM2LPhase; ++mm) {
                if (mm < mc) {
                    const cplx wm = w[mm * ns];
#pragma unroll
                    for (int k = 0; k < CH; ++k) cfma(acc[k], T[k + mm], wm);
                }
            }
            if (ph == 0 && n0 == 0) cfma(acc0, a.Lfree[oc] - mk(ll, 0.0), w[0]);
        }
    }
    if (b < 0) return;
    const int64_t stride = (int64_t)(PB + 1) * a.nbox;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int n = n0 + k;
        if (n <= PB) {
            cplx v = -acc[k];
            if (n == 0) v += acc0;
            Lam[(int64_t)n * a.nbox + b] = v;
            if (a.nloc == 2) Lam[stride + (int64_t)n * a.nbox + b] = v;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// M2L of upper sources on the FP64 matrix cores (FMMHP_FLAG_M2L_MFMA; the tuner times it against the
// vector form).  On gfx950 an FP64 matrix instruction (16 x 16 x 4, 2048 flops) occupies the SIMD's
// matrix unit for 64 cycles: the same FP64 rate as the vector ALUs, and the 2x2 embedding padded to
// 16 output columns and 4 source coefficients keeps 77% of the instructions' work at p = 20 (94% at
// p = 30): this form has been measured slower than k_m2l at p = 20 and p = 30.
// Per offset slot the tile's contraction acc_n += sum_m T_{n+m} w_m is a real GEMM in the 2x2
// embedding of complex numbers,
//   D[target][2n + c] += sum_m (Re w_m B[2m][2n + c] + Im w_m B[2m + 1][2n + c]),
//   B[2m][2n] = B[2m + 1][2n + 1] = Re T_{n+m},  B[2m][2n + 1] = -B[2m + 1][2n] = Im T_{n+m},
// run as v_mfma_f64_16x16x4f64 (lane layout measured on the device: A[i][k] from lane i + 16k,
// B[k][j] from lane j + 16k, D[i][j] in element i / 4 of lane j + 16 (i % 4)).  The K order makes
// every lane read whole complex numbers: at step s lane group g = l / 16 takes source coefficient
// m = 4s + g, the step's first instruction its real part with row 2m of B, the second its imaginary
// part with row 2m + 1, both rows from the one complex T_{n+m}.  Wave cb of the workgroup owns the
// output columns [16 cb, 16 cb + 16) (coefficients 8 cb .. 8 cb + 7) of all 64 targets of the tile:
// four 16-row blocks, four independent accumulators.  The tile's sources are staged in LDS SPP steps
// (4 SPP coefficients) at a time, with a zero row for targets that have no source at a slot; the
// operator values of the next used slot are loaded (the table stays in L2) while the current slot's
// instructions run.
// ---------------------------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kMfSteps = 1;        // steps of 4 source coefficients staged in LDS per phase


template <int PB, int SPP>
__global__ __launch_bounds__(64 * mf_ncb(PB)) void k_m2l_mf(M2LArgs a) {
    constexpr int P1 = PB + 1, NCB = mf_ncb(PB), NKS = mf_nks(PB), NTP = m2l_row(PB);
    constexpr int MPH = 4 * SPP;                        // source coefficients per phase
    constexpr int NPH = (NKS + SPP - 1) / SPP;
    constexpr int NTH = 64 * NCB;
    static_assert(kNumSlots * kTile % 8 == 0, "the slot table is copied in 16-byte pieces");
    static_assert(8 * NCB + MPH * NPH - 1 <= NTP, "operator rows cover every padded (n, m) pair");
    __shared__ cplx sW[MPH * (kM2LMaxSrc + 1)];         // [coefficient][source], row ns all zeros
    __shared__ int4 s_slot4[kNumSlots * kTile / 8];     // (slot, target) -> source, or -1
    __shared__ int32_t s_box[kTile];                    // the tile's target boxes
    __shared__ int32_t s_src[kM2LMaxSrc];               // the tile's source boxes
    __shared__ cplx s_acc0[kTile];                      // log term of lambda_0 per target
    const int16_t *s_slot = (const int16_t *)s_slot4;
    const int tile = blockIdx.x + a.tile0;
    const int tid = threadIdx.x, lane = tid & 63;
    const int cb = __builtin_amdgcn_readfirstlane(tid >> 6);
    const cplx *W = a.W + (int64_t)blockIdx.y * P1 * a.nbox;  // charge vector
    cplx *Lam = a.Lam + (int64_t)blockIdx.y * a.nloc * P1 * a.nbox;
    const int s0 = a.tile_src_off[tile];
    const int ns = a.tile_src_off[tile + 1] - s0;
    const int ns1 = ns + 1;
    const uint64_t mask = a.tile_mask[tile];
    {
        const int4 *gs = (const int4 *)(a.tile_slot + (int64_t)tile * kNumSlots * kTile);
        for (int i = tid; i < kNumSlots * kTile / 8; i += NTH) s_slot4[i] = gs[i];
        if (tid < kTile) s_box[tid] = a.tiles[tile * kTile + tid];
        for (int sj = tid; sj < ns; sj += NTH) s_src[sj] = a.tile_src[s0 + sj];
    }
    const int g = lane >> 4, c = lane & 15;
    const int nb = 8 * cb + (c >> 1);  // output coefficient of this lane's column
    const bool odd = (c & 1) != 0;     // the column holds imaginary parts
    f64x4 acc[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = (f64x4){0.0, 0.0, 0.0, 0.0};
    cplx acc0 = mk(0.0, 0.0);  // wave 0: the log term of the lane's target
#pragma unroll 1
    for (int ph = 0; ph < NPH; ++ph) {
        const int m0 = ph * MPH;
        __syncthreads();
        for (int idx = tid; idx < MPH * ns1; idx += NTH) {
            const int mm = idx / ns1, sj = idx - mm * ns1;
            cplx v = mk(0.0, 0.0);
            if (sj < ns && m0 + mm <= PB) v = W[(int64_t)(m0 + mm) * a.nbox + s_src[sj]];
            sW[idx] = v;
        }
        __syncthreads();
        if (ph == 0 && cb == 0) {
            const int bo = s_box[lane];
            const double ll = bo >= 0 ? a.logside[bo] * kInv4Pi : 0.0;
            uint64_t rest = mask;
            while (rest) {
                const int o = __builtin_ctzll(rest);
                rest &= rest - 1;
                const int li = s_slot[o * kTile + lane];
                if (li >= 0) cfma(acc0, a.Lfree[o] - mk(ll, 0.0), sW[li]);
            }
        }
        if (mask == 0) continue;
        const cplx *Tb = a.Tfree + nb + m0 + g;  // this lane's operator value: Tb[o NTP + 4 st]
        const cplx *sWg = sW + g * ns1;          // this lane's coefficient row of step 0
        // software pipeline over the used slots: the slot map, source values and operator values of
        // the next slot are loaded before the current slot's instructions issue (one basic block per
        // slot, so that the loads stay ahead of the matrix instructions)
        uint64_t rest = mask;
        int o = __builtin_ctzll(rest);
        rest &= rest - 1;
        cplx tc[SPP], wc[SPP][4];
#pragma unroll
        for (int st = 0; st < SPP; ++st) tc[st] = Tb[o * NTP + 4 * st];
        {
            int row[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int li = s_slot[o * kTile + 16 * rb + c];
                row[rb] = li >= 0 ? li : ns;
            }
#pragma unroll
            for (int st = 0; st < SPP; ++st)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) wc[st][rb] = sWg[4 * st * ns1 + row[rb]];
        }
        int left = __builtin_popcountll(mask);
        do {
            const int on = rest ? __builtin_ctzll(rest) : o;  // the last slot reloads its own values
            rest &= rest - 1;
            cplx tn[SPP], wn[SPP][4];
            int row[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int li = s_slot[on * kTile + 16 * rb + c];
                row[rb] = li >= 0 ? li : ns;
            }
#pragma unroll
            for (int st = 0; st < SPP; ++st) tn[st] = Tb[on * NTP + 4 * st];
#pragma unroll
            for (int st = 0; st < SPP; ++st)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) wn[st][rb] = sWg[4 * st * ns1 + row[rb]];
#pragma unroll
            for (int st = 0; st < SPP; ++st) {
                const double b1 = odd ? tc[st].im : tc[st].re;
                const double b2 = odd ? tc[st].re : -tc[st].im;
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
                    acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(wc[st][rb].re, b1, acc[rb], 0, 0, 0);
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
                    acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(wc[st][rb].im, b2, acc[rb], 0, 0, 0);
            }
#pragma unroll
            for (int st = 0; st < SPP; ++st) {
                tc[st] = tn[st];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) wc[st][rb] = wn[st][rb];
            }
            o = on;
        } while (--left > 0);
    }
    if (cb == 0) s_acc0[lane] = acc0;
    __syncthreads();
    if (nb > PB) return;  // padding columns
    // lambda_n = -acc_n (+ the log term for n = 0); element r of block rb: target 16 rb + 4 r + g
    const int64_t stride = (int64_t)P1 * a.nbox;
    double *out = (double *)(Lam + (int64_t)nb * a.nbox) + (odd ? 1 : 0);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = 16 * rb + 4 * r + g;
            const int b = s_box[t];
            double v = -acc[rb][r];
            if (nb == 0) v += odd ? s_acc0[t].im : s_acc0[t].re;
            if (b >= 0) {
                out[2 * (int64_t)b] = v;
                if (a.nloc == 2) out[2 * (stride + b)] = v;
            }
        }
}

// ---------------------------------------------------------------------------------------------
// M2L of upper sources on the FP32 matrix cores (FMMHP_FLAG_M2L_FP32).  Per offset slot the tile's
// contraction is a real GEMM in the 2x2 embedding of complex numbers:
//   [Re acc, Im acc](64 x 2(p+1)) += [Re w'', Im w''](64 x 2(p+1)) * [[Re T'', Im T''], [-Im T'', Re T'']]
// with the factorial scaling w''_m = m! w_m, T''_{nm} = T_{n+m} / (n! m!), acc''_n = lambda_n / n!,
// which keeps every operand within FP32 range (|T''_{nm}| <= 2^-(n+m) for separated boxes).  The
// FP32 sums of one slot are added into FP64 accumulators before the next slot; the log term of
// lambda_0 stays in FP64.
//
// Instruction: v_mfma_f32_16x16x1f32, four independent 16 x 16 rank-one updates (blocks).  Lane l
// gives A[block l / 16][row l % 16] and B[block l / 16][column l % 16]; element r of lane l holds
// D[block r / 4][row 4 (l / 16) + r % 4][column l % 16] (layout measured on the device).  The four
// blocks are the four 16-target row groups of a 64-target tile (lane l: target l), all with the
// same operator column block, so one instruction is a 64 x 16 x 1 step.  Wave pair w of the workgroup
// owns output columns [16 w, 16 w + 16), its two waves taking every other used slot (their sums
// joined through LDS at the end); K = 2(p+1) steps per slot run as two independent accumulation
// chains; the other dimension is not padded (2(p+1) columns padded to 16 only).
// (v_mfma_f32_16x16x4f32, the 16 x 16 x 4 single-block form, issues at about a fifth of this rate on
// gfx950.)  The operator column of the next slot is prefetched from global memory (the [slot]
// [column][k] table stays in L2) while the current slot runs; the tile's sources, all coefficients,
// and its (slot, target) -> source map are staged in LDS once, so waves walk their slots without
// barriers or global loads on the path to the instructions.
// ---------------------------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Row length of a source in the FP32 M2L: 2(p+1) embedded coefficients, the low parts of Re w_0 and
// Im w_0, zero padding to a multiple of 4.
__host__ __device__ constexpr int m2l32_kp(int PB) { return ((2 * (PB + 1) + 2 + 3) / 4) * 4; }
__host__ __device__ constexpr int m2l32_np(int PB) { return ((2 * (PB + 1) + 15) / 16) * 16; }

struct M2L32Args {
    int nbox;
    int tile0;               // first tile of this launch
    const int32_t *tiles, *tile_src_off, *tile_src;
    const int16_t *tile_slot;
    const uint64_t *tile_mask;
    const float *B;          // [kNumSlots][NP][KP] embedded scaled operators, column-major per slot
    const cplx *Lfree;
    const double *logside;
    const double *fact;      // n!
    const float *Wf;         // [nv][nbox][KP] FP32 source rows (k_w_f32)
    cplx *Lam;               // [nv][nloc][PB + 1][nbox]
    int nloc;
};

// One K pass of a slot: A from the target's source row in LDS (the zero row when the target has
// no source at this slot), B from the prefetched operator column; two accumulation chains.
template <int K, int KQ>
__device__ __forceinline__ void m2l32_slot(const float4 *__restrict__ ar, const float4 (&bc)[KQ], double (&acc)[16]) {
    f32x16 d0, d1;
#pragma unroll
    for (int r = 0; r < 16; ++r) d0[r] = d1[r] = 0.f;
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
        const float4 av = ar[q];
        if (4 * q + 0 < K) d0 = __builtin_amdgcn_mfma_f32_16x16x1f32(av.x, bc[q].x, d0, 0, 0, 0);
        if (4 * q + 1 < K) d1 = __builtin_amdgcn_mfma_f32_16x16x1f32(av.y, bc[q].y, d1, 0, 0, 0);
        if (4 * q + 2 < K) d0 = __builtin_amdgcn_mfma_f32_16x16x1f32(av.z, bc[q].z, d0, 0, 0, 0);
        if (4 * q + 3 < K) d1 = __builtin_amdgcn_mfma_f32_16x16x1f32(av.w, bc[q].w, d1, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] += (double)(d0[r] + d1[r]);
}

// FP32 source rows of the matrix-core M2L for the boxes [lo, hi): row b = [Re w''_0..p, Im w''_0..p]
// (w''_m = m! w_m, FP32), then w_0 - (its FP32 part) for the real and imaginary parts (so that the
// log term recovers w_0 in FP64 to about 2^-48), zero padding.  Written once per evaluation, so that
// each M2L tile stages a source with contiguous 16-byte loads.
template <int PB>
__global__ __launch_bounds__(256) void k_w_f32(int lo, int hi, int nbox, const double *__restrict__ fact,
                                               const cplx *__restrict__ W, float *__restrict__ Wf) {
    constexpr int P1 = PB + 1, K = 2 * P1, KP = m2l32_kp(PB);
    const int b = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= hi) return;
    W += (int64_t)blockIdx.y * P1 * nbox;  // charge vector
    Wf += (int64_t)blockIdx.y * nbox * KP;
    float row[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) row[k] = 0.f;
#pragma unroll
    for (int m = 0; m < P1; ++m) {
        const cplx w = W[(int64_t)m * nbox + b];
        row[m] = (float)(fact[m] * w.re);
        row[P1 + m] = (float)(fact[m] * w.im);
        if (m == 0) {
            row[K] = (float)(w.re - (double)row[0]);
            row[K + 1] = (float)(w.im - (double)row[P1]);
        }
    }
    float4 *dst = (float4 *)(Wf + (int64_t)b * KP);
#pragma unroll
    for (int q = 0; q < KP / 4; ++q) dst[q] = make_float4(row[4 * q], row[4 * q + 1], row[4 * q + 2], row[4 * q + 3]);
}

template <int PB>
__global__ __launch_bounds__(128 * (m2l32_np(PB) / 16)) void k_m2l_f32(M2L32Args a) {
    constexpr int P1 = PB + 1, K = 2 * P1, KP = m2l32_kp(PB), NP = m2l32_np(PB), NT = NP / 16;
    constexpr int KQ = KP / 4, NW = 2 * NT;  // waves: two per column block, taking alternate slots
    static_assert((kM2LMaxSrc + 1) * KQ * 16 >= NT * 64 * 16 * 8, "the partial sums reuse the source rows");
    static_assert(kNumSlots * kTile * 2 % 16 == 0, "the slot table is copied in 16-byte pieces");
    __shared__ float4 sA4[(kM2LMaxSrc + 1) * KQ];   // source rows, then one zero row
    __shared__ int4 s_slot4[kNumSlots * kTile / 8]; // (slot, target) -> source
    __shared__ cplx s_acc0[kTile];
    __shared__ cplx s_lfree[kNumSlots];
    __shared__ int32_t s_box[kTile];                // the tile's target boxes
    __shared__ int32_t s_src[kM2LMaxSrc];           // the tile's source boxes
    const float *sA = (const float *)sA4;
    const int16_t *s_slot = (const int16_t *)s_slot4;
    const int tile = blockIdx.x + a.tile0;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const float *Wf = a.Wf + (int64_t)blockIdx.y * a.nbox * KP;  // charge vector
    cplx *Lam = a.Lam + (int64_t)blockIdx.y * a.nloc * P1 * a.nbox;
    const int s0 = a.tile_src_off[tile];
    const int ns = a.tile_src_off[tile + 1] - s0;
    const uint64_t mask = a.tile_mask[tile];
    // prologue in two rounds of independent loads: first the tile's tables (slot map, boxes, source
    // indices, log-term constants), then the source rows (scaled, embedded FP32) and a zero row
    {
        const int4 *g = (const int4 *)(a.tile_slot + (int64_t)tile * kNumSlots * kTile);
        for (int i = tid; i < kNumSlots * kTile / 8; i += 64 * NW) s_slot4[i] = g[i];
        if (tid < kTile) s_box[tid] = a.tiles[tile * kTile + tid];
        if (tid < kNumSlots) s_lfree[tid] = a.Lfree[tid];
        for (int sj = tid; sj < ns; sj += 64 * NW) s_src[sj] = a.tile_src[s0 + sj];
    }
    __syncthreads();
    for (int sj = tid; sj < ns; sj += 2 * 64 * NW) {
        const int sj2 = sj + 64 * NW;
        const float4 *r1 = (const float4 *)(Wf + (int64_t)s_src[sj] * KP);
        const float4 *r2 = sj2 < ns ? (const float4 *)(Wf + (int64_t)s_src[sj2] * KP) : r1;
        float4 v1[KQ], v2[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            v1[q] = r1[q];
            v2[q] = r2[q];
        }
#pragma unroll
        for (int q = 0; q < KQ; ++q) sA4[sj * KQ + q] = v1[q];
        if (sj2 < ns) {
#pragma unroll
            for (int q = 0; q < KQ; ++q) sA4[sj2 * KQ + q] = v2[q];
        }
    }
    for (int q = tid; q < KQ; q += 64 * NW) sA4[ns * KQ + q] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int b_own = s_box[lane];
    const double ll = wave == 0 && b_own >= 0 ? a.logside[b_own] * kInv4Pi : 0.0;
    __syncthreads();
    // log term of lambda_0 in FP64, one lane per target (wave 0): w_0 from its FP32 part and remainder
    if (wave == 0) {
        cplx acc0 = mk(0.0, 0.0);
        uint64_t rest = mask;
        while (rest) {
            const int o = __builtin_ctzll(rest);
            rest &= rest - 1;
            const int li = s_slot[o * kTile + lane];
            if (li >= 0) {
                const float *row = sA + li * KP;
                const cplx w0 = mk((double)row[0] + (double)row[K], (double)row[P1] + (double)row[K + 1]);
                cfma(acc0, s_lfree[o] - mk(ll, 0.0), w0);
            }
        }
        s_acc0[lane] = acc0;
    }
    double acc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0;
    const int nt = wave % NT, half = wave / NT;
    const int col = 16 * nt + (lane & 15);  // operator column of this lane in all four blocks
    const bool im = col >= P1;
    const int n = im ? col - P1 : col;       // output coefficient of the column (col < K)
    const double fn = col < K ? a.fact[n] : 0.0;
    const float4 *Bcol = (const float4 *)(a.B + (int64_t)col * KP);
    constexpr int64_t kSlotQ = (int64_t)NP * KQ;  // float4 per slot
    auto row_of = [&](int o) -> const float4 * {
        const int li = s_slot[o * kTile + lane];
        return sA4 + (li >= 0 ? li : ns) * KQ;
    };
    // this wave's used slots (every other one, ascending), operator columns in two register buffers
    // (ping-pong): the column of the next slot loads while the current one runs
    uint64_t rest = mask;
    int rc = 0;  // used slots passed so far
    auto next = [&]() -> int {  // the next used slot of this half, or -1
        while (rest) {
            const int o = __builtin_ctzll(rest);
            rest &= rest - 1;
            if ((rc++ & 1) == half) return o;
        }
        return -1;
    };
    float4 b0[KQ], b1[KQ];
    int o0 = next();
    if (o0 >= 0) {
#pragma unroll
        for (int q = 0; q < KQ; ++q) b0[q] = Bcol[o0 * kSlotQ + q];
    }
    while (o0 >= 0) {
        const int o1 = next();
        if (o1 >= 0) {
#pragma unroll
            for (int q = 0; q < KQ; ++q) b1[q] = Bcol[o1 * kSlotQ + q];
        }
        m2l32_slot<K, KQ>(row_of(o0), b0, acc);
        if (o1 < 0) break;
        o0 = next();
        if (o0 >= 0) {
#pragma unroll
            for (int q = 0; q < KQ; ++q) b0[q] = Bcol[o0 * kSlotQ + q];
        }
        m2l32_slot<K, KQ>(row_of(o1), b1, acc);
    }
    // the second half's sums join the first's through LDS (the source rows are no longer needed)
    __syncthreads();
    double *sred = (double *)sA4;
    if (half == 1) {
#pragma unroll
        for (int e = 0; e < 16; ++e) sred[(nt * 16 + e) * 64 + lane] = acc[e];
    }
    __syncthreads();
    if (half == 1) return;
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] += sred[(nt * 16 + e) * 64 + lane];
    // lambda_n = -n! acc''_n (+ the log term for n = 0); element e: target 16 (e/4) + 4 (l/16) + e%4.
    // Box indices and log terms come from LDS, so the stores do not wait on memory loads.
    if (col >= K) return;
    const int64_t stride = (int64_t)P1 * a.nbox;
    double *out = (double *)(Lam + (int64_t)n * a.nbox) + (im ? 1 : 0);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int t = 16 * (e >> 2) + 4 * (lane >> 4) + (e & 3);
        const int b = s_box[t];
        double v = -fn * acc[e];
        if (n == 0) v += im ? s_acc0[t].im : s_acc0[t].re;
        if (b >= 0) {
            out[2 * (int64_t)b] = v;
            if (a.nloc == 2) out[2 * (stride + b)] = v;
        }
    }
}

// Image V entries (target boxes in the two rows nearest y = 0 at each level): log M2L of the image
// box plus the reaction M2L, added to the locals written by k_m2l.  One block per target box and all
// vectors of the pass: entry group g (G = min(kImgThreads / (p + 1), kImgGroups) groups) sums every
// G-th V entry of the box, lane n of its thread group computing output coefficient n and reading the
// entry's operator row coalesced across n; the groups' sums are joined through LDS in a fixed order.
// The same partition for any number of vectors, so a vector's result does not depend on the others
// in its pass.
constexpr int kImgThreads = 256;
constexpr int kImgGroups = 8;
// Threads of a block: 256 for one vector; 64 for several (each thread then holds every vector's
// sums, and a small block keeps more boxes in flight per CU).
__host__ __device__ constexpr int img_threads(int nv) { return nv == 1 ? kImgThreads : 64; }

template <int PB, int NV>
__global__ __launch_bounds__(img_threads(NV)) void k_m2l_img(const int32_t *__restrict__ ibox, int nbox, int nloc,
                                                             const int32_t *__restrict__ ibase,
                                                             const int32_t *__restrict__ vimg_off,
                                                             const int32_t *__restrict__ vimg_ent,
                                                             const cplx *__restrict__ TH, const cplx *__restrict__ TG,
                                                             const cplx *__restrict__ Limg,
                                                             const double *__restrict__ logside, double isg,
                                                             const cplx *__restrict__ W, cplx *__restrict__ Lam) {
    constexpr int NTP = m2l_row(PB);
    constexpr int P1 = PB + 1;
    // G entry groups (entry e in group e mod G), the same for every vector count so that the sums
    // are formed in one order; GT thread groups of p + 1 lanes each take groups tg + k GT in turn
    constexpr int G = kImgThreads / P1 < kImgGroups ? kImgThreads / P1 : kImgGroups;
    constexpr int GT = img_threads(NV) / P1 < G ? img_threads(NV) / P1 : G;
    static_assert(G >= 1 && GT >= 1, "one group of p + 1 lanes fits the block");
    __shared__ cplx red[G > 1 ? G - 1 : 1][NV][2][P1];
    const int b = ibox[blockIdx.x];
    const int tid = threadIdx.x;
    const int tg = tid / P1, n = tid - tg * P1;
    const int l = ibase[b];  // table block of the box's (instance, level)
    const double ll = logside[b] * kInv4Pi;
    cplx aH[NV], aG[NV];
    if (tg < GT) {
        // this thread group's entry groups, highest first: thread group 0 ends on group 0, whose
        // sums stay in registers; every other group's sums go to LDS
        for (int g = tg + ((G - 1 - tg) / GT) * GT; g >= 0; g -= GT) {
#pragma unroll
            for (int v = 0; v < NV; ++v) aH[v] = aG[v] = mk(0.0, 0.0);
            for (int e = vimg_off[b] + g; e < vimg_off[b + 1]; e += G) {
                const int code = vimg_ent[e];
                const int src = code >> 5, is = code & 31;
                const cplx *th = TH + ((int64_t)l * kNumImgSlots + is) * NTP + n;
                const cplx *tg_ = TG + ((int64_t)l * kNumImgSlots + is) * NTP + n;
                // several loads of an entry in flight for one vector; fewer registers with several
#pragma unroll(NV == 1 ? 8 : 2)
                for (int m = 0; m <= PB; ++m) {
                    const cplx t = th[m];
                    const cplx tq = nloc == 2 ? tg_[m] : mk(0.0, 0.0);
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const cplx wm = conj(W[((int64_t)v * P1 + m) * nbox + src]);
                        cfma(aH[v], t, wm);
                        if (nloc == 2) cfma(aG[v], tq, wm);
                    }
                }
                if (n == 0) {  // the log term: lambda_0 += (L + log side) conj(w_0), entered with the sign of -a
                    const cplx f = -(Limg[is] + mk(isg * ll, 0.0));
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const cplx w0 = conj(W[(int64_t)v * P1 * nbox + src]);
                        cfma(aH[v], f, w0);
                        cfma(aG[v], f, w0);
                    }
                }
            }
            if (g >= 1) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    red[g - 1][v][0][n] = aH[v];
                    red[g - 1][v][1][n] = aG[v];
                }
            }
        }
    }
    // the groups' sums meet in thread group 0, groups in ascending order for every vector
    if (G > 1) {
        __syncthreads();
        if (tg == 0) {
            for (int h = 0; h + 1 < G; ++h)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    aH[v] += red[h][v][0][n];
                    aG[v] += red[h][v][1][n];
                }
        }
    }
    if (tg == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            cplx *Lv = Lam + (int64_t)v * nloc * P1 * nbox;
            Lv[(int64_t)n * nbox + b] += -aH[v];
            if (nloc == 2) Lv[(int64_t)P1 * nbox + (int64_t)n * nbox + b] += -aG[v];
        }
    }
}

__global__ void k_zero_lam(int lo, int hi, int nbox, int ncoef, int nrow, cplx *__restrict__ Lam) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nb = hi - lo;
    if (i >= nb * ncoef * nrow) return;
    const int64_t b = lo + i % nb;
    const int64_t r = i / nb;  // (vector * nloc + loc) * ncoef + n
    Lam[r * nbox + b] = mk(0.0, 0.0);
}

// Lane moves within a wave by DPP (no LDS traffic, a few cycles), for doubles as two 32-bit halves.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Lane l's value of x in every lane (l uniform; reads the lane's register whatever the exec mask).
__device__ __forceinline__ double read_lane_f64(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// Sum over aligned groups of IA = 1, 2, 4 or 8 consecutive lanes (every lane of a group gets it).
__device__ __forceinline__ double lane_group_sum(double s, int IA) {
    if (IA >= 2) s += dpp_move<0xB1, 0xF>(s);   // quad_perm [1, 0, 3, 2]
    if (IA >= 4) s += dpp_move<0x4E, 0xF>(s);   // quad_perm [2, 3, 0, 1]
    if (IA >= 8) s += dpp_move<0x141, 0xF>(s);  // row_half_mirror
    return s;
}

// ---------------------------------------------------------------------------------------------
// P2L (X list): sources of a coarse leaf straight into the local of a finer box.  A wave takes a
// group of X boxes of one level (consecutive boxes whose X sources total at most 64, or one larger
// box) and walks the group's sources in chunks of 64, one source per lane in the order (box, list
// entry, point).  Each lane computes its source's terms for unit charge into LDS, a phase of
// coefficients at a time: 16 when the chunk has no reaction rows (the G local's terms then equal the
// H local's), else 8 of every local.  With one vector, lane (k, g) sums coefficient k of each box of
// the chunk over the box's rows g, g + G, ... (G = 4 or 8) times the charges, and the G partial sums
// meet by lane moves; with several, lane (k, vector group) forms the same G partial sums itself and
// joins them in the same order.  The sums are added to the locals by atomics that return nothing.
// Dipole sources (DIP) take the derivative of these contributions along the source normal: the log
// local is holomorphic in d = z_j - c_b (upper box) or in conj(z_j) - c_b (image), so the derivative
// is nu d/dd (nu = n_x + i n_y, or its conjugate for the image), and for the reaction local
// n_j . grad_{r_j} [n! rho^n I_n] = -(1/rho) i conj(nu) K_{n+1} (d_X I_n = i (n+1) I_{n+1},
// d_Y I_n = -(n+1) I_{n+1}, from eq. (generalintegral)); the same holds for the mirrored G local.
// ---------------------------------------------------------------------------------------------
constexpr int kP2LPhase = 8;   // coefficients per LDS phase with reaction rows (16 without)
constexpr int kP2LRows = 72;   // row stride of the 8-coefficient layout (68 in the 16-coefficient one)

// Plan-time tables of the P2L: each group entry's first source point (w), and each X box's centre,
// half side and instance, so that a chunk's loads depend only on its group entries.
__global__ void k_xgent_first(int64_t m, int4 *__restrict__ gent, const int32_t *__restrict__ first) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) gent[e].w = first[gent[e].x >> 1];
}

__global__ void k_xgeo(int nx, const int32_t *__restrict__ xbox, const InstInfo *__restrict__ ii,
                       const int32_t *__restrict__ inst, const int32_t *__restrict__ level,
                       const int32_t *__restrict__ bx, const int32_t *__restrict__ by, double4 *__restrict__ xgeo) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx) return;
    const int b = xbox[i], l = level[b], k = inst[b];
    const Geo g = geo_of(ii, k);
    const cplx cb = centre_of(g, l, bx[b], by[b]);
    xgeo[i] = make_double4(cb.re, cb.im, 0.5 * side_of(g, l), (double)k);
}

// A box slot's sums for several vectors: lane group vg takes vectors vg VPL .. vg VPL + VPL - 1 of
// the coefficient row Ck and forms, per vector, the G row-group sums that the single-vector lanes
// form (group g: rows r0 + g, r0 + g + G, ...) and joins them in the order of their lane-move tree,
// so that every vector's result is bitwise the one of a single-vector pass.
template <int PB, int NV, int G, int VPL>
__device__ __forceinline__ void p2l_slot_vectors(const cplx *Ck, const double (*sq)[NV], int r0, int r1, int vg,
                                                 int m, int ld0, int ld1, int nloc, int nbox, int bsl,
                                                 cplx *__restrict__ Lam) {
    constexpr int P1 = PB + 1;
    cplx pg[G][VPL];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int u = 0; u < VPL; ++u) pg[g][u] = mk(0.0, 0.0);
    // a block's G rows are loaded together (at a valid row past the end) and added in row order
    for (int r = r0; r < r1; r += G) {
        cplx t[G];
        double qv[G][VPL];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int rr = r + g < r1 ? r + g : r1 - 1;
            t[g] = Ck[rr];
#pragma unroll
            for (int u = 0; u < VPL; ++u) {
                const int v = vg * VPL + u;
                qv[g][u] = sq[rr][v < NV ? v : 0];
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (r + g < r1) {
#pragma unroll
                for (int u = 0; u < VPL; ++u)
                    if (vg * VPL + u < NV) pg[g][u] += qv[g][u] * t[g];
            }
        }
    }
    if (m > PB) return;
#pragma unroll
    for (int u = 0; u < VPL; ++u) {
        const int v = vg * VPL + u;
        if (v >= NV) continue;
        cplx a = (pg[0][u] + pg[1][u]) + (pg[2][u] + pg[3][u]);
        if constexpr (G == 8) a = a + ((pg[4][u] + pg[5][u]) + (pg[6][u] + pg[7][u]));
        for (int ld = ld0; ld < ld1; ++ld) {
            cplx *dst = Lam + (((int64_t)v * nloc + ld) * P1 + m) * nbox + bsl;
            unsafeAtomicAdd(&dst->re, a.re);
            unsafeAtomicAdd(&dst->im, a.im);
        }
    }
}

template <int PB, bool DIP, int NV>
__global__ __launch_bounds__(64) void k_p2l(const InstInfo *__restrict__ ii, const int32_t *__restrict__ inst,
                                            int nloc, const int4 *__restrict__ grp, const int4 *__restrict__ gent,
                                            const int32_t *__restrict__ xbox, const double4 *__restrict__ xgeo,
                                            int nbox, const double *__restrict__ xs, const double *__restrict__ ys,
                                            const double *__restrict__ qs, const double2 *__restrict__ nrm,
                                            const double *__restrict__ fact, cplx *__restrict__ Lam) {
    constexpr int P1 = PB + 1;
    // [local][coefficient in phase][source row], 2 x 8 coefficients or 1 x 16 (row strides 72 and 68
    // with one vector, 65 with several)
    __shared__ cplx C[2 * kP2LPhase * kP2LRows];
    __shared__ double sq[64][NV];
    const int lane = threadIdx.x;
    // n! in lane n: the term loops read it by lane moves (a scalar load there would wait for the
    // LDS writes before it, which count on the same counter)
    const double fact_l = lane <= PB ? fact[lane] : 0.0;
    const int4 gd = grp[blockIdx.x], gn = grp[blockIdx.x + 1];
    const int gs = gd.x, K = gd.y, eg1 = gn.z;
    int elo = gd.z;                            // first list entry of the current chunk
    for (int F = 0; F < K; F += 64) {
        const int f = F + lane;
        // the chunk's entries {code, slot, first row, first source point}: at most 64 (every entry
        // holds a source), in order of first row; lane f takes the last one starting at or before f
        const int ne = eg1 - elo < 64 ? eg1 - elo : 64;
        const int4 en = lane < ne ? gent[elo + lane] : make_int4(0, 0, 0, 0);
        int my = 0;
        for (int t = 1; t < ne; ++t) {
            const int st = __builtin_amdgcn_readlane(en.z, t);
            if (st > F + 63) break;
            if (st <= f) my = t;
        }
        const int code = __shfl(en.x, my), s = __shfl(en.y, my), f0 = __shfl(en.z, my), j0 = __shfl(en.w, my);
        {
            // first entry of the next chunk: lane 63's, or the one after it if that starts the chunk
            const int m63 = __builtin_amdgcn_readlane(my, 63);
            const int nx = elo + m63 + 1;
            const int stn = nx < eg1 ? gent[nx].z : 0x7fffffff;
            elo = stn <= F + 64 ? nx : elo + m63;
        }
        const bool act = f < K;
        // the lane's source, target box and the state of its term recursions
        const int img = act ? code & 1 : 0;
        const int j = act ? j0 + (f - f0) : 0;
        const int b = xbox[gs + (act ? s : 0)];
        const double4 bg = xgeo[gs + (act ? s : 0)];  // target box: centre, half side, instance
        const cplx cb = mk(bg.x, bg.y);
        const double rho = bg.z;
        const int k = (int)bg.w;
        const bool rx = act && img && ii[k].react;
        cplx sig = mk(0.0, 0.0), pw = mk(0.0, 0.0), l0 = mk(0.0, 0.0);
        double sgn = 0.0;
        cplx sw[2], Fr[2], Kr[2], zr = mk(0.0, 0.0), cn = mk(0.0, 0.0);
#pragma unroll
        for (int lc = 0; lc < 2; ++lc) sw[lc] = Fr[lc] = Kr[lc] = mk(0.0, 0.0);
        if (act) {
#pragma unroll
            for (int v = 0; v < NV; ++v) sq[lane][v] = qs[(int64_t)j * NV + v];
            const double yj = img ? -ys[j] : ys[j];
            const cplx d = mk(xs[j] - cb.re, yj - cb.im);   // source - centre
            sgn = img ? ii[k].isg : -1.0;                     // -(1/4pi) upper, +-(1/4pi) image
            sig = rho * inv(d);
            if (DIP) {
                // nu d/dd of the charge's local below: (nu / rho) n! sig^(n+1)
                const double2 nj = nrm[j];
                pw = ((sgn * kInv4Pi / rho) * mk(nj.x, img ? -nj.y : nj.y)) * sig;
            } else {
                // local of log(z - z_j) about c_b: log(c_b - z_j) - sum_n (z - c_b)^n / (n (z_j - c_b)^n)
                l0 = (sgn * kInv4Pi) * clog_(-d);
                pw = sig;
            }
            if (rx) {
                // reaction S2L (eq. (LEcoefficients)) re-expanded in powers of (z - c_b):
                // lambda_n += i^n n! rho^n q I_n(x_c - x_j, y_c + y_j)  (G: conj of I_n(-X, Y))
                const double X = cb.re - xs[j], Y = cb.im + ys[j];
                const cplx Z = ii[k].Z;
                zr = rho * Z;
                if (DIP) {
                    const double2 nj = nrm[j];
                    cn = (-1.0 / rho) * mk(nj.x, -nj.y);  // lambda_(n-1) += -(mu conj(nu) / rho) i^n K_n
                }
#pragma unroll
                for (int lc = 0; lc < 2; ++lc) {
                    if (lc == nloc) break;
                    const double Xs = lc == 0 ? X : -X;
                    sw[lc] = rho * inv(mk(Y, -Xs));
                    Kr[lc] = reaction_I0_general(Xs, Y, Z);
                    Fr[lc] = mk(1.0, 0.0);
                }
            }
        }
        // every load of the chunk has landed before the phases: otherwise the compiler's merged wait
        // state keeps a count wait in each coefficient step, which from the second phase on also
        // waits for the previous phase's local adds
        __builtin_amdgcn_s_waitcnt(0);
        // box slots present in this chunk
        const int sa = __builtin_amdgcn_readlane(s, 0);
        const int sb = __builtin_amdgcn_readlane(s, K - F < 64 ? K - F - 1 : 63);
        // Without reaction rows the G terms equal the H terms: one set of terms, one sum added to
        // every local, 16 coefficients a phase summed by 4 lanes each.  With reaction rows, every
        // local has its own terms, 8 coefficients a phase summed by 8 lanes each.  Row strides keep
        // the 16 lanes of an LDS access on distinct banks in either layout.
        const bool mixed = __ballot(rx) != 0;
        const int ph = mixed ? kP2LPhase : 2 * kP2LPhase;
        const int nl = mixed ? nloc : 1;
        const int G = mixed ? 8 : 4;
        const int rs = NV > 1 ? kP2LRows - 7 : mixed ? kP2LRows : kP2LRows - 4;
        const int gq = lane & (G - 1), kq = mixed ? lane >> 3 : lane >> 2;
        for (int m0 = 0; m0 <= PB; m0 += ph) {
            if (act) {
#pragma unroll
                for (int kk = 0; kk < 2 * kP2LPhase; ++kk) {
                    const int m = m0 + kk;
                    if (kk == ph || m > PB) break;
                    cplx t;
                    if (DIP) {
                        t = read_lane_f64(fact_l, m) * pw;
                        pw = pw * sig;
                    } else if (m == 0) {
                        t = l0;
                    } else {
                        t = (-sgn * kInv4Pi * read_lane_f64(fact_l, m - 1)) * pw;
                        pw = pw * sig;
                    }
#pragma unroll
                    for (int lc = 0; lc < 2; ++lc) {
                        if (lc == nl) break;
                        cplx u = t;
                        if (rx) {
                            const int n = DIP ? m + 1 : m;  // order of I_n this coefficient takes
                            if (n > 0) {
                                Fr[lc] = Fr[lc] * sw[lc] * (n > 1 ? (double)(n - 1) : 1.0);  // (n-1)! sw^n
                                Kr[lc] = Fr[lc] * kInv2Pi + zr * Kr[lc];
                            }
                            const cplx kn = mul_ipow(lc == 0 ? Kr[lc] : conj(Kr[lc]), n);
                            u += DIP ? cn * kn : kn;
                        }
                        C[(lc * ph + kk) * rs + lane] = u;
                    }
                }
            }
            __syncthreads();
            const int m = m0 + kq;
            for (int sl = sa; sl <= sb; ++sl) {
                const uint64_t msk = __ballot(act && s == sl);
                const int r0 = __builtin_ctzll(msk), r1 = 64 - __builtin_clzll(msk);
                const int bsl = __builtin_amdgcn_readlane(b, r0);  // the slot's box, from its first row
                for (int lc = 0; lc < nl; ++lc) {
                    if constexpr (NV > 1) {
                        // lane (coefficient, vector group); row stride 65: the 16 coefficient rows
                        // of an access fall on distinct banks
                        const int kv = lane & (ph - 1), vg = lane / ph;
                        const cplx *Cv = C + (lc * ph + kv) * rs;
                        const int ld0 = mixed ? lc : 0, ld1 = mixed ? lc + 1 : nloc;
                        if (mixed)
                            p2l_slot_vectors<PB, NV, 8, (NV + 7) / 8>(Cv, sq, r0, r1, vg, m0 + kv, ld0, ld1, nloc,
                                                                       nbox, bsl, Lam);
                        else
                            p2l_slot_vectors<PB, NV, 4, (NV + 3) / 4>(Cv, sq, r0, r1, vg, m0 + kv, ld0, ld1, nloc,
                                                                       nbox, bsl, Lam);
                        continue;
                    }
                    const cplx *Ck = C + (lc * ph + kq) * rs;
                    cplx acc[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) acc[v] = mk(0.0, 0.0);
                    // four of the lane's rows loaded together (at a valid row past the end), added
                    // in row order
                    for (int r = r0 + gq; r < r1; r += 4 * G) {
                        cplx t[4];
                        double qv[4][NV];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int ri = r + i * G < r1 ? r + i * G : r;
                            t[i] = Ck[ri];
#pragma unroll
                            for (int v = 0; v < NV; ++v) qv[i][v] = sq[ri][v];
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (r + i * G < r1) {
#pragma unroll
                                for (int v = 0; v < NV; ++v) acc[v] += qv[i][v] * t[i];
                            }
                        }
                    }
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        acc[v].re = lane_group_sum(acc[v].re, G);
                        acc[v].im = lane_group_sum(acc[v].im, G);
                    }
                    // only this wave adds to the box's locals here, one lane per coefficient in
                    // program order, so the sums stay deterministic; the adds return nothing and the
                    // wave does not wait for them
                    if (gq == 0 && m <= PB && kq < ph) {
                        for (int ld = mixed ? lc : 0; ld < (mixed ? lc + 1 : nloc); ++ld) {
#pragma unroll
                            for (int v = 0; v < NV; ++v) {
                                cplx *dst = Lam + (((int64_t)v * nloc + ld) * P1 + m) * nbox + bsl;
                                unsafeAtomicAdd(&dst->re, acc[v].re);
                                unsafeAtomicAdd(&dst->im, acc[v].im);
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------------------------
// L2L.  A block takes kL2LChildren consecutive children and stages each child's parent local in
// LDS (siblings share cache lines).  Thread (child, m) adds 2^-m sum_{n>=m} eps^{n-m}/(n-m)!
// lambda^P_n to lambda^c_m.  k_l2l runs one level of children; k_l2l_sub every level below a cut
// level, one block per subtree rooted at the cut, top level first.
// ---------------------------------------------------------------------------------------------
constexpr int kL2LChildren = 64;

template <int PB>
struct L2LShared {
    cplx sE[4 * (PB + 1)];
};

// Children [c0, c0 + nc) of one level, nc <= kL2LChildren; called by every thread of the block.
// The parents' locals are staged in the LDS rows sl (row length ld >= kL2LChildren).  The
// children's own locals are read before the parents' are staged, so that both loads overlap.
// Ends with a barrier, so the locals written are visible to the whole block.
template <int PB>
__device__ __forceinline__ void l2l_children(L2LShared<PB> &sh, cplx *sl, int ld, int c0, int nc, int nbox, int nloc,
                             const int32_t *__restrict__ parent, const int32_t *__restrict__ bx,
                             const int32_t *__restrict__ by, cplx *__restrict__ Lam) {
    constexpr int MS = 256 / kL2LChildren;         // threads per child
    constexpr int MP = (PB + MS) / MS;             // coefficients per thread
    const int ci = threadIdx.x % kL2LChildren;
    const int mt = threadIdx.x / kL2LChildren;
    const int c = c0 + ci;
    const int q = ci < nc ? ((bx[c] & 1) | ((by[c] & 1) << 1)) : 0;
    for (int loc = 0; loc < nloc; ++loc) {
        cplx *L = Lam + (int64_t)loc * (PB + 1) * nbox;
        cplx own[MP];
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            const int m = mt + k * MS;
            own[k] = (ci < nc && m <= PB) ? L[(int64_t)m * nbox + c] : mk(0.0, 0.0);
        }
        for (int idx = threadIdx.x; idx < (PB + 1) * nc; idx += blockDim.x) {
            const int n = idx / nc, k = idx - n * nc;
            sl[n * ld + k] = L[(int64_t)n * nbox + parent[c0 + k]];
        }
        __syncthreads();
        if (ci < nc) {
#pragma unroll
            for (int k = 0; k < MP; ++k) {
                const int m = mt + k * MS;
                if (m <= PB) {
                    const cplx s = l2l_coef<PB>(sh.sE + q * (PB + 1) - m, sl + ci, ld, m);
                    L[(int64_t)m * nbox + c] = own[k] + s * ldexp(1.0, -m);
                }
            }
        }
        __syncthreads();
    }
}

template <int PB>
__global__ __launch_bounds__(256) void k_l2l(int lo, int nb, int nbox, int nloc, const int32_t *__restrict__ parent,
                                             const int32_t *__restrict__ bx, const int32_t *__restrict__ by,
                                             const cplx *__restrict__ E, cplx *__restrict__ Lam) {
    __shared__ L2LShared<PB> sh;
    extern __shared__ cplx dyn_lds[];  // (PB + 1) x kL2LChildren
    Lam += (int64_t)blockIdx.y * nloc * (PB + 1) * nbox;  // charge vector
    for (int k = threadIdx.x; k < 4 * (PB + 1); k += blockDim.x) sh.sE[k] = E[k];
    const int c0 = lo + blockIdx.x * kL2LChildren;
    l2l_children<PB>(sh, dyn_lds, kL2LChildren, c0, min(kL2LChildren, lo + nb - c0), nbox, nloc, parent, bx, by,
                     Lam);
}

// L2L of the children [c.x, c.y) of one level for each chunk c (at most kL2LChildren children): the
// subtrees too large for LDS, one launch per level, top level first.
template <int PB>
__global__ __launch_bounds__(256) void k_l2l_chunks(const int2 *__restrict__ chunks, int nbox, int nloc,
                                                    const int32_t *__restrict__ parent, const int32_t *__restrict__ bx,
                                                    const int32_t *__restrict__ by, const cplx *__restrict__ E,
                                                    cplx *__restrict__ Lam) {
    __shared__ L2LShared<PB> sh;
    extern __shared__ cplx dyn_lds[];  // (PB + 1) x kL2LChildren
    Lam += (int64_t)blockIdx.y * nloc * (PB + 1) * nbox;  // charge vector
    for (int k = threadIdx.x; k < 4 * (PB + 1); k += blockDim.x) sh.sE[k] = E[k];
    const int2 c = chunks[blockIdx.x];
    l2l_children<PB>(sh, dyn_lds, kL2LChildren, c.x, c.y - c.x, nbox, nloc, parent, bx, by, Lam);
}

// skip_big: a subtree whose locals do not fit the block's LDS rows is left to k_l2l_chunks.
template <int PB>
__global__ __launch_bounds__(256) void k_l2l_sub(int nlev, const int2 *__restrict__ rng, int ld, int skip_big, int nbox,
                                                 int nloc,
                                                 const int32_t *__restrict__ parent, const int32_t *__restrict__ bx,
                                                 const int32_t *__restrict__ by, const cplx *__restrict__ E,
                                                 cplx *__restrict__ Lam) {
    __shared__ L2LShared<PB> sh;
    __shared__ SubShared ss;
    extern __shared__ cplx dyn_lds[];  // (PB + 1) x ld
    cplx *sl = dyn_lds;
    Lam += (int64_t)blockIdx.y * nloc * (PB + 1) * nbox;  // charge vector
    for (int k = threadIdx.x; k < 4 * (PB + 1); k += blockDim.x) sh.sE[k] = E[k];
    const int2 *R = rng + (int64_t)blockIdx.x * nlev;
    sub_ranges(ss, R, nlev);
    const int tot = ss.base[nlev];
    if (tot * nloc > ld) {
        if (skip_big) return;
        for (int k = 1; k < nlev; ++k) {
            const int2 r = R[k];
            for (int c0 = r.x; c0 < r.y; c0 += kL2LChildren)
                l2l_children<PB>(sh, sl, ld, c0, min(kL2LChildren, r.y - c0), nbox, nloc, parent, bx, by, Lam);
        }
        return;
    }
    // resident: slot loc * tot + i holds local loc of box i, coefficient n at sl[n * ld + slot];
    // the root's local is final (the levels above ran first), the others hold their own M2L/P2L
    // parts until their level is reached
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        const int k = sub_level_of(ss, nlev, i);
        const int b = ss.first[k] + (i - ss.base[k]);
        ss.slot[i] = k == 0 ? -1 : ss.base[k - 1] + (parent[b] - ss.first[k - 1]);
        ss.quad[i] = (bx[b] & 1) | ((by[b] & 1) << 1);
    }
    for (int idx = threadIdx.x; idx < nloc * tot * (PB + 1); idx += blockDim.x) {
        const int n = idx / (nloc * tot), r = idx - n * nloc * tot, loc = r / tot, i = r - loc * tot;
        const int k = sub_level_of(ss, nlev, i);
        const int b = ss.first[k] + (i - ss.base[k]);
        sl[n * ld + r] = Lam[((int64_t)loc * (PB + 1) + n) * nbox + b];
    }
    __syncthreads();
    for (int k = 1; k < nlev; ++k) {
        const int i0 = ss.base[k], nc = ss.base[k + 1] - i0;
        for (int idx = threadIdx.x; idx < nloc * nc * (PB + 1); idx += blockDim.x) {
            const int m = idx / (nloc * nc), r = idx - m * nloc * nc, loc = r / nc, i = i0 + (r - loc * nc);
            const int ps = loc * tot + ss.slot[i], cs = loc * tot + i;
            const cplx acc = l2l_coef<PB>(sh.sE + ss.quad[i] * (PB + 1) - m, sl + ps, ld, m);
            const cplx v = sl[m * ld + cs] + acc * ldexp(1.0, -m);
            sl[m * ld + cs] = v;
            Lam[((int64_t)loc * (PB + 1) + m) * nbox + ss.first[k] + (i - i0)] = v;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Surface term for a real impedance: s_k = sum_{j in instance k} q_j exp(-Z_k (y_j - i x_j)) per
// instance and charge vector.  Partial sums over point chunks that never straddle instances, then
// a fixed-order sum over each instance's chunks.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ cplx block_sum(cplx v) {
    __shared__ double sr[256], si[256];
    sr[threadIdx.x] = v.re;
    si[threadIdx.x] = v.im;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sr[threadIdx.x] += sr[threadIdx.x + off];
            si[threadIdx.x] += si[threadIdx.x + off];
        }
        __syncthreads();
    }
    return mk(sr[0], si[0]);
}

// Surface sums s = sum_j q_j e^{-Z(y_j - i x_j)}; for dipoles (DIP) the normal derivative of each
// term, mu_j Z (i n_x - n_y) e^{-Z(y_j - i x_j)} (the exponential is holomorphic in z_j).
template <bool DIP>
__global__ __launch_bounds__(256) void k_rank1_partial(const double *__restrict__ xs, const double *__restrict__ ys,
                                                       const double *__restrict__ qs, int nv,
                                                       const PtChunk *__restrict__ ch, int nch,
                                                       const InstInfo *__restrict__ ii, const double2 *__restrict__ nrm,
                                                       cplx *__restrict__ part) {
    const PtChunk c = ch[blockIdx.x];
    const int v = blockIdx.y;
    const double Z = ii[c.inst].Z.re;
    double ar = 0.0, ai = 0.0;
    for (int64_t i = c.start + threadIdx.x; i < c.end; i += 256) {
        const double e = qs[i * nv + v] * exp(-Z * ys[i]);
        double sn, cs;
        sincos(Z * xs[i], &sn, &cs);
        if (DIP) {
            const double2 nj = nrm[i];
            const double ez = Z * e;
            ar -= ez * (nj.y * cs + nj.x * sn);
            ai += ez * (nj.x * cs - nj.y * sn);
        } else {
            ar += e * cs;
            ai += e * sn;
        }
    }
    const cplx t = block_sum(mk(ar, ai));
    if (threadIdx.x == 0) part[(int64_t)v * nch + blockIdx.x] = t;
}

// out[v][k] = sum of part[v][c] over the chunks c of instance k, in chunk order
__global__ __launch_bounds__(256) void k_rank1_final(const cplx *__restrict__ part, int nch,
                                                     const int32_t *__restrict__ inst_ch, int n_inst,
                                                     cplx *__restrict__ out) {
    const int k = blockIdx.x, v = blockIdx.y;
    double ar = 0.0, ai = 0.0;
    for (int c = inst_ch[k] + threadIdx.x; c < inst_ch[k + 1]; c += 256) {
        ar += part[(int64_t)v * nch + c].re;
        ai += part[(int64_t)v * nch + c].im;
    }
    const cplx t = block_sum(mk(ar, ai));
    if (threadIdx.x == 0) out[(int64_t)v * n_inst + k] = t;
}

// ---------------------------------------------------------------------------------------------
// Leaf evaluation.  k_near: the log parts of the U list; k_near_reaction: the reaction part of the
// U list's image entries, for the targets whose leaf has them; k_leaf: L2P of the local(s) plus
// the near-field sums and the surface term; k_leaf_w: the rarer W list (M2P).
//
// Each kernel has three modes: kPhi (the potential, in caller order), kGrad (the gradient
// (d_x phi, d_y phi) only) and kPhiGrad (both); the near-field kernels have a fourth, kDip, the
// double-layer potential of dipole sources (density q_j, normal n_j): the same sums with each
// pair's kernel replaced by its derivative along the source normal,
//   n . grad' (s/2pi) log|r - r'| = (s/2pi) (-n_x dx + t n_y dy) / r^2   (dx = x - x', dy = y + t y',
//   t = -1 free, +1 image), and n . grad' I_0(X, Y) = -i conj(nu) I_1(X, Y), n . grad' I_0(-X, Y) =
//   i nu I_1(-X, Y), nu = n_x + i n_y.  Gradients follow from the same expansions: the
// far field is 2 Re H + surface (real impedance) or H + conj(G) with H, G holomorphic in the
// target z, so d_x = 2 Re H', d_y = -2 Im H' (resp. d_x = H' + conj(G'), d_y = i H' - i conj(G'));
// the surface term i e^{-Z(y + ix)} s has d_x = Z e^{-Z(y+ix)} s and d_y = -i Z e^{-Z(y+ix)} s.
// Near-field kernel derivatives: d_x log|r - r'| = (x - x') / |r - r'|^2 (and alike in y), and
// d_x I_0(X, Y) = i I_1(X, Y), d_y I_0(X, Y) = -I_1(X, Y), I_1 = 1 / (2 pi w) + Z I_0, w = Y - iX
// (differentiating eq. (generalintegral) under the integral; eq. (integralrecursion) for n = 1).
// ---------------------------------------------------------------------------------------------
enum LeafMode { kPhi = 0, kGrad = 1, kPhiGrad = 2, kDip = 3 };
__host__ __device__ constexpr bool has_phi(int m) { return m != kGrad; }
__host__ __device__ constexpr bool has_grad(int m) { return m == kGrad || m == kPhiGrad; }
__host__ __device__ constexpr bool is_dip(int m) { return m == kDip; }

struct LeafArgs {
    const InstInfo *ii;      // [n_inst]
    const int32_t *inst;     // box -> instance
    int n_inst;
    int nv;                  // charge vectors in this pass (interleaved in qs)
    int64_t n;
    int nbox, nloc;
    const double *xs, *ys, *qs;
    const double2 *xy;
    const int32_t *perm, *leaf_of, *level, *bx, *by, *first, *count;
    const int32_t *uoff, *uent, *woff, *went;
    const cplx *W, *Lam;
    const double *invfact, *fact;
    const cplx *rank1;       // [nv][n_inst] surface sums (real impedance) or null
    const int32_t *wpts;     // targets whose leaf has a W list
    int64_t n_wpts;
    const int32_t *rpts;     // targets whose leaf has image U entries
    const double2 *logtab;   // [kLogTable] (1/c_k, -log(1/c_k))
    double2 *near;           // [nv][n] near-field potential per sorted target
    cplx *near_gx, *near_gy; // [n] near-field gradient per sorted target (gradient modes)
    double *qc;              // [n] sum of the charges coincident with each sorted target, or null
    double *phi;             // [nv][n][2] potential, caller order (potential modes)
    cplx *gx, *gy;           // [n] gradient, caller order (gradient modes)
    const int2 *u2;          // per U entry: (first point, point count | image << 31) of its source box
    double isg;              // sign of the image log term: +1 (Robin, Dirichlet), -1 (Neumann)
    const double2 *nrm;      // [n] source normals (sorted order), kDip only
    int sorted_out;          // phi, gx, gy in sorted order instead (outputs an internal pass reads)
};

// The hardware places workgroup b on XCD b % 8, and each XCD has its own L2.  xcd_chunks gives a
// grid-stride loop over nch chunks whose workgroups on one XCD walk one contiguous range of chunks
// (XCD x holds the x-th eighth), so that the workgroups sharing an L2 work on neighbouring leaves,
// whose U lists share source points.  Every chunk is taken exactly once for any grid size.
constexpr int kXcds = 8;
struct XcdChunks {
    int64_t c0, c1;  // this workgroup's first chunk, end of its XCD's range
    int step;        // workgroups on this XCD
};
__device__ __forceinline__ XcdChunks xcd_chunks(int64_t nch) {
    const int G = gridDim.x, X = G < kXcds ? G : kXcds;
    const int x = blockIdx.x % X;
    const int64_t base = nch / X, rem = nch % X;
    XcdChunks r;
    r.step = G / X + (x < G % X ? 1 : 0);
    r.c0 = x * base + (x < rem ? x : rem) + blockIdx.x / X;
    r.c1 = (x + 1) * base + (x + 1 < rem ? x + 1 : rem);
    return r;
}

// Near field, log terms of the U list: one thread per target (sorted order; workgroups take chunks
// of blockDim targets by xcd_chunks).  NV charge vectors share each pair's kernel value.  The
// thread loads each source point (and the next U entry's range) one step ahead of its use, so that
// the memory latency overlaps the arithmetic; free-space and image terms go into one signed sum,
// (1/4 pi) sum_j q_j (log r_img^2 - log r^2).
template <int MODE, int NV>
__global__ __launch_bounds__(256) void k_near(LeafArgs a) {
    __shared__ double2 s_logtab[kLogTable];
    if (has_phi(MODE)) {
        for (int k = threadIdx.x; k < kLogTable; k += blockDim.x) s_logtab[k] = a.logtab[k];
        __syncthreads();
    }
    const double2 *__restrict__ xy = a.xy;
    const double2 *__restrict__ tab = s_logtab;
    const double *__restrict__ qs = a.qs;
    const int2 *__restrict__ u2 = a.u2;
    const XcdChunks ch = xcd_chunks((a.n + blockDim.x - 1) / blockDim.x);
    for (int64_t c = ch.c0; c < ch.c1; c += ch.step) {
        const int64_t i = c * blockDim.x + threadIdx.x;
        if (i >= a.n) break;
        const int b = a.leaf_of[i];
        const double2 pi = a.xy[i];
        const double x = pi.x, y = pi.y;
        double acc[NV], gxa[NV], gya[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = gxa[v] = gya[v] = 0.0;
        double qc = 0.0;  // coincident charge of vector 0
        // a leaf's U list holds at least the leaf itself, and every listed box holds a point
        int e = a.uoff[b];
        const int e1 = a.uoff[b + 1];
        int2 fc = u2[e];
        int2 fn = e + 1 < e1 ? u2[e + 1] : fc;  // range of entry e + 1
        double2 pj = xy[fc.x];
        double2 nj = is_dip(MODE) ? a.nrm[fc.x] : make_double2(0.0, 0.0);
        double qj[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) qj[v] = qs[(int64_t)fc.x * NV + v];
        while (true) {
            const int j0 = fc.x, jend = fc.x + (fc.y & 0x7fffffff);
            const double ysg = fc.y < 0 ? 1.0 : -1.0;   // image: y + y', free: y - y'
            const double sg = fc.y < 0 ? a.isg : -1.0;  // image: +-log|r - r_img|, free: - log|r - r'|
            const bool last = e + 1 >= e1;
            const int jnext = last ? jend - 1 : fn.x;  // the point loaded after this entry's last
            double ea[NV];  // this entry's sum, its sign applied once after the loop
#pragma unroll
            for (int v = 0; v < NV; ++v) ea[v] = 0.0;
#pragma unroll 2
            for (int j = j0; j < jend; ++j) {
                const int jp = j + 1 < jend ? j + 1 : jnext;
                const double2 pn = xy[jp];
                const double2 nn = is_dip(MODE) ? a.nrm[jp] : make_double2(0.0, 0.0);
                double qn[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) qn[v] = qs[(int64_t)jp * NV + v];
                const double dx = x - pj.x, dy = fma(ysg, pj.y, y);  // y - y' or y + y'
                const double r2 = fma(dx, dx, dy * dy);
                // r2 = 0 only for a coincident free pair, skipped (eq. (1.2)), or between two
                // target-only points on y = 0 (no charge); image distances to sources are positive
                const bool nz = r2 > 0.0;
                if (is_dip(MODE)) {
                    const double kv = nz ? rcp_pos(nz ? r2 : 1.0) * fma(ysg * nj.y, dy, -nj.x * dx) : 0.0;
#pragma unroll
                    for (int v = 0; v < NV; ++v) ea[v] = fma(qj[v], kv, ea[v]);
                } else if (has_phi(MODE)) {
                    const double lg = log_tab(r2, tab);  // finite for r2 = 0, masked below
#pragma unroll
                    for (int v = 0; v < NV; ++v) ea[v] = fma(qj[v], nz ? lg : 0.0, ea[v]);
                }
                if (has_grad(MODE)) {
                    const double sr = sg * rcp_pos(nz ? r2 : 1.0);
                    const double irx = nz ? sr * dx : 0.0, iry = nz ? sr * dy : 0.0;
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        gxa[v] = fma(qj[v], irx, gxa[v]);
                        gya[v] = fma(qj[v], iry, gya[v]);
                    }
                    qc += nz ? 0.0 : qj[0];
                }
                pj = pn;
                nj = nn;
#pragma unroll
                for (int v = 0; v < NV; ++v) qj[v] = qn[v];
            }
            if (has_phi(MODE)) {
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] = fma(sg, ea[v], acc[v]);
            }
            if (last) break;
            ++e;
            fc = fn;
            if (e + 1 < e1) fn = u2[e + 1];
        }
        if (has_phi(MODE)) {
            constexpr double kc = is_dip(MODE) ? kInv2Pi : kInv4Pi;
#pragma unroll
            for (int v = 0; v < NV; ++v) a.near[(int64_t)v * a.n + i] = make_double2(kc * acc[v], 0.0);
        }
        if (has_grad(MODE)) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                a.near_gx[(int64_t)v * a.n + i] = mk(kInv2Pi * gxa[v], 0.0);
                a.near_gy[(int64_t)v * a.n + i] = mk(kInv2Pi * gya[v], 0.0);
            }
            if (a.qc) a.qc[i] = qc;
        }
    }
}

// Near field, log terms, symmetric leaf-pair walk (near_walk 3; potential only).  The log kernel of
// a pair is symmetric in its two points, for the free-space term log|r - r'| and for the image term
// log|r - conj r'| = log|r' - conj r| alike, and the U lists are symmetric (B, or its mirror image, is
// listed for leaf A exactly when A, or its mirror image, is listed for B).  So each cross pair of
// leaves (A, B), B > A, is evaluated once, by the wave of A (a leaf of more than 64 points is split
// into records of 64 targets, each with partial slots of its own): lane (i, g) holds target i and
// takes every G-th point of B; the row sums (B's charges) accumulate in the lanes, the column sums
// (A's charges, for B's targets) are reduced over the lanes of a group by DPP lane moves and written
// to a partial-sum slot of the pair.  The self pair (A, A) and the self-image pair (A, A_img) give row sums only.  A
// second kernel adds the partials to B's targets in a fixed order (pairs in ascending A), so the
// result is reproducible.
struct SymArgs {
    int nrec;
    const int4 *rec;          // [nrec] (first target point, targets (<= 64), first job, end of jobs)
    const int4 *jobs;         // (first point of B, count | image << 31, partial offset or -1, 0)
    const double2 *xy;
    const double *qs;         // [n][NV]
    const double2 *logtab;
    double isg;               // sign of the image log term
    double *part;             // [partial entries][NV]
    double2 *near;            // [NV][n]
    int64_t n;
};


// Sum over aligned groups of TP lanes (TP = 8, 16, 32, 64).  Lanes [8k, 8k + 8) and rows of 16 are
// reduced by quad swaps (xor 1, xor 2), the half-row mirror and the row mirror, after which every
// lane of a row holds its sum; for TP = 32 row 2k + 1 adds row 2k's sum (row broadcast of lane 15),
// for TP = 64 row 3 adds lane 31's (row broadcast of lane 31).  The group's sum is complete in
// lane sum_lane(TP) of the group (and, for TP <= 16, in all of its lanes).
__device__ __forceinline__ int sum_lane(int TP) { return TP == 64 ? 48 : TP == 32 ? 16 : 0; }
__device__ __forceinline__ double group_sum(double s, int TP) {
    s += dpp_move<0xB1, 0xF>(s);   // quad_perm [1, 0, 3, 2]
    s += dpp_move<0x4E, 0xF>(s);   // quad_perm [2, 3, 0, 1]
    s += dpp_move<0x141, 0xF>(s);  // row_half_mirror
    if (TP >= 16) s += dpp_move<0x140, 0xF>(s);  // row_mirror
    if (TP >= 32) s += dpp_move<0x142, 0xA>(s);  // row_bcast:15 into rows 1 and 3
    if (TP >= 64) s += dpp_move<0x143, 0x8>(s);  // row_bcast:31 into row 3
    return s;
}

// One wave per record (a leaf, or 64 of its targets).  Within a record, the jobs' source steps form
// one stream: the next step's source point (across job boundaries) and the job after the next are
// loaded ahead of the current step's arithmetic.
template <int NV>
__global__ __launch_bounds__(256) void k_near_sym(SymArgs a) {
    __shared__ double2 s_logtab[kLogTable];
    for (int k = threadIdx.x; k < kLogTable; k += blockDim.x) s_logtab[k] = a.logtab[k];
    __syncthreads();
    const double2 *__restrict__ tab = s_logtab;
    const double2 *__restrict__ xy = a.xy;
    const double *__restrict__ qs = a.qs;
    const int4 *__restrict__ jobs = a.jobs;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const XcdChunks ch = xcd_chunks((a.nrec + 3) / 4);  // four records (one per wave) per chunk
    for (int64_t c = ch.c0; c < ch.c1; c += ch.step) {
        const int ri = (int)(c * 4 + wave);
        if (ri >= a.nrec) continue;
        const int4 rc = a.rec[ri];
        const int ft = rc.x, nt = rc.y, e0 = rc.z, e1 = rc.w;
        // lanes per target group: the targets rounded up to a power of two
        const int TP = nt <= 8 ? 8 : nt <= 16 ? 16 : nt <= 32 ? 32 : 64;
        const int G = 64 / TP;
        const int i = lane & (TP - 1), g = lane / TP;
        const bool act = i < nt;
        const int wl = sum_lane(TP);  // the lane of a group that holds its column sums
        const int64_t pi = ft + (act ? i : 0);
        const double2 P = xy[pi];
        double qi[NV], R[NV], ea[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            qi[v] = act ? qs[pi * NV + v] : 0.0;
            R[v] = ea[v] = 0.0;
        }
        int e = e0;
        int4 jb = jobs[e];
        int4 jn = e + 1 < e1 ? jobs[e + 1] : jb;
        int jj = 0;
        int bcount = jb.y & 0x7fffffff;
        int j = g;
        bool vj = j < bcount;
        double2 Q = xy[jb.x + (vj ? j : 0)];
        double qj[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) qj[v] = vj ? qs[(int64_t)(jb.x + j) * NV + v] : 0.0;
        while (true) {
            // the next step: the same job's next G sources, or the next job's first ones
            int njj = jj + G, ne = e;
            int4 nb = jb;
            const bool switch_job = njj >= bcount;
            if (switch_job) {
                ne = e + 1;
                njj = 0;
                nb = jn;
            }
            const bool more = ne < e1;
            const int ncount = nb.y & 0x7fffffff;
            const int jnx = njj + g;
            const bool vn = more && jnx < ncount;
            const int64_t pn = nb.x + (vn ? jnx : 0);
            const double2 Qn = xy[pn];
            double qn[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) qn[v] = vn ? qs[pn * NV + v] : 0.0;
            // this step
            const double ysg = jb.y < 0 ? 1.0 : -1.0;   // image: y + y', free: y - y'
            const double dx = P.x - Q.x, dy = fma(ysg, Q.y, P.y);
            const double r2 = fma(dx, dx, dy * dy);
            // r2 = 0 only for a coincident free pair, skipped (eq. (1.2)), or between two target-only
            // points on y = 0 (no charge)
            const double lg = log_tab(r2, tab);
            const double K = r2 > 0.0 ? lg : 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) ea[v] = fma(qj[v], K, ea[v]);
            const double sg = jb.y < 0 ? a.isg : -1.0;  // image: +-log|r - r_img|, free: - log|r - r'|
            if (jb.z >= 0) {
                double cv[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) cv[v] = group_sum(qi[v] * K, TP);
                if (i == wl && vj) {
                    double *dst = a.part + ((int64_t)jb.z + j) * NV;
#pragma unroll
                    for (int v = 0; v < NV; ++v) dst[v] = sg * cv[v];
                }
            }
            if (switch_job) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    R[v] = fma(sg, ea[v], R[v]);
                    ea[v] = 0.0;
                }
                if (!more) break;
                e = ne;
                jb = jn;
                jn = e + 1 < e1 ? jobs[e + 1] : jb;
                bcount = ncount;
            }
            jj = njj;
            j = jnx;
            vj = vn;
            Q = Qn;
#pragma unroll
            for (int v = 0; v < NV; ++v) qj[v] = qn[v];
        }
        // the G groups of a target hold parts of its row sum
        for (int off = TP; off < 64; off <<= 1) {
#pragma unroll
            for (int v = 0; v < NV; ++v) R[v] += __shfl_xor(R[v], off);
        }
        if (g == 0 && act) {
#pragma unroll
            for (int v = 0; v < NV; ++v) a.near[(int64_t)v * a.n + ft + i] = make_double2(kInv4Pi * R[v], 0.0);
        }
    }
}

// Near field, log terms, symmetric leaf pairs with the pairs blocked in registers (near_walk 4;
// potential passes).  The records, jobs and partial slots are those of walk 3.  A record's lanes form
// IA target groups (consecutive lanes) by JG = 64 / IA source groups, IA the smallest power of two
// with IA * kBlkTargets >= the record's targets: lane (ig, jg) holds the targets ig, ig + IA, ...
// (at most kBlkTargets, in registers) and takes the source points jg, jg + JG, ... of the record's
// job stream (the points of its jobs one after another, a step may span several jobs).  Each pair
// adds to the lane's row sums (the charges of the source point, with the job's sign); for a cross
// pair the column sum over the lane's targets is reduced over the IA lanes of the source group by
// DPP lane moves (none when IA = 1) and written to the pair's partial slot.  The row sums of a
// target are reduced over its JG lanes once per record.
constexpr int kBlkTargets = 8;


// One record with TI targets per lane (compile-time, so that a step's TI pair evaluations are
// straight-line code whose table loads issue together).
template <int NV, int TI>
__device__ __forceinline__ void near_blk_record(const SymArgs &a, const double2 *__restrict__ tab, int lane, int ft,
                                                int nt, int e0, int e1, int IA) {
    const double2 *__restrict__ xy = a.xy;
    const double *__restrict__ qs = a.qs;
    const int4 *__restrict__ jobs = a.jobs;
    const int JG = 64 / IA;
    const int ig = lane & (IA - 1), jg = lane / IA;
    double tx[TI], ty[TI], tq[TI][NV], R[TI][NV];
#pragma unroll
    for (int k = 0; k < TI; ++k) {
        const int i = ig + IA * k;
        const bool act = i < nt;
        const double2 P = xy[ft + (act ? i : 0)];
        tx[k] = P.x;
        ty[k] = P.y;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            tq[k][v] = act ? qs[(int64_t)(ft + i) * NV + v] : 0.0;
            R[k][v] = 0.0;
        }
    }
    int tot = 0;  // points in the record's job stream
    for (int e = e0; e < e1; ++e) tot += jobs[e].y & 0x7fffffff;
    // the lane's job: index, stream position of its first point, the job itself
    int e = e0, js = 0;
    int4 jb = jobs[e0];
    for (int p0 = 0; p0 < tot; p0 += JG) {
        const int p = p0 + jg;
        const bool valid = p < tot;
        while (valid && p >= js + (jb.y & 0x7fffffff)) {
            js += jb.y & 0x7fffffff;
            jb = jobs[++e];
        }
        const int j = jb.x + (valid ? p - js : 0);
        const bool img = jb.y < 0;
        const double ysg = img ? 1.0 : -1.0;    // image: y + y', free: y - y'
        const double sg = img ? a.isg : -1.0;  // image: +-log|r - r_img|, free: - log|r - r'|
        const double2 Q = xy[j];
        double qj[NV], cs[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            qj[v] = valid ? sg * qs[(int64_t)j * NV + v] : 0.0;
            cs[v] = 0.0;
        }
        double K[TI];
#pragma unroll
        for (int k = 0; k < TI; ++k) {
            const double dx = tx[k] - Q.x, dy = fma(ysg, Q.y, ty[k]);
            const double r2 = fma(dx, dx, dy * dy);
            // r2 = 0 only for a coincident free pair, skipped (eq. (1.2)), or between two target-only
            // points on y = 0 (no charge)
            const double lg = log_tab(r2, tab);
            K[k] = r2 > 0.0 ? lg : 0.0;
        }
#pragma unroll
        for (int k = 0; k < TI; ++k)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                R[k][v] = fma(qj[v], K[k], R[k][v]);
                cs[v] = fma(tq[k][v], K[k], cs[v]);
            }
        // the source group's column sums (all IA lanes share p, hence the job)
#pragma unroll
        for (int v = 0; v < NV; ++v) cs[v] = lane_group_sum(cs[v], IA);
        if (valid && ig == 0 && jb.z >= 0) {
            double *dst = a.part + ((int64_t)jb.z + (p - js)) * NV;
#pragma unroll
            for (int v = 0; v < NV; ++v) dst[v] = sg * cs[v];
        }
    }
    // a target's row sum is spread over its JG lanes (stride IA)
    for (int off = IA; off < 64; off <<= 1) {
#pragma unroll
        for (int k = 0; k < TI; ++k)
#pragma unroll
            for (int v = 0; v < NV; ++v) R[k][v] += __shfl_xor(R[k][v], off);
    }
    if (jg == 0) {
#pragma unroll
        for (int k = 0; k < TI; ++k) {
            const int i = ig + IA * k;
            if (i < nt) {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    a.near[(int64_t)v * a.n + ft + i] = make_double2(kInv4Pi * R[k][v], 0.0);
            }
        }
    }
}

template <int NV>
__global__ __launch_bounds__(256, 4) void k_near_blk(SymArgs a) {
    constexpr int TM = kBlkTargets;
    static_assert(TM == 8, "the dispatch below covers 1..8 targets per lane");
    __shared__ double2 s_logtab[kLogTable];
    for (int k = threadIdx.x; k < kLogTable; k += blockDim.x) s_logtab[k] = a.logtab[k];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const XcdChunks ch = xcd_chunks((a.nrec + 3) / 4);  // four records (one per wave) per chunk
    for (int64_t c = ch.c0; c < ch.c1; c += ch.step) {
        const int ri = (int)(c * 4 + wave);
        if (ri >= a.nrec) continue;
        const int4 rc = a.rec[ri];
        const int ft = rc.x, nt = rc.y, e0 = rc.z, e1 = rc.w;
        const int IA = nt <= TM ? 1 : nt <= 2 * TM ? 2 : nt <= 4 * TM ? 4 : 8;
        switch ((nt + IA - 1) / IA) {  // targets of lane group 0 (the others hold as many or one fewer)
        case 1: near_blk_record<NV, 1>(a, s_logtab, lane, ft, nt, e0, e1, IA); break;
        case 2: near_blk_record<NV, 2>(a, s_logtab, lane, ft, nt, e0, e1, IA); break;
        case 3: near_blk_record<NV, 3>(a, s_logtab, lane, ft, nt, e0, e1, IA); break;
        case 4: near_blk_record<NV, 4>(a, s_logtab, lane, ft, nt, e0, e1, IA); break;
        case 5: near_blk_record<NV, 5>(a, s_logtab, lane, ft, nt, e0, e1, IA); break;
        case 6: near_blk_record<NV, 6>(a, s_logtab, lane, ft, nt, e0, e1, IA); break;
        case 7: near_blk_record<NV, 7>(a, s_logtab, lane, ft, nt, e0, e1, IA); break;
        default: near_blk_record<NV, 8>(a, s_logtab, lane, ft, nt, e0, e1, IA); break;
        }
    }
}

// Adds the column sums of the cross pairs (A, B), A < B, to B's targets, pairs in ascending A.
template <int NV>
__global__ __launch_bounds__(256) void k_near_gather(int64_t n, const int32_t *__restrict__ leaf_of,
                                                     const int32_t *__restrict__ first,
                                                     const int32_t *__restrict__ in_off,
                                                     const int32_t *__restrict__ in_ent,
                                                     const double *__restrict__ part, double2 *__restrict__ near) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int B = leaf_of[i];
    const int e0 = in_off[B], e1 = in_off[B + 1];
    if (e1 == e0) return;
    const int jb = (int)(i - first[B]);
    double sv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) sv[v] = 0.0;
    for (int e = e0; e < e1; ++e) {
        const double *src = part + ((int64_t)in_ent[e] + jb) * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) sv[v] += src[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) near[(int64_t)v * n + i].x += kInv4Pi * sv[v];
}

// The same sums with a plain walk: the U list entry by entry, a source point loaded where it is
// used (fewer instructions per pair; the memory latency is hidden by other waves only), free-space
// and image terms in separate sums.
template <int MODE, int NV>
__global__ __launch_bounds__(256) void k_near_plain(LeafArgs a) {
    __shared__ double2 s_logtab[kLogTable];
    if (has_phi(MODE)) {
        for (int k = threadIdx.x; k < kLogTable; k += blockDim.x) s_logtab[k] = a.logtab[k];
        __syncthreads();
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x) {
        const int b = a.leaf_of[i];
        const double2 pi = a.xy[i];
        const double x = pi.x, y = pi.y;
        double lfree[NV], limg[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) lfree[v] = limg[v] = 0.0;
        double fx[NV], fy[NV], mx[NV], my[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) fx[v] = fy[v] = mx[v] = my[v] = 0.0;
        double qc = 0.0;  // coincident charge of vector 0
        const double2 *__restrict__ xy = a.xy;
        const double2 *__restrict__ tab = s_logtab;
        const double *__restrict__ qs = a.qs;
        for (int e = a.uoff[b]; e < a.uoff[b + 1]; ++e) {
            const int code = a.uent[e];
            const int c = code >> 1;
            const int j0 = a.first[c], j1 = j0 + a.count[c];
            if (!(code & 1)) {
                for (int j = j0; j < j1; ++j) {
                    const double2 pj = xy[j];
                    const double dx = x - pj.x, dy = y - pj.y;
                    const double r2 = fma(dx, dx, dy * dy);
                    const bool nz = r2 > 0.0;  // skip the self pair (eq. (1.2))
                    if (is_dip(MODE)) {
                        const double2 nj = a.nrm[j];
                        const double kv = nz ? -rcp_pos(nz ? r2 : 1.0) * fma(nj.x, dx, nj.y * dy) : 0.0;
#pragma unroll
                        for (int v = 0; v < NV; ++v) lfree[v] = fma(qs[(int64_t)j * NV + v], kv, lfree[v]);
                    } else if (has_phi(MODE)) {
                        const double lg = nz ? log_tab(nz ? r2 : 1.0, tab) : 0.0;
#pragma unroll
                        for (int v = 0; v < NV; ++v) lfree[v] = fma(qs[(int64_t)j * NV + v], lg, lfree[v]);
                    }
                    if (has_grad(MODE)) {
                        const double ir = nz ? rcp_pos(nz ? r2 : 1.0) : 0.0;
                        const double irx = ir * dx, iry = ir * dy;
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            const double qj = qs[(int64_t)j * NV + v];
                            fx[v] = fma(qj, irx, fx[v]);
                            fy[v] = fma(qj, iry, fy[v]);
                        }
                        qc += nz ? 0.0 : qs[(int64_t)j * NV];
                    }
                }
            } else {
                for (int j = j0; j < j1; ++j) {
                    const double2 pj = xy[j];
                    const double dx = x - pj.x, dy = y + pj.y;
                    const double r2 = fma(dx, dx, dy * dy);
                    // r2 = 0 only between two target-only points on y = 0 (no charge): skipped
                    const bool nz = r2 > 0.0;
                    if (is_dip(MODE)) {
                        const double2 nj = a.nrm[j];
                        const double kv = nz ? rcp_pos(nz ? r2 : 1.0) * fma(nj.y, dy, -nj.x * dx) : 0.0;
#pragma unroll
                        for (int v = 0; v < NV; ++v) limg[v] = fma(qs[(int64_t)j * NV + v], kv, limg[v]);
                    } else if (has_phi(MODE)) {
                        const double lg = nz ? log_tab(nz ? r2 : 1.0, tab) : 0.0;
#pragma unroll
                        for (int v = 0; v < NV; ++v) limg[v] = fma(qs[(int64_t)j * NV + v], lg, limg[v]);
                    }
                    if (has_grad(MODE)) {
                        const double ir = nz ? rcp_pos(nz ? r2 : 1.0) : 0.0;
                        const double irx = ir * dx, iry = ir * dy;
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            const double qj = qs[(int64_t)j * NV + v];
                            mx[v] = fma(qj, irx, mx[v]);
                            my[v] = fma(qj, iry, my[v]);
                        }
                    }
                }
            }
        }
        if (has_phi(MODE)) {
            constexpr double kc = is_dip(MODE) ? kInv2Pi : kInv4Pi;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                a.near[(int64_t)v * a.n + i] = make_double2(kc * (a.isg * limg[v] - lfree[v]), 0.0);
        }
        if (has_grad(MODE)) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                a.near_gx[(int64_t)v * a.n + i] = mk(kInv2Pi * (a.isg * mx[v] - fx[v]), 0.0);
                a.near_gy[(int64_t)v * a.n + i] = mk(kInv2Pi * (a.isg * my[v] - fy[v]), 0.0);
            }
            if (a.qc) a.qc[i] = qc;
        }
    }
}

// L2P of the local(s), plus the near-field sums and the surface term; writes caller order (sorted
// order for a pass whose outputs only the adjoint's combination reads).
template <int PB, int MODE>
__global__ __launch_bounds__(256) void k_leaf(LeafArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int v = blockIdx.y;  // charge vector
    const int b = a.leaf_of[i];
    const int l = a.level[b];
    const int k = a.inst[b];
    const Geo g = geo_of(a.ii, k);
    const cplx Zk = a.ii[k].Z;
    const double x = a.xs[i], y = a.ys[i];
    const cplx cb = centre_of(g, l, a.bx[b], a.by[b]);
    const double irho = 2.0 / side_of(g, l);
    // L2P: H(z) = sum_n lambda_n / n! zeta^n, H'(z) = irho sum_{n>=1} lambda_n / (n-1)! zeta^(n-1)
    const cplx zeta = mk((x - cb.re) * irho, (y - cb.im) * irho);
    cplx H = mk(0.0, 0.0), G = mk(0.0, 0.0), Hd = mk(0.0, 0.0), Gd = mk(0.0, 0.0);
    for (int loc = 0; loc < a.nloc; ++loc) {
        const cplx *L = a.Lam + ((int64_t)v * a.nloc + loc) * (PB + 1) * a.nbox + b;
        cplx h = mk(0.0, 0.0), hd = mk(0.0, 0.0);
#pragma unroll
        for (int n = PB; n >= 0; --n) {
            const cplx ln = L[(int64_t)n * a.nbox];
            if (has_phi(MODE)) {
                cplx t = ln * a.invfact[n];
                cfma(t, h, zeta);
                h = t;
            }
            if (has_grad(MODE) && n >= 1) {
                cplx t = ln * a.invfact[n - 1];
                cfma(t, hd, zeta);
                hd = t;
            }
        }
        if (loc == 0) {
            H = h;
            Hd = irho * hd;
        } else {
            G = h;
            Gd = irho * hd;
        }
    }
    const int64_t o = a.sorted_out ? i : a.perm[i];
    cplx E = mk(0.0, 0.0);  // e^{-Z(y + ix)} s (real impedance)
    if (a.nloc == 1 && a.rank1) E = cexp_(-(Zk * mk(y, x))) * a.rank1[(int64_t)v * a.n_inst + k];
    if (has_phi(MODE)) {
        const double2 nr = a.near[(int64_t)v * a.n + i];
        cplx phi;
        if (a.nloc == 1) phi = mk(2.0 * H.re + nr.x, nr.y) + mul_ipow(E, 1);
        else phi = H + conj(G) + mk(nr.x, nr.y);
        double *out = a.phi + (int64_t)v * 2 * a.n;
        out[2 * o] = phi.re;
        out[2 * o + 1] = phi.im;
    }
    if (has_grad(MODE)) {
        cplx gx = a.near_gx[(int64_t)v * a.n + i], gy = a.near_gy[(int64_t)v * a.n + i];
        if (a.nloc == 1) {
            const cplx ZE = Zk * E;
            gx += mk(2.0 * Hd.re, 0.0) + ZE;
            gy += mk(-2.0 * Hd.im, 0.0) + mul_ipow(ZE, 3);
        } else {
            gx += Hd + conj(Gd);
            gy += mul_ipow(Hd - conj(Gd), 1);
        }
        a.gx[(int64_t)v * a.n + o] = gx;
        a.gy[(int64_t)v * a.n + o] = gy;
    }
}

// Steps of the W-list evaluation below: term k of the log-kernel multipole (powers of tau) and
// term n of the reaction ME (the I_n recursion), for every vector of the pass.
template <int MODE, int NV>
__device__ __forceinline__ void leafw_log_step(const LeafArgs &a, int64_t vstride, int d, int img, int k, cplx &pw,
                                               const cplx &tau, cplx (&u)[NV], cplx (&ud)[NV]) {
    const double fk1 = a.fact[k - 1], fk = a.fact[k];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        cplx wk = a.W[(int64_t)v * vstride + (int64_t)k * a.nbox + d];
        if (img) wk = conj(wk);
        const cplx pk = pw * wk;
        if (has_phi(MODE)) u[v] -= fk1 * pk;
        if (has_grad(MODE)) ud[v] += fk * pk;
    }
    pw = pw * tau;
}

template <int PB, int MODE, int NV>
__device__ __forceinline__ void leafw_react_step(const LeafArgs &a, int64_t vstride, int d, int pass, int n,
                                                 const cplx &sw, const cplx &zr, cplx &F, cplx &K, cplx (&acc)[NV],
                                                 cplx (&accd)[NV]) {
    F = F * sw * (n > 1 ? (double)(n - 1) : 1.0);
    K = F * kInv2Pi + zr * K;
    const cplx Kn = mul_ipow(pass == 0 ? K : conj(K), n);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const cplx *Wv = a.W + (int64_t)v * vstride;
        if (has_phi(MODE) && n <= PB) acc[v] += Kn * conj(Wv[(int64_t)n * a.nbox + d]);
        if (has_grad(MODE)) accd[v] += Kn * conj(Wv[(int64_t)(n - 1) * a.nbox + d]);
    }
}

// W list for the targets whose leaf has one: multipoles of smaller non-adjacent boxes evaluated
// at the target (log kernel, and the paper's reaction ME for image boxes).  Adds to the near-field
// sums (before k_leaf reads them).
template <int PB, int MODE, int NV>
__global__ __launch_bounds__(128) void k_leaf_w(LeafArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n_wpts) return;
    // one thread per target, every charge vector of the pass: the geometric factors (powers of
    // tau, the logarithm, the reaction integrals) are computed once for all vectors
    const int64_t vstride = (int64_t)(PB + 1) * a.nbox;
    const int64_t i = a.wpts[t];
    const int b = a.leaf_of[i];
    const Geo g = geo_of(a.ii, a.inst[b]);
    const cplx Zk = a.ii[a.inst[b]].Z;
    const double x = a.xs[i], y = a.ys[i];
    const cplx z = mk(x, y);
    cplx H[NV], G[NV], Hd[NV], Gd[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) H[v] = G[v] = Hd[v] = Gd[v] = mk(0.0, 0.0);
    for (int e = a.woff[b]; e < a.woff[b + 1]; ++e) {
        const int code = a.went[e];
        const int d = code >> 1, img = code & 1;
        const int ld = a.level[d];
        const cplx cd0 = centre_of(g, ld, a.bx[d], a.by[d]);
        const double rd = 0.5 * side_of(g, ld);
        const cplx cd = img ? conj(cd0) : cd0;
        const cplx dz = z - cd;
        const cplx idz = inv(dz);
        const cplx tau = -rd * idz;
        // u = w0 log(z - c) - sum_k (k-1)! tau^k w_k,  u' = (w0 + sum_k k! tau^k w_k) / (z - c)
        // (conjugated w for the image box)
        const cplx lg = has_phi(MODE) ? clog_(dz) : mk(0.0, 0.0);
        cplx u[NV], ud[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            cplx w0 = a.W[(int64_t)v * vstride + d];
            if (img) w0 = conj(w0);
            u[v] = has_phi(MODE) ? w0 * lg : mk(0.0, 0.0);
            ud[v] = w0;
        }
        cplx pw = tau;
        // one vector: the k loop unrolled in full; several: the compiler's own choice (unrolling a
        // body that already spans every vector crowds the registers)
        if constexpr (NV == 1) {
#pragma unroll
            for (int k = 1; k <= PB; ++k) leafw_log_step<MODE, NV>(a, vstride, d, img, k, pw, tau, u, ud);
        } else {
            for (int k = 1; k <= PB; ++k) leafw_log_step<MODE, NV>(a, vstride, d, img, k, pw, tau, u, ud);
        }
        const double sgn = (img ? a.ii[a.inst[b]].isg : -1.0) * kInv4Pi;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            H[v] += sgn * u[v];
            G[v] += sgn * u[v];
            const cplx udv = sgn * (ud[v] * idz);
            Hd[v] += udv;
            Gd[v] += udv;
        }
        if (img && a.ii[a.inst[b]].react) {
            // reaction ME (eq. (truncatedME)) of the image box: sum_n alpha_n I_n(x - x'_c, y - y'_c),
            // alpha_n = rho^n (-i)^n conj(mu_n) = i^n n! rho^n conj(w_n); with K_n = n! rho^n I_n its
            // z-derivative is (1/rho) sum_n i^(n+1) K_(n+1) conj(w_n)
            const double X = x - cd0.re, Y = y + cd0.im;
            for (int pass = 0; pass < a.nloc; ++pass) {
                const double Xs = pass == 0 ? X : -X;
                const cplx sw = rd * inv(mk(Y, -Xs));
                const cplx zr = rd * Zk;
                cplx K = reaction_I0_general(Xs, Y, Zk);
                cplx F = mk(1.0, 0.0);
                cplx acc[NV], accd[NV];
                const cplx K0 = pass == 0 ? K : conj(K);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    acc[v] = has_phi(MODE) ? K0 * conj(a.W[(int64_t)v * vstride + d]) : mk(0.0, 0.0);
                    accd[v] = mk(0.0, 0.0);
                }
                constexpr int NTOP = has_grad(MODE) ? PB + 1 : PB;
                if constexpr (NV == 1) {
#pragma unroll
                    for (int n = 1; n <= NTOP; ++n)
                        leafw_react_step<PB, MODE, NV>(a, vstride, d, pass, n, sw, zr, F, K, acc, accd);
                } else {
                    for (int n = 1; n <= NTOP; ++n)
                        leafw_react_step<PB, MODE, NV>(a, vstride, d, pass, n, sw, zr, F, K, acc, accd);
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    if (pass == 0) {
                        H[v] += acc[v];
                        Hd[v] += accd[v] * (1.0 / rd);
                    } else {
                        G[v] += acc[v];
                        Gd[v] += accd[v] * (1.0 / rd);
                    }
                }
            }
        }
    }
    // into the near-field sums of the target (sorted order), which k_leaf adds to the far field
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (has_phi(MODE)) {
            double2 *nr = a.near + (int64_t)v * a.n + i;
            double2 hv = *nr;
            if (a.nloc == 1) {
                hv.x += 2.0 * H[v].re;
            } else {
                const cplx c = H[v] + conj(G[v]);
                hv.x += c.re;
                hv.y += c.im;
            }
            *nr = hv;
        }
        if (has_grad(MODE)) {
            cplx *gx = a.near_gx + (int64_t)v * a.n + i, *gy = a.near_gy + (int64_t)v * a.n + i;
            if (a.nloc == 1) {
                *gx += mk(2.0 * Hd[v].re, 0.0);
                *gy += mk(-2.0 * Hd[v].im, 0.0);
            } else {
                *gx += Hd[v] + conj(Gd[v]);
                *gy += mul_ipow(Hd[v] - conj(Gd[v]), 1);
            }
        }
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Reaction part of the near field: sum over the image sources of a leaf's U list of
// q_j [I_0(X, Y) + I_0(-X, Y)], X = x_i - x_j, Y = y_i + y_j (eq. (reactdecomposition)); for a
// real impedance only 2 Re I_0(X, Y) (the rest is the surface term).  One wave per target whose
// leaf touches y = 0; lanes take image sources, a fixed-order butterfly sums them.  NV charge
// vectors share each pair's kernel value.  Adds to the near-field sums.
template <int MODE, int NV>
__global__ __launch_bounds__(64) void k_near_reaction(LeafArgs a) {
    const int i = a.rpts[blockIdx.x];
    const int b = a.leaf_of[i];
    const cplx Z = a.ii[a.inst[b]].Z;
    const int lane = threadIdx.x;
    const double x = a.xs[i], y = a.ys[i];
    double sr[NV], si[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) sr[v] = si[v] = 0.0;
    cplx s1p[NV], s1m[NV];  // sum q I_1(X, Y), sum q I_1(-X, Y) per vector
#pragma unroll
    for (int v = 0; v < NV; ++v) s1p[v] = s1m[v] = mk(0.0, 0.0);
    for (int e = a.uoff[b]; e < a.uoff[b + 1]; ++e) {
        const int code = a.uent[e];
        if (!(code & 1)) continue;
        const int c = code >> 1;
        const int j1 = a.first[c] + a.count[c];
        for (int j = a.first[c] + lane; j < j1; j += 64) {
            const double dx = x - a.xs[j], dy = y + a.ys[j];
            if (!(dy > 0.0)) continue;  // two target-only points on y = 0 (no charge)
            const cplx I = reaction_I0_near(dx, dy, Z);
            if (is_dip(MODE)) {
                // -i conj(nu) I_1(X, Y) (+ i nu I_1(-X, Y) with a complex impedance)
                const double2 nj = a.nrm[j];
                const cplx I1 = kInv2Pi * inv(mk(dy, -dx)) + Z * I;
                cplx hv = mk(-nj.y, -nj.x) * I1;
                if (a.nloc != 1) {
                    const cplx I1m = kInv2Pi * inv(mk(dy, dx)) + Z * reaction_I0_near(-dx, dy, Z);
                    hv += mk(-nj.y, nj.x) * I1m;
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const double qj = a.qs[(int64_t)j * NV + v];
                    sr[v] += qj * hv.re;
                    si[v] += qj * hv.im;
                }
                continue;
            }
            if (has_grad(MODE)) {
                const cplx I1 = kInv2Pi * inv(mk(dy, -dx)) + Z * I;
#pragma unroll
                for (int v = 0; v < NV; ++v) s1p[v] += a.qs[(int64_t)j * NV + v] * I1;
            }
            if (a.nloc == 1) {
                if (has_phi(MODE)) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) sr[v] += a.qs[(int64_t)j * NV + v] * I.re;
                }
            } else {
                const cplx Im_ = reaction_I0_near(-dx, dy, Z);
                if (has_phi(MODE)) {
                    const cplx hv = I + Im_;
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const double qj = a.qs[(int64_t)j * NV + v];
                        sr[v] += qj * hv.re;
                        si[v] += qj * hv.im;
                    }
                }
                if (has_grad(MODE)) {
                    const cplx I1m = kInv2Pi * inv(mk(dy, dx)) + Z * Im_;
#pragma unroll
                    for (int v = 0; v < NV; ++v) s1m[v] += a.qs[(int64_t)j * NV + v] * I1m;
                }
            }
        }
    }
    if (has_phi(MODE)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            sr[v] = wave_sum(sr[v]);
            si[v] = wave_sum(si[v]);
        }
    }
    if (has_grad(MODE)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            s1p[v] = mk(wave_sum(s1p[v].re), wave_sum(s1p[v].im));
            s1m[v] = mk(wave_sum(s1m[v].re), wave_sum(s1m[v].im));
        }
    }
    if (lane == 0) {
        if (has_phi(MODE)) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double2 *nv_ = a.near + (int64_t)v * a.n + i;
                double2 hv = *nv_;
                if (a.nloc == 1) {
                    hv.x += 2.0 * sr[v];
                } else {
                    hv.x += sr[v];
                    hv.y += si[v];
                }
                *nv_ = hv;
            }
        }
        if (has_grad(MODE)) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                cplx *gx = a.near_gx + (int64_t)v * a.n + i, *gy = a.near_gy + (int64_t)v * a.n + i;
                if (a.nloc == 1) {
                    // d_x 2 Re sum q I_0 = 2 Re(i S1) ; d_y = -2 Re S1
                    *gx += mk(-2.0 * s1p[v].im, 0.0);
                    *gy += mk(-2.0 * s1p[v].re, 0.0);
                } else {
                    *gx += mul_ipow(s1p[v] - s1m[v], 1);
                    *gy -= s1p[v] + s1m[v];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Direct evaluation and reaction integrals (standalone entry points)
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_direct(int64_t ns, const double *__restrict__ sx, const double *__restrict__ sy,
                                                const double *__restrict__ q, int64_t nt,
                                                const double *__restrict__ tx, const double *__restrict__ ty,
                                                cplx Z, double *__restrict__ phi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    const double x = tx[i], y = ty[i];
    double lfree = 0.0, limg = 0.0;
    cplx rc = mk(0.0, 0.0);
    for (int64_t j = 0; j < ns; ++j) {
        const double dx = x - sx[j];
        const double dy = y - sy[j], dyi = y + sy[j];
        const double r2 = dx * dx + dy * dy;
        const double qj = q[j];
        if (r2 > 0.0) lfree += qj * log_pos(r2);
        limg += qj * log_pos(dx * dx + dyi * dyi);
        rc += qj * (reaction_I0_near(dx, dyi, Z) + reaction_I0_near(-dx, dyi, Z));
    }
    const cplx v = mk(kInv4Pi * (limg - lfree), 0.0) + rc;
    phi[2 * i] = v.re;
    phi[2 * i + 1] = v.im;
}

__global__ void k_reaction_integrals(int64_t m, const double *__restrict__ x, const double *__restrict__ y, int nmax,
                                     cplx Z, double *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const double xx = x[k], yy = y[k];
    const cplx w = mk(yy, -xx);
    const cplx iw = inv(w);
    cplx I = reaction_I0(xx, yy, Z);
    out[2 * k * (nmax + 1)] = I.re;
    out[2 * k * (nmax + 1) + 1] = I.im;
    cplx pw = mk(1.0, 0.0);
    for (int n = 1; n <= nmax; ++n) {
        pw = pw * iw;
        I = pw * (kInv2Pi / n) + Z * I * (1.0 / n);
        out[2 * (k * (nmax + 1) + n)] = I.re;
        out[2 * (k * (nmax + 1) + n) + 1] = I.im;
    }
}

fmmhp_status run_direct(int64_t ns, const double *sx, const double *sy, int nvec, const double *q, int64_t nt,
                        const double *tx, const double *ty, cplx Z, double *phi, hipStream_t s) {
    for (int v = 0; v < nvec; ++v) {
        hipLaunchKernelGGL(k_direct, dim3(nblk(nt, 256)), dim3(256), 0, s, ns, sx, sy, q + (int64_t)v * ns, nt, tx, ty,
                           Z, phi + (int64_t)v * 2 * nt);
        FMMHP_HIP(hipGetLastError());
    }
    return FMMHP_OK;
}

fmmhp_status run_reaction_integrals(int64_t m, const double *x, const double *y, int nmax, cplx Z, double *out,
                                    hipStream_t s) {
    hipLaunchKernelGGL(k_reaction_integrals, dim3(nblk(m, 128)), dim3(128), 0, s, m, x, y, nmax, Z, out);
    FMMHP_HIP(hipGetLastError());
    return FMMHP_OK;
}

// ---------------------------------------------------------------------------------------------
// Schedule and tables (host)
// ---------------------------------------------------------------------------------------------
// ---------------------------------------------------------------------------------------------
// Reaction integrals for the M2L tables, on the host in extended precision.  The upward recursion
// of eq. (integralrecursion) amplifies the rounding error of I_0 by up to about
// e^{|P|} / sqrt(2 pi |P|), P = Z (y - i x); at coarse levels |P| reaches ~20 when the impedance is
// large.  The tables are computed once per plan, so they use long double (64-bit significand),
// which keeps the coefficients to ~1e-11 relative up to |P| = 21 and ~1e-10 at the limit of 24.
// I_0 uses the same three regimes as the device routine: the power series of Ei, the asymptotic
// series of e^{-P} E_1(-P) near the positive real axis, and a continued fraction elsewhere.
// ---------------------------------------------------------------------------------------------
using CL = std::complex<long double>;

static CL reaction_I0_ld(long double x, long double y, CL Z) {
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double gamma = 0.577215664901532860606512090082402431L;
    const CL P = Z * CL(y, -x);
    const long double r = std::abs(P);
    const long double ang = std::fabs(std::atan2(P.imag(), P.real()));
    const long double sg = P.imag() > 0 ? 1.0L : (P.imag() < 0 ? -1.0L : 0.0L);
    const long double tiny = 1e-40L;
    CL A;
    if (r <= 2 || (r <= 4 && P.real() >= 0) || (ang <= 0.125L * pi && r <= 50)) {
        CL sum(0, 0), t(1, 0);
        for (int k = 1; k < 600; ++k) {
            t = t * P / (long double)k;
            const CL term = t / (long double)k;
            sum += term;
            if (std::norm(term) < tiny * std::norm(sum)) break;
        }
        const CL ei = gamma + std::log(P) + sum;
        return (std::exp(-P) * CL(-ei.real(), pi - ei.imag())) / (2 * pi);
    }
    if (ang <= 0.125L * pi) {
        const CL ip = 1.0L / P;
        CL t = ip, sum = ip;
        for (int k = 1; k < 400; ++k) {
            const CL tn = t * ip * (long double)k;
            if (std::norm(tn) > std::norm(t)) break;
            sum += tn;
            t = tn;
            if (std::norm(tn) < tiny * std::norm(sum)) break;
        }
        A = -sum;
    } else {
        const CL w = -P;
        CL b = w + 1.0L, c(1e4000L, 0), d = 1.0L / b, h = d;
        for (int i = 1; i < 20000; ++i) {
            const long double a = -(long double)i * (long double)i;
            b += 2.0L;
            d = 1.0L / (a * d + b);
            c = b + a / c;
            const CL del = c * d;
            h *= del;
            if (std::norm(del - 1.0L) < 1e-38L) break;
        }
        A = h;
    }
    return (A + CL(0, 1) * std::exp(-P) * (pi * (1 - sg))) / (2 * pi);
}

// rho^j I_j(x, y) for j = 0..nmax (upward recursion in long double), rounded to double.
static void reaction_In_scaled_ld(double x, double y, cplx Z, double rho, int nmax, cplx *out) {
    const long double pi = 3.141592653589793238462643383279502884L;
    const CL Zl((long double)Z.re, (long double)Z.im);
    const CL sigma = (long double)rho / CL((long double)y, -(long double)x);
    const CL zr = (long double)rho * Zl;
    CL K = reaction_I0_ld(x, y, Zl), sp(1, 0);
    out[0] = mk((double)K.real(), (double)K.imag());
    for (int n = 1; n <= nmax; ++n) {
        sp *= sigma;
        K = sp / (2 * pi * n) + zr * K / (long double)n;
        out[n] = mk((double)K.real(), (double)K.imag());
    }
}

static inline int slot_of(int dx, int dy) { return (dy + 3) * 7 + (dx + 3); }

template <class T>
static fmmhp_status to_dev(Arena &A, T **dst, const std::vector<T> &src, const char *what, hipStream_t s) {
    FMMHP_CHECK(A.alloc_n(dst, src.size(), what));
    if (!src.empty()) FMMHP_HIP(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return FMMHP_OK;
}

template <class T>
static fmmhp_status to_host(std::vector<T> &dst, const T *src, size_t n, hipStream_t s) {
    dst.resize(n);
    if (n) FMMHP_HIP(hipMemcpyAsync(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost, s));
    return FMMHP_OK;
}

static fmmhp_status ensure_vec_ws(Arena &A, const Tree &T, Sched &S, int nv);

fmmhp_status build_schedule(Arena &A, const Tree &T, Sched &S, int PB, const cplx *Zs, hipStream_t s) {
    S.PB = PB;
    S.Z = Zs[0];
    S.real_Z = true;
    for (int k = 0; k < T.n_inst; ++k) S.real_Z = S.real_Z && Zs[k].im == 0.0;
    if (S.bc != 0) S.real_Z = true;  // Dirichlet and Neumann kernels are real
    S.nloc = S.real_Z ? 1 : 2;
    const bool react = S.bc == 0;
    const double isg = S.bc == 2 ? -1.0 : 1.0;
    const int nbox = T.nbox;
    if (nbox >= (1 << 28)) {  // the tile builder packs a box index and its class into one int32
        set_error("%d boxes: the schedule supports fewer than 2^28", nbox);
        return FMMHP_EUNSUPPORTED;
    }
    std::vector<int32_t> level, bx, by, leaf, voff, vent, xoff, binst;
    FMMHP_CHECK(to_host(binst, T.inst, nbox, s));
    FMMHP_CHECK(to_host(level, T.level, nbox, s));
    FMMHP_CHECK(to_host(bx, T.bx, nbox, s));
    FMMHP_CHECK(to_host(by, T.by, nbox, s));
    FMMHP_CHECK(to_host(leaf, T.leaf, nbox, s));
    FMMHP_CHECK(to_host(voff, T.off[1], (size_t)nbox + 1, s));
    FMMHP_CHECK(to_host(vent, T.ent[1], (size_t)T.len[1], s));
    FMMHP_CHECK(to_host(xoff, T.off[3], (size_t)nbox + 1, s));
    std::vector<int32_t> uoff, uent, cnt, xent;
    FMMHP_CHECK(to_host(xent, T.ent[3], (size_t)T.len[3], s));
    FMMHP_CHECK(to_host(uoff, T.off[0], (size_t)nbox + 1, s));
    FMMHP_CHECK(to_host(uent, T.ent[0], (size_t)T.len[0], s));
    FMMHP_CHECK(to_host(cnt, T.count, (size_t)nbox, s));
    FMMHP_HIP(hipStreamSynchronize(s));
    S.p2p_pairs[0] = S.p2p_pairs[1] = 0;
    for (int b = 0; b < nbox; ++b)
        for (int e = uoff[b]; e < uoff[b + 1]; ++e)
            S.p2p_pairs[uent[e] & 1] += (int64_t)cnt[b] * cnt[uent[e] >> 1];
    S.m2l_pairs[0] = S.m2l_pairs[1] = 0;
    for (size_t e = 0; e < vent.size(); ++e) S.m2l_pairs[vent[e] & 1] += 1;

    // Host threads for the slot table and the M2L tiles (each takes whole box ranges or tiles)
    const int nthr = (int)std::max<size_t>(1, std::min<size_t>((size_t)16, (size_t)std::max(1u, std::thread::hardware_concurrency())));
    auto run_threads = [&](auto &&fn) {
        std::vector<std::thread> pool;
        for (int t = 1; t < nthr; ++t) pool.emplace_back(fn, t);
        fn(0);
        for (auto &th : pool) th.join();
    };
    // M2L slots: vslot[b * kNumSlots + o] = upper V source of box b at offset slot o, or -1; image
    // V entries (source << 5 | slot) per box.  Threads take contiguous box ranges.
    std::unique_ptr<int32_t[]> vslot(new int32_t[(size_t)kNumSlots * std::max(1, nbox)]);
    std::vector<int32_t> vimg_off(nbox + 1, 0), vimg_ent;
    {
        std::vector<std::vector<int32_t>> img_t(nthr);
        std::atomic<int> bad{0};  // 1: V entry outside the 7 x 7 block, 2: image entry above its target
        run_threads([&](int t) {
            const int b0 = (int)((int64_t)nbox * t / nthr), b1 = (int)((int64_t)nbox * (t + 1) / nthr);
            std::fill(vslot.get() + (size_t)b0 * kNumSlots, vslot.get() + (size_t)b1 * kNumSlots, -1);
            std::vector<int32_t> &out = img_t[t];
            for (int b = b0; b < b1; ++b) {
                const int l = level[b];
                for (int e = voff[b]; e < voff[b + 1]; ++e) {
                    const int c = vent[e] >> 1, img = vent[e] & 1;
                    const int dx = bx[c] - bx[b];
                    const int cy = img ? ((1 << l) - 1 - by[c]) : by[c];
                    const int dy = cy - by[b];
                    if (dx < -3 || dx > 3 || dy < -3 || dy > 3) {
                        bad = 1;
                        continue;
                    }
                    if (!img) {
                        vslot[(size_t)b * kNumSlots + slot_of(dx, dy)] = c;
                    } else {
                        if (dy > -1) bad = 2;
                        out.push_back((c << 5) | slot_of(dx, dy));
                    }
                }
                vimg_off[b + 1] = (int32_t)out.size();
            }
        });
        if (bad == 1) {
            set_error("internal: V entry outside the 7x7 offset block");
            return FMMHP_EUNSUPPORTED;
        }
        if (bad == 2) {
            set_error("internal: image V entry above its target");
            return FMMHP_EUNSUPPORTED;
        }
        // per-range counts to offsets, then the ranges' entries in box order
        int32_t base = 0;
        for (int t = 0; t < nthr; ++t) {
            const int b0 = (int)((int64_t)nbox * t / nthr), b1 = (int)((int64_t)nbox * (t + 1) / nthr);
            for (int b = b0; b < b1; ++b) vimg_off[b + 1] += base;
            base += (int32_t)img_t[t].size();
            vimg_ent.insert(vimg_ent.end(), img_t[t].begin(), img_t[t].end());
        }
    }
    FMMHP_CHECK(to_dev(A, &S.vimg_off, vimg_off, "vimg_off", s));
    {
        std::vector<int32_t> ib;
        for (int b = 0; b < nbox; ++b)
            if (vimg_off[b + 1] > vimg_off[b]) ib.push_back(b);
        S.nibox = (int)ib.size();
        FMMHP_CHECK(to_dev(A, &S.ibox, ib, "image V boxes", s));
        S.ibox_lev.assign(T.depth + 2, 0);
        for (int l = 0; l <= T.depth + 1; ++l)
            S.ibox_lev[l] = (int)(std::lower_bound(ib.begin(), ib.end(), T.lev_start[std::max(1, std::min(l, T.depth + 1))]) - ib.begin());
    }
    FMMHP_CHECK(to_dev(A, &S.vimg_ent, vimg_ent, "vimg_ent", s));

    // M2L tiles: up to kTile boxes of one level and one child class (bx & 1, by & 1), consecutive in
    // Morton order.  Boxes of one class have the same V offsets away from boundaries, so the lanes
    // of a tile walk the same offset slots.  A tile whose distinct upper V sources do not fit the
    // LDS staging buffer is split in halves.  The FP32 matrix-core M2L builds its tiles the same way
    // with a smaller source cap (it stages all coefficients of the sources at once, in FP32).
    // The tiles are built by host threads, each taking whole initial tiles (and their halves).
    std::vector<int32_t> tiles, tlev, tsoff(1, 0), tsrc;
    std::vector<int16_t> tslot;
    std::vector<uint64_t> tmask;
    {
        struct TileOut {
            std::vector<int32_t> boxes, src, nsrc, lev;  // kTile boxes (-1 padded) and sources per tile
            std::vector<int16_t> slot;                    // kNumSlots x kTile per tile
            std::vector<uint64_t> mask;
        };
        std::vector<int32_t> seq;                          // boxes grouped by (level, class), Morton order
        std::vector<std::pair<int, int>> init;             // initial tiles: [lo, hi) ranges of seq
        std::vector<int> init_lev(T.depth + 2, 0);         // first initial tile of each level
        for (int l = 2; l <= T.depth; ++l) {
            init_lev[l] = (int)init.size();
            for (int cls = 0; cls < 4; ++cls) {
                const int g0 = (int)seq.size();
                for (int b = T.lev_start[l]; b < T.lev_start[l + 1]; ++b)
                    if (((bx[b] & 1) | ((by[b] & 1) << 1)) == cls) seq.push_back(b);
                for (int a0 = g0; a0 < (int)seq.size(); a0 += kTile)
                    init.push_back({a0, std::min(a0 + kTile, (int)seq.size())});
            }
        }
        init_lev[T.depth + 1] = (int)init.size();
        const int max_src = kM2LMaxSrc;
        std::vector<TileOut> outs(init.size());
        // one range: its distinct sources; halves while they do not fit the LDS staging
        auto build_range = [&](auto &&self, int lo, int hi, std::vector<int32_t> &pos, std::vector<int32_t> &uniq,
                               TileOut &o) -> void {
            uniq.clear();
            for (int q = lo; q < hi; ++q) {
                const int32_t *vs = vslot.get() + (size_t)seq[q] * kNumSlots;
                for (int k = 0; k < kNumSlots; ++k)
                    if (vs[k] >= 0 && pos[vs[k]] < 0) {
                        pos[vs[k]] = 0;
                        uniq.push_back(vs[k]);
                    }
            }
            if ((int)uniq.size() > max_src && hi - lo > 1) {
                for (int c : uniq) pos[c] = -1;
                const int mid = lo + (hi - lo) / 2;
                self(self, lo, mid, pos, uniq, o);
                self(self, mid, hi, pos, uniq, o);
                return;
            }
            // sources by child class, then box: at one slot the lanes of a one-class tile read
            // nearly consecutive LDS entries (few bank conflicts)
            // (class, box) as one key, class above bit 28 (box indices stay below 2^28)
            for (int32_t &u : uniq) u |= ((bx[u] & 1) | ((by[u] & 1) << 1)) << 28;
            std::sort(uniq.begin(), uniq.end());
            for (int32_t &u : uniq) u &= (1 << 28) - 1;
            for (int i = 0; i < (int)uniq.size(); ++i) pos[uniq[i]] = i;
            const size_t t0 = o.slot.size();
            o.slot.resize(t0 + (size_t)kNumSlots * kTile, (int16_t)-1);
            uint64_t msk = 0;
            for (int lane = 0; lane < kTile; ++lane) {
                const int q = lo + lane;
                const int b = q < hi ? seq[q] : -1;
                o.boxes.push_back(b);
                if (b < 0) continue;
                const int32_t *vs = vslot.get() + (size_t)b * kNumSlots;
                for (int k = 0; k < kNumSlots; ++k) {
                    if (vs[k] < 0) continue;
                    o.slot[t0 + (size_t)k * kTile + lane] = (int16_t)pos[vs[k]];
                    msk |= 1ull << k;
                }
            }
            for (int c : uniq) pos[c] = -1;
            o.lev.push_back(level[seq[lo]]);
            o.mask.push_back(msk);
            o.src.insert(o.src.end(), uniq.begin(), uniq.end());
            o.nsrc.push_back((int32_t)uniq.size());
        };
        run_threads([&](int tid) {
            std::vector<int32_t> pos(nbox, -1), uniq;
            for (size_t i = tid; i < init.size(); i += nthr)
                build_range(build_range, init[i].first, init[i].second, pos, uniq, outs[i]);
        });
        // the initial tiles' outputs in order (levels ascending): offsets, then threads copy
        const size_t ni = init.size();
        std::vector<size_t> at(ni + 1, 0), as(ni + 1, 0);  // tiles before initial tile i, sources before it
        for (size_t i = 0; i < ni; ++i) {
            at[i + 1] = at[i] + outs[i].lev.size();
            as[i + 1] = as[i] + outs[i].src.size();
        }
        const size_t ntile = at[ni];
        tiles.resize(ntile * kTile);
        tslot.resize(ntile * kNumSlots * kTile);
        tmask.resize(ntile);
        tlev.resize(ntile);
        tsrc.resize(as[ni]);
        tsoff.resize(ntile + 1);
        tsoff[0] = 0;
        run_threads([&](int tid) {
            for (size_t i = tid; i < ni; i += nthr) {
                const TileOut &o = outs[i];
                std::copy(o.boxes.begin(), o.boxes.end(), tiles.begin() + at[i] * kTile);
                std::copy(o.slot.begin(), o.slot.end(), tslot.begin() + at[i] * kNumSlots * kTile);
                std::copy(o.mask.begin(), o.mask.end(), tmask.begin() + at[i]);
                std::copy(o.lev.begin(), o.lev.end(), tlev.begin() + at[i]);
                std::copy(o.src.begin(), o.src.end(), tsrc.begin() + as[i]);
                int32_t off = (int32_t)as[i];
                for (size_t k = 0; k < o.nsrc.size(); ++k) tsoff[at[i] + k + 1] = (off += o.nsrc[k]);
            }
        });
        S.tile_lev.assign(T.depth + 2, 0);
        for (int l = 2; l <= T.depth + 1; ++l) S.tile_lev[l] = (int)at[init_lev[l]];
        S.tile_lev[0] = S.tile_lev[1] = 0;
    }
    S.ntiles = (int)tlev.size();
    FMMHP_CHECK(to_dev(A, &S.tiles, tiles, "tiles", s));
    FMMHP_CHECK(to_dev(A, &S.tile_level, tlev, "tile levels", s));
    FMMHP_CHECK(to_dev(A, &S.tile_src_off, tsoff, "tile source offsets", s));
    FMMHP_CHECK(to_dev(A, &S.tile_src, tsrc, "tile sources", s));
    FMMHP_CHECK(to_dev(A, &S.tile_slot, tslot, "tile slots", s));
    FMMHP_CHECK(to_dev(A, &S.tile_mask, tmask, "tile masks", s));

    // X-list targets, leaves
    std::vector<int32_t> xb, lv;
    for (int b = 0; b < nbox; ++b) {
        if (xoff[b + 1] > xoff[b]) xb.push_back(b);
        if (leaf[b]) lv.push_back(b);
    }
    S.nxbox = (int)xb.size();
    FMMHP_CHECK(to_dev(A, &S.xbox, xb, "xbox", s));
    // P2L groups: consecutive X boxes of a level while their sources total at most one chunk of 64;
    // per group its list entries that hold sources, {code, box slot, first row}, in row order
    {
        std::vector<int4> grp, gent;
        S.xgrp_lev.assign(T.depth + 2, 0);
        int l = 0;
        for (int i = 0; i < (int)xb.size(); ++i) {
            const int b = xb[i];
            int kb = 0;
            for (int e = xoff[b]; e < xoff[b + 1]; ++e) kb += cnt[xent[e] >> 1];
            const bool new_level = level[b] != l;
            while (level[b] > l) S.xgrp_lev[++l] = (int)grp.size();
            if (new_level || grp.empty() || grp.back().y + kb > 64)
                grp.push_back(make_int4(i, 0, (int)gent.size(), 0));
            int4 &g = grp.back();
            for (int e = xoff[b]; e < xoff[b + 1]; ++e) {
                const int k = cnt[xent[e] >> 1];
                if (k == 0) continue;
                gent.push_back(make_int4(xent[e], i - g.x, g.y, 0));
                g.y += k;
            }
        }
        while (l < T.depth + 1) S.xgrp_lev[++l] = (int)grp.size();
        grp.push_back(make_int4((int)xb.size(), 0, (int)gent.size(), 0));
        FMMHP_CHECK(to_dev(A, &S.xgrp, grp, "P2L groups", s));
        FMMHP_CHECK(to_dev(A, &S.xgent, gent, "P2L group entries", s));
        FMMHP_CHECK(A.alloc_n(&S.xgeo, xb.size(), "P2L box geometry"));
        if (!gent.empty())
            hipLaunchKernelGGL(k_xgent_first, dim3(nblk((int64_t)gent.size(), 256)), dim3(256), 0, s,
                               (int64_t)gent.size(), S.xgent, T.first);
        FMMHP_HIP(hipGetLastError());  // (xgeo is filled once the instance table is on the device)
    }
    // deep split: the finest levels holding at least half of the M2L tiles run on a second stream
    // as soon as their multipoles exist, beside the rest of the upward pass
    S.deep_level = 0;
    if (S.ntiles > 0) {
        for (int l = T.depth; l >= 3; --l)
            if (2 * (S.tile_lev[T.depth + 1] - S.tile_lev[l]) >= S.ntiles) {
                S.deep_level = l;
                break;
            }
    }
    FMMHP_CHECK(to_dev(A, &S.leaves, lv, "leaves", s));
    // subtree passes: below the first level (>= 3) with at least four boxes per CU, one block per
    // subtree runs all of that subtree's M2M (and later L2L) levels; the levels above run one
    // launch each.  A subtree's boxes at each level are a contiguous range (boxes are ordered by
    // level, instance, Morton prefix).
    S.sub_level = 0;
    {
        std::vector<int32_t> cfirst, nch;
        FMMHP_CHECK(to_host(cfirst, T.child_first, nbox, s));
        FMMHP_CHECK(to_host(nch, T.nchild, nbox, s));
        FMMHP_HIP(hipStreamSynchronize(s));
        int cus = 0, dev = 0;
        FMMHP_HIP(hipGetDevice(&dev));
        FMMHP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        // box ranges per level of the subtrees rooted at the boxes of level lr, nlev levels deep;
        // returns the largest subtree's box count; nonres (if given) gets the number of boxes in
        // subtrees of more than cap boxes
        auto subtree_ranges = [&](int lr, int nlev, std::vector<int2> &rng, int cap_, int64_t *nonres) {
            const int r0 = T.lev_start[lr], nr = T.lev_start[lr + 1] - r0;
            rng.assign((size_t)nr * nlev, make_int2(0, 0));
            int maxtot = 0;
            if (nonres) *nonres = 0;
            for (int r = 0; r < nr; ++r) {
                int a = r0 + r, b = a + 1, tot = 0;
                for (int k = 0; k < nlev && a < b; ++k) {
                    rng[(size_t)r * nlev + k] = make_int2(a, b);
                    tot += b - a;
                    int na = -1, nb = -1;
                    for (int x = a; x < b; ++x)
                        if (!leaf[x]) {
                            if (na < 0) na = cfirst[x];
                            nb = cfirst[x] + nch[x];
                        }
                    if (na < 0) break;
                    a = na;
                    b = nb;
                }
                maxtot = std::max(maxtot, tot);
                if (nonres && tot > cap_) *nonres += tot;
            }
            return maxtot;
        };
        // resident LDS rows: enough for the largest subtree, within 48 KB of expansions per block
        const int cap = std::min(kSubMaxSlots, (int)(48 * 1024 / ((PB + 1) * sizeof(cplx))));
        // the cut: the first level (>= 3) with at least four boxes per CU whose subtrees nearly all
        // fit in LDS (at most 5% of the boxes below the cut in larger ones, which take the slower
        // level-by-level path inside their block); deep narrow trees with no such level run one
        // launch per level instead
        std::vector<int2> rng;
        int maxtot = 0;
        // a forest runs one launch per level: its many small subtrees, each set up once per charge
        // vector, make the subtree blocks slower than the plain level launches there
        for (int l = 3; l < T.depth && T.n_inst == 1; ++l) {
            if (T.lev_start[l + 1] - T.lev_start[l] < 4 * std::max(1, cus)) continue;
            int64_t nonres = 0;
            const int mt = subtree_ranges(l, T.depth - l + 1, rng, cap, &nonres);
            if (nonres * 20 <= (int64_t)(T.lev_start[T.depth + 1] - T.lev_start[l])) {
                S.sub_level = l;
                maxtot = mt;
                break;
            }
        }
        // consecutive subtrees whose boxes together fit the LDS rows run in one block: their box
        // ranges at each level are contiguous (boxes are ordered by level, instance, Morton prefix),
        // so a group is handled like one subtree with several roots.  Subtrees larger than the rows
        // stay alone.  Returns the largest group's box count among those that fit.
        auto group_subtrees = [&](std::vector<int2> &r, int nlev, int lim, int *ngroups) {
            const int nr = (int)(r.size() / nlev);
            std::vector<int2> g;
            int gmax = 0, i = 0;
            auto size_of = [&](int k) {
                int t = 0;
                for (int l = 0; l < nlev; ++l) t += r[(size_t)k * nlev + l].y - r[(size_t)k * nlev + l].x;
                return t;
            };
            while (i < nr) {
                int tot = size_of(i), j = i + 1;
                if (tot <= lim)
                    for (int t; j < nr && (t = size_of(j)) <= lim && tot + t <= lim; ++j) tot += t;
                for (int l = 0; l < nlev; ++l) {
                    int a = 0, b = 0;
                    for (int k = i; k < j; ++k) {
                        const int2 q = r[(size_t)k * nlev + l];
                        if (q.y > q.x) {
                            if (b == 0) a = q.x;
                            b = q.y;
                        }
                    }
                    g.push_back(make_int2(a, b));
                }
                if (tot <= lim) gmax = std::max(gmax, tot);
                i = j;
            }
            r.swap(g);
            *ngroups = (int)(r.size() / nlev);
            return gmax;
        };
        S.m2m_ch_lev.assign(T.depth + 2, 0);
        S.l2l_ch_lev.assign(T.depth + 2, 0);
        if (S.sub_level > 0) {
            const int lc = S.sub_level;
            S.sub_nlev = T.depth - lc + 1;
            maxtot = group_subtrees(rng, S.sub_nlev, cap, &S.n_sub);
            FMMHP_CHECK(to_dev(A, &S.sub_rng, rng, "subtree ranges", s));
            S.sub_ld_m2m = std::max(4 * kM2MParents, std::min(maxtot, cap));
            S.sub_ld_l2l = std::max(kL2LChildren, std::min(maxtot * S.nloc, cap));
            // the subtrees whose expansions do not fit those rows: their parents (M2M) and children
            // (L2L) level by level in chunks, so that all of them run in parallel
            {
                const int nl = S.sub_nlev;
                std::vector<std::vector<int2>> mc(T.depth + 1), lcx(T.depth + 1);
                for (int r = 0; r < S.n_sub; ++r) {
                    const int2 *R = &rng[(size_t)r * nl];
                    int tot = 0;
                    for (int k = 0; k < nl; ++k) tot += R[k].y - R[k].x;
                    if (tot > S.sub_ld_m2m)
                        for (int k = 0; k + 1 < nl; ++k)
                            for (int a0 = R[k].x; a0 < R[k].y; a0 += kM2MParents)
                                mc[lc + k].push_back(make_int2(a0, std::min(a0 + kM2MParents, R[k].y)));
                    if (tot * S.nloc > S.sub_ld_l2l)
                        for (int k = 1; k < nl; ++k)
                            for (int a0 = R[k].x; a0 < R[k].y; a0 += kL2LChildren)
                                lcx[lc + k].push_back(make_int2(a0, std::min(a0 + kL2LChildren, R[k].y)));
                }
                std::vector<int2> mall, lall;
                for (int l = 0; l <= T.depth; ++l) {
                    S.m2m_ch_lev[l] = (int)mall.size();
                    S.l2l_ch_lev[l] = (int)lall.size();
                    mall.insert(mall.end(), mc[l].begin(), mc[l].end());
                    lall.insert(lall.end(), lcx[l].begin(), lcx[l].end());
                }
                S.m2m_ch_lev[T.depth + 1] = (int)mall.size();
                S.l2l_ch_lev[T.depth + 1] = (int)lall.size();
                if (!mall.empty()) FMMHP_CHECK(to_dev(A, &S.m2m_ch, mall, "M2M chunks", s));
                if (!lall.empty()) FMMHP_CHECK(to_dev(A, &S.l2l_ch, lall, "L2L chunks", s));
            }
            // the L2L levels 4..lc in one launch of level-3-rooted subtrees (after level 3's own L2L)
            // (only when those subtrees fit in LDS)
            if (lc >= 5) {
                std::vector<int2> trng;
                int tmax = subtree_ranges(3, lc - 3 + 1, trng, cap, nullptr);
                if (tmax <= cap) {
                    S.top_nlev = lc - 3 + 1;
                    tmax = group_subtrees(trng, S.top_nlev, cap / S.nloc, &S.n_top);
                    FMMHP_CHECK(to_dev(A, &S.top_rng, trng, "top subtree ranges", s));
                    S.top_ld_l2l = std::max(kL2LChildren, std::min(tmax * S.nloc, cap));
                    S.top_ld_m2m = std::max(4 * kM2MParents, std::min(tmax, cap));
                }
            }
        }
    }
    {
        std::vector<int32_t> woff, first, wp, rl;
        FMMHP_CHECK(to_host(woff, T.off[2], (size_t)nbox + 1, s));
        FMMHP_CHECK(to_host(first, T.first, (size_t)nbox, s));
        FMMHP_HIP(hipStreamSynchronize(s));
        for (int b : lv) {
            if (woff[b + 1] > woff[b])
                for (int j = first[b]; j < first[b] + cnt[b]; ++j) wp.push_back(j);
            bool img = false;
            for (int e = uoff[b]; e < uoff[b + 1] && !img; ++e) img = (uent[e] & 1) != 0;
            if (img)
                for (int j = first[b]; j < first[b] + cnt[b]; ++j) rl.push_back(j);
        }
        S.n_wpts = (int64_t)wp.size();
        S.n_rpts = (int64_t)rl.size();
        FMMHP_CHECK(to_dev(A, &S.wpts, wp, "W-list targets", s));
        FMMHP_CHECK(to_dev(A, &S.rpts, rl, "near-axis targets", s));
    }

    // tables
    const int NT = 2 * PB + 1;
    const int NTP = m2l_row(PB);
    std::vector<double> fact(NT + 1), ifact(NT + 1);
    fact[0] = 1.0;
    for (int j = 1; j <= NT; ++j) fact[j] = fact[j - 1] * j;
    for (int j = 0; j <= NT; ++j) ifact[j] = 1.0 / fact[j];
    FMMHP_CHECK(to_dev(A, &S.fact, fact, "factorials", s));
    FMMHP_CHECK(to_dev(A, &S.invfact, ifact, "inverse factorials", s));

    using C = std::complex<double>;
    auto cx = [](C v) { return mk(v.real(), v.imag()); };
    const double i4p = 1.0 / (4.0 * M_PI);
    std::vector<cplx> Tfree((size_t)kNumSlots * NTP, mk(0, 0)), Lfree(kNumSlots, mk(0, 0));
    for (int dy = -3; dy <= 3; ++dy)
        for (int dx = -3; dx <= 3; ++dx) {
            if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
            const int o = slot_of(dx, dy);
            const C D((double)dx, (double)dy);
            const C t = 1.0 / (2.0 * D);
            C tj = t;  // (j-1)! t^j
            for (int j = 1; j < NT; ++j) {
                Tfree[(size_t)o * NTP + j] = cx(-i4p * tj);
                tj = tj * t * (double)j;
            }
            Lfree[o] = cx(-i4p * std::log(-D));
        }
    FMMHP_CHECK(to_dev(A, &S.Tfree, Tfree, "Tfree", s));
    if (S.m2l_fp32) {
        // FP32 matrix-core operators: B[o][c][k] (column c, row k) of the 2x2 embedding of
        // T''_{nm} = T_{n+m} / (n! m!); rows k = m (Re w''_m) and P1 + m (Im w''_m), columns c = n
        // (Re acc''_n) and P1 + n (Im acc''_n), zero padding
        const int P1 = PB + 1, KP = m2l32_kp(PB), NP = m2l32_np(PB);
        std::vector<float> B((size_t)kNumSlots * KP * NP, 0.f);
        for (int o = 0; o < kNumSlots; ++o)
            for (int n = 0; n <= PB; ++n)
                for (int m = 0; m <= PB; ++m) {
                    const cplx t = Tfree[(size_t)o * NTP + n + m];
                    const double sc = ifact[n] * ifact[m];
                    const float tr = (float)(t.re * sc), ti = (float)(t.im * sc);
                    float *Bo = B.data() + (size_t)o * KP * NP;
                    Bo[(size_t)n * KP + m] = tr;
                    Bo[(size_t)(P1 + n) * KP + m] = ti;
                    Bo[(size_t)n * KP + P1 + m] = -ti;
                    Bo[(size_t)(P1 + n) * KP + P1 + m] = tr;
                }
        FMMHP_CHECK(to_dev(A, &S.Bf32, B, "FP32 M2L operators", s));
    }
    FMMHP_CHECK(to_dev(A, &S.Lfree, Lfree, "Lfree", s));
    {
        std::vector<double> ls(nbox);
        // log(2 rho) per (instance, level), the same value for every box there
        const int nl = T.depth + 1;
        std::vector<double> lt((size_t)T.n_inst * nl);
        for (int k = 0; k < T.n_inst; ++k)
            for (int l = 0; l < nl; ++l) lt[(size_t)k * nl + l] = std::log(ldexp(T.inst_S[k], -l));
        for (int b = 0; b < nbox; ++b) ls[b] = lt[(size_t)binst[b] * nl + level[b]];
        FMMHP_CHECK(to_dev(A, &S.logside, ls, "log side", s));
        std::vector<InstInfo> ii(T.n_inst);
        for (int k = 0; k < T.n_inst; ++k) ii[k] = InstInfo{T.inst_xlo[k], T.inst_S[k], Zs[k], isg, react ? 1 : 0, 0};
        FMMHP_CHECK(to_dev(A, &S.inst_info, ii, "instance info", s));
        if (S.nxbox > 0) {  // P2L box geometry (the instance table is needed)
            hipLaunchKernelGGL(k_xgeo, dim3(nblk((int64_t)S.nxbox, 256)), dim3(256), 0, s, S.nxbox, S.xbox,
                               S.inst_info, T.inst, T.level, T.bx, T.by, S.xgeo);
            FMMHP_HIP(hipGetLastError());
        }
    }

    // image M2L tables: one block of kNumImgSlots operators per (instance, level) that has image V
    // entries; ibase[b] is the block of box b
    std::vector<int32_t> ibase(nbox, -1);
    std::vector<std::pair<int, int>> blocks;  // (instance, level)
    {
        std::map<std::pair<int, int>, int> bid;
        for (int b = 0; b < nbox; ++b) {
            if (vimg_off[b + 1] == vimg_off[b]) continue;
            const auto key = std::make_pair(binst[b], level[b]);
            auto it = bid.find(key);
            if (it == bid.end()) {
                it = bid.emplace(key, (int)blocks.size()).first;
                blocks.push_back(key);
            }
            ibase[b] = it->second;
        }
    }
    FMMHP_CHECK(to_dev(A, &S.ibase, ibase, "image table blocks", s));
    const size_t nblkimg = std::max<size_t>(1, blocks.size());
    std::vector<cplx> TH(nblkimg * kNumImgSlots * NTP, mk(0, 0)), TG(TH.size(), mk(0, 0)),
        Limg(kNumImgSlots, mk(0, 0));
    for (int dy = -3; dy <= -1; ++dy)
        for (int dx = -3; dx <= 3; ++dx) {
            const int is = slot_of(dx, dy);
            const C D((double)dx, (double)dy);
            Limg[is] = cx(isg * i4p * std::log(-D));
        }
    // the blocks are independent (a forest has one per instance and level): host threads take them in
    // turn, each with its own scratch and its own largest |Z| x separation
    std::vector<double> pmax_t(nthr, 0.0);
    run_threads([&](int th) {
        std::vector<cplx> K(NT), Km(NT);
        double &pmax = pmax_t[th];
        for (size_t bi = th; bi < blocks.size(); bi += nthr) {
            const int k = blocks[bi].first, l = blocks[bi].second;
            const cplx Z = Zs[k];
            const C Zc(Z.re, Z.im);
            const double sl = ldexp(T.inst_S[k], -l), rho = 0.5 * sl;
            for (int dy = -3; dy <= -1; ++dy)
                for (int dx = -3; dx <= 3; ++dx) {
                    if (std::abs(dx) <= 1 && dy == -1) continue;  // adjacent: never in V
                    const int is = slot_of(dx, dy);
                    const C D((double)dx, (double)dy);
                    const C t = 1.0 / (2.0 * D);
                    const double X = -dx * sl, Y = -dy * sl;
                    if (react) {
                        pmax = std::max(pmax, std::abs(Zc) * std::hypot(X, Y));
                        reaction_In_scaled_ld(X, Y, Z, rho, NT - 1, K.data());
                        reaction_In_scaled_ld(-X, Y, Z, rho, NT - 1, Km.data());
                    } else {
                        std::fill(K.begin(), K.end(), mk(0.0, 0.0));
                        std::fill(Km.begin(), Km.end(), mk(0.0, 0.0));
                    }
                    C tj = t;
                    for (int j = 0; j < NT; ++j) {
                        C fr(0.0, 0.0);
                        if (j >= 1) {
                            fr = isg * i4p * tj;
                            tj = tj * t * (double)j;
                        }
                        // - j! i^j K_j
                        C ij(1.0, 0.0);
                        for (int r = 0; r < (j & 3); ++r) ij *= C(0.0, 1.0);
                        const C kp(K[j].re, K[j].im), km(Km[j].re, -Km[j].im);
                        const size_t idx = (bi * kNumImgSlots + is) * NTP + j;
                        TH[idx] = cx(fr - fact[j] * ij * kp);
                        TG[idx] = cx(fr - fact[j] * ij * km);
                    }
                }
        }
    });
    const double pmax = *std::max_element(pmax_t.begin(), pmax_t.end());
    if (pmax > kMaxTablePZ) {
        set_error("impedance times box separation reaches %.3g at the coarsest level; the M2L tables "
                  "are accurate up to %.0f",
                  pmax, kMaxTablePZ);
        return FMMHP_EUNSUPPORTED;
    }
    // P2L (X list) and M2P (W list) run the double-precision recursion on the device: keep
    // |Z| * distance within the range where it loses at most ~4 digits
    {
        std::vector<int32_t> went, woff2;
        FMMHP_CHECK(to_host(woff2, T.off[2], (size_t)nbox + 1, s));
        FMMHP_CHECK(to_host(went, T.ent[2], (size_t)T.len[2], s));
        FMMHP_HIP(hipStreamSynchronize(s));
        double wxmax = 0.0;
        auto reach = [&](int b, int c) {  // |Z| * (centre distance to the image of c + half diagonals)
            const int k = binst[b];
            const double Sk = T.inst_S[k];
            const double sb = ldexp(Sk, -level[b]), sc = ldexp(Sk, -level[c]);
            const double xb = (bx[b] + 0.5) * sb, yb = -0.5 * Sk + (by[b] + 0.5) * sb;
            const double xc = (bx[c] + 0.5) * sc, yc = 0.5 * Sk - (by[c] + 0.5) * sc;  // image centre
            const double d = std::hypot(xb - xc, yb - yc) + 0.7072 * (sb + sc);
            return std::hypot(Zs[k].re, Zs[k].im) * d;
        };
        for (int b = 0; b < nbox; ++b) {
            for (int e = woff2[b]; e < woff2[b + 1]; ++e)
                if (went[e] & 1) wxmax = std::max(wxmax, reach(b, went[e] >> 1));
            for (int e = xoff[b]; e < xoff[b + 1]; ++e)
                if (xent[e] & 1) wxmax = std::max(wxmax, reach(b, xent[e] >> 1));
        }
        if (react && wxmax > kMaxDevicePZ) {
            set_error("impedance times distance reaches %.3g on a W or X list entry; the device I_n "
                      "recursion is used up to %.0f",
                      wxmax, kMaxDevicePZ);
            return FMMHP_EUNSUPPORTED;
        }
    }
    FMMHP_CHECK(to_dev(A, &S.TimgH, TH, "TimgH", s));
    FMMHP_CHECK(to_dev(A, &S.TimgG, TG, "TimgG", s));
    FMMHP_CHECK(to_dev(A, &S.Limg, Limg, "Limg", s));

    std::vector<cplx> Em((size_t)4 * (PB + 1)), El((size_t)4 * (PB + 1));
    for (int q = 0; q < 4; ++q) {
        const C eps(((q & 1) ? 0.5 : -0.5), ((q & 2) ? 0.5 : -0.5));
        C pm(1.0, 0.0), pl(1.0, 0.0);
        for (int j = 0; j <= PB; ++j) {
            Em[(size_t)q * (PB + 1) + j] = cx(pm * ifact[j]);
            El[(size_t)q * (PB + 1) + j] = cx(pl * ifact[j]);
            pm *= -eps;
            pl *= eps;
        }
    }
    FMMHP_CHECK(to_dev(A, &S.E_m2m, Em, "E_m2m", s));
    {
        std::vector<double2> lt(kLogTable);
        for (int k = 0; k < kLogTable; ++k) log_table_entry(k, &lt[k].x, &lt[k].y);
        FMMHP_CHECK(to_dev(A, &S.logtab, lt, "log table", s));
    }
    FMMHP_CHECK(to_dev(A, &S.E_l2l, El, "E_l2l", s));
    // point range of every U entry's source box, for the near-field walk
    if (T.len[0] > 0) {
        FMMHP_CHECK(A.alloc_n(&S.u2, (size_t)T.len[0], "U entry ranges"));
        hipLaunchKernelGGL(k_u2, dim3(nblk(T.len[0], 256)), dim3(256), 0, s, (int64_t)T.len[0], T.ent[0], T.first,
                           T.count, S.u2);
        FMMHP_HIP(hipGetLastError());
    }

    // surface-term chunks: at most kSurfChunk points, within one instance
    {
        std::vector<PtChunk> ch;
        std::vector<int32_t> ich(T.n_inst + 1, 0);
        for (int k = 0; k < T.n_inst; ++k) {
            for (int64_t a0 = T.inst_off[k]; a0 < T.inst_off[k + 1]; a0 += kSurfChunk)
                ch.push_back(PtChunk{a0, std::min(T.inst_off[k + 1], a0 + kSurfChunk), k, 0});
            ich[k + 1] = (int32_t)ch.size();
        }
        S.n_rch = (int)ch.size();
        FMMHP_CHECK(to_dev(A, &S.rch, ch, "surface chunks", s));
        FMMHP_CHECK(to_dev(A, &S.inst_ch, ich, "instance chunk ranges", s));
    }
    // workspace
    FMMHP_CHECK(ensure_vec_ws(A, T, S, 1));
    FMMHP_CHECK(A.alloc_n(&S.xy, (size_t)T.n, "sorted coordinates (x, y)"));
    FMMHP_HIP(hipStreamCreateWithFlags(&S.side, hipStreamNonBlocking));
    FMMHP_HIP(hipStreamCreateWithFlags(&S.side2, hipStreamNonBlocking));
    FMMHP_HIP(hipEventCreateWithFlags(&S.ev_deep_ready, hipEventDisableTiming));
    FMMHP_HIP(hipEventCreateWithFlags(&S.ev_deep_done, hipEventDisableTiming));
    {
        int dev = 0, cus = 0;
        FMMHP_HIP(hipGetDevice(&dev));
        FMMHP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        S.cus = std::max(1, cus);
    }
    FMMHP_HIP(hipEventCreateWithFlags(&S.ev_fork, hipEventDisableTiming));
    FMMHP_HIP(hipEventCreateWithFlags(&S.ev_join, hipEventDisableTiming));
    FMMHP_HIP(hipEventCreateWithFlags(&S.ev_up, hipEventDisableTiming));
    hipLaunchKernelGGL(k_pack_xy, dim3(nblk(T.n, 256)), dim3(256), 0, s, T.xs, T.ys, T.n, S.xy);
    FMMHP_HIP(hipGetLastError());
    FMMHP_HIP(hipStreamSynchronize(s));
    return FMMHP_OK;
}

// Schedule of the symmetric near-field walks (near_walk 3 and 4), built the first time a plan
// selects one of them.
static fmmhp_status build_sym_walk(Arena &A, const Tree &T, Sched &S, hipStream_t s) {
    const int nbox = T.nbox;
    S.sym_built = true;
    // Symmetric near-field walk: records of at most 64 targets (a leaf, or a piece of a larger one),
    // each with its jobs (the self pair, the self-image pair when listed, each cross pair with
    // B > A); the cross jobs of a record own partial slots for B's points.  Per leaf B, the slots
    // of its cross pairs in ascending A (and record).  Every cross pair's mirror entry is checked; a
    // list that is not symmetric leaves the walk off for this plan.
    {
        std::vector<int32_t> first_h, uoff, uent, cnt;
        FMMHP_CHECK(to_host(first_h, T.first, (size_t)nbox, s));
        FMMHP_CHECK(to_host(uoff, T.off[0], (size_t)nbox + 1, s));
        FMMHP_CHECK(to_host(uent, T.ent[0], (size_t)T.len[0], s));
        FMMHP_CHECK(to_host(cnt, T.count, (size_t)nbox, s));
        FMMHP_HIP(hipStreamSynchronize(s));
        std::vector<int4> recs, jobs;
        std::vector<int32_t> in_cnt((size_t)nbox + 1, 0);
        int64_t npart = 0;
        bool ok = true;
        for (int la = 0; la < nbox && ok; ++la) {
            if (uoff[la + 1] == uoff[la]) continue;
            for (int e = uoff[la]; e < uoff[la + 1] && ok; ++e) {
                const int lb = uent[e] >> 1, img = uent[e] & 1;
                if (lb > la && !std::binary_search(uent.begin() + uoff[lb], uent.begin() + uoff[lb + 1], 2 * la + img))
                    ok = false;
            }
            for (int t0 = 0; t0 < cnt[la] && ok; t0 += 64) {
                const int e0 = (int)jobs.size();
                for (int e = uoff[la]; e < uoff[la + 1]; ++e) {
                    const int lb = uent[e] >> 1, img = uent[e] & 1;
                    if (lb < la) continue;
                    const int code = (int)(((unsigned)cnt[lb]) | ((unsigned)img << 31));
                    if (lb == la) {
                        jobs.push_back(make_int4(first_h[lb], code, -1, 0));
                        continue;
                    }
                    jobs.push_back(make_int4(first_h[lb], code, (int)npart, 0));
                    in_cnt[lb + 1] += 1;
                    npart += cnt[lb];
                }
                if (npart >= ((int64_t)1 << 31) || jobs.size() >= ((size_t)1 << 31)) ok = false;
                recs.push_back(make_int4(first_h[la] + t0, std::min(64, cnt[la] - t0), e0, (int)jobs.size()));
            }
        }
        S.sym_ok = ok && !recs.empty();
        if (S.sym_ok) {
            for (int b = 0; b < nbox; ++b) in_cnt[b + 1] += in_cnt[b];
            // each box's slots in the order the jobs were made (A ascending, then record)
            std::vector<int32_t> in_ent((size_t)in_cnt[nbox]), fill(in_cnt.begin(), in_cnt.end() - 1);
            size_t k = 0;
            for (int la = 0; la < nbox; ++la) {
                if (uoff[la + 1] == uoff[la]) continue;
                for (int t0 = 0; t0 < cnt[la]; t0 += 64)
                    for (int e = uoff[la]; e < uoff[la + 1]; ++e) {
                        const int lb = uent[e] >> 1;
                        if (lb < la) continue;
                        const int4 &jb = jobs[k++];
                        if (lb > la) in_ent[fill[lb]++] = jb.z;
                    }
            }
            S.sym_nrec = (int)recs.size();
            S.sym_npart = npart;
            FMMHP_CHECK(to_dev(A, &S.sym_rec, recs, "symmetric walk records", s));
            FMMHP_CHECK(to_dev(A, &S.sym_jobs, jobs, "symmetric walk jobs", s));
            FMMHP_CHECK(to_dev(A, &S.sym_in_off, in_cnt, "symmetric walk gather offsets", s));
            FMMHP_CHECK(to_dev(A, &S.sym_in, in_ent, "symmetric walk gather entries", s));
        }
    }

    return FMMHP_OK;
}

// Launch shape of the near field.  walk: 1 = sources loaded one step ahead, 2 = plain walk;
// groups: workgroups per CU of its bounded grid.  0 selects the default: the prefetching walk on
// two workgroups per CU, or for p >= 30 (far-field kernels heavy enough that the near field's
// instruction count matters more than its latency) the plain walk on four.
fmmhp_status apply_launch_shape(Arena &A, const Tree &T, Sched &S, int walk, int groups, hipStream_t s) {
    if (walk == 0) walk = S.PB >= 30 ? 2 : 1;
    if (groups == 0) groups = walk == 2 ? 4 : 2;
    if ((walk == 3 || walk == 4) && !S.sym_built) FMMHP_CHECK(build_sym_walk(A, T, S, s));
    S.near_walk = walk;
    S.near_blocks = (int64_t)groups * S.cus;
    return FMMHP_OK;
}

// Phase markers: when timing is on, one event per phase boundary on the eval stream.
struct Marks {
    hipEvent_t ev[FMMHP_NUM_PHASES + 1];  // main-stream boundaries; the NEAR slot pair is unused
    hipEvent_t near0 = nullptr, near1 = nullptr;
    hipEvent_t deep0 = nullptr, deep1 = nullptr;  // deep-level M2L on the second stream
    hipEvent_t km[4] = {nullptr, nullptr, nullptr, nullptr};  // k_m2l launches: deep (0, 1), coarse (2, 3)
    bool km_rec[2] = {false, false};
    bool on = false;
    fmmhp_status init(const Sched &S) {
        on = S.timing;
        if (!on) return FMMHP_OK;
        for (auto &e : ev) FMMHP_HIP(hipEventCreate(&e));
        FMMHP_HIP(hipEventCreate(&near0));
        FMMHP_HIP(hipEventCreate(&near1));
        FMMHP_HIP(hipEventCreate(&deep0));
        FMMHP_HIP(hipEventCreate(&deep1));
        for (auto &e : km) FMMHP_HIP(hipEventCreate(&e));
        return FMMHP_OK;
    }
    // bracket one k_m2l launch (k = 0 deep, 1 coarse) on its stream
    fmmhp_status km_mark(int k, int end, hipStream_t st) {
        if (!on) return FMMHP_OK;
        FMMHP_HIP(hipEventRecord(km[2 * k + end], st));
        km_rec[k] = true;
        return FMMHP_OK;
    }
    fmmhp_status mark(int k, hipStream_t s) {
        if (on) FMMHP_HIP(hipEventRecord(ev[k], s));
        return FMMHP_OK;
    }
    fmmhp_status commit(const Sched &S, hipStream_t s) {
        if (!on) return FMMHP_OK;
        int n = 0;
        for (int k = 0; k < 2; ++k) {
            if (km_rec[k]) {
                ++n;
            } else {  // no launch: an empty pair
                FMMHP_HIP(hipEventRecord(km[2 * k], s));
                FMMHP_HIP(hipEventRecord(km[2 * k + 1], s));
            }
        }
        for (auto &e : ev) S.events->push_back(e);
        S.events->push_back(near0);
        S.events->push_back(near1);
        S.events->push_back(deep0);
        S.events->push_back(deep1);
        for (auto &e : km) S.events->push_back(e);
        S.m2l_n->push_back(n);
        return FMMHP_OK;
    }
};

// Outputs of one evaluation pass (caller order): the potential and/or its gradient, and the
// coincident-charge sums (sorted order) used by the impedance gradient.
struct PassOut {
    double *phi = nullptr;      // [nv][n][2]
    cplx *gx = nullptr, *gy = nullptr;
    double *qc = nullptr;
    bool sorted = false;  // outputs in sorted (tree) order instead of caller order
};

// One pass over NV charge vectors q [NV][n] (caller order).  Far-field kernels take the vector
// from blockIdx.y; the near-field kernels share each pair's kernel value among the NV vectors.
template <int PB, int MODE, int NV>
static fmmhp_status eval_pass(const Tree &T, const Sched &S, const VecWs &ws, const double *q, const PassOut &out,
                              hipStream_t s) {
    // the near field and the deep-level M2L run on streams of their own (all on s when serial)
    hipStream_t side_ = S.serial ? s : S.side, side2_ = S.serial ? s : S.side2;
    constexpr bool DIP = is_dip(MODE);
    constexpr int LM = DIP ? (int)kPhi : MODE;
    const int nbox = T.nbox;
    Marks mk_;
    FMMHP_CHECK(mk_.init(S));
    FMMHP_CHECK(mk_.mark(FMMHP_PHASE_P2M, s));
    hipLaunchKernelGGL(k_gather_q, dim3(nblk(T.n, 256)), dim3(256), 0, s, q, T.perm, T.n, NV, ws.qs);
    // the near field needs only the sorted charges: run it on the side stream, concurrently with
    // the far-field chain, and join before the final leaf kernel
    LeafArgs la{S.inst_info, T.inst,    T.n_inst, NV,       T.n,      nbox,     S.nloc,   T.xs,     T.ys,
                ws.qs,        S.xy,      T.perm,   T.leaf_of, T.level, T.bx,     T.by,     T.first,  T.count,
                T.off[0],    T.ent[0],  T.off[2], T.ent[2], ws.W,      ws.Lam,    S.invfact, S.fact,
                S.bc == 0 ? ws.rank1 : nullptr,
                S.wpts,      S.n_wpts,  S.rpts,   S.logtab, ws.near,   S.bw.near_gx, S.bw.near_gy, out.qc,
                out.phi,     out.gx,    out.gy,   S.u2,     S.bc == 2 ? -1.0 : 1.0, S.nrm,
                out.sorted ? 1 : 0};
    FMMHP_HIP(hipEventRecord(S.ev_fork, s));
    FMMHP_HIP(hipStreamWaitEvent(side_, S.ev_fork, 0));
    if (mk_.on) FMMHP_HIP(hipEventRecord(mk_.near0, side_));
    // a bounded grid (a few workgroups per CU) leaves room on every CU for the far-field kernels
    // running concurrently on the main stream.  The launch shape is tuned on potentials; the near
    // fields of gradients and double layers do several times the work per pair and take at least
    // kNearHeavyGroups workgroups per CU (eight-vector potentials measured slower so).
    constexpr bool heavy_near = MODE != kPhi;
    const int64_t near_blocks = heavy_near ? std::max<int64_t>(S.near_blocks, (int64_t)kNearHeavyGroups * S.cus)
                                           : S.near_blocks;
    const dim3 near_grid((unsigned)std::min<int64_t>(nblk(T.n, 256), near_blocks));
    // walk 4 keeps each lane's targets and row sums in registers: single-vector passes only (the
    // others take walk 1)
    const bool sym_walk = MODE == kPhi && S.sym_ok && ws.part && (S.near_walk == 3 || (S.near_walk == 4 && NV == 1));
    if constexpr (MODE == kPhi) {
        if (sym_walk) {
            SymArgs sa{S.sym_nrec, S.sym_rec, S.sym_jobs, S.xy, ws.qs, S.logtab, S.bc == 2 ? -1.0 : 1.0,
                       ws.part,    ws.near,   T.n};
            const dim3 sym_grid((unsigned)std::min<int64_t>(nblk(S.sym_nrec, 4), near_blocks));
            if constexpr (NV == 1) {
                if (S.near_walk == 4)
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_near_blk<NV>), sym_grid, dim3(256), 0, side_, sa);
                else
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_near_sym<NV>), sym_grid, dim3(256), 0, side_, sa);
            } else {
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_near_sym<NV>), sym_grid, dim3(256), 0, side_, sa);
            }
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_near_gather<NV>), dim3(nblk(T.n, 256)), dim3(256), 0, side_, T.n,
                               T.leaf_of, T.first, S.sym_in_off, S.sym_in, ws.part, ws.near);
        }
    }
    if (!sym_walk && S.near_walk == 2)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_near_plain<MODE, NV>), near_grid, dim3(256), 0, side_, la);
    else if (!sym_walk)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_near<MODE, NV>), near_grid, dim3(256), 0, side_, la);
    if (S.n_rpts > 0 && S.bc == 0)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_near_reaction<MODE, NV>), dim3((unsigned)S.n_rpts), dim3(64), 0,
                           side_, la);
    FMMHP_HIP(hipGetLastError());
    // the surface sums also need only the sorted charges
    if (S.nloc == 1 && S.bc == 0 && S.rank1_side) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rank1_partial<DIP>), dim3(S.n_rch, NV), dim3(256), 0, side_, T.xs,
                           T.ys, ws.qs, NV, S.rch, S.n_rch, S.inst_info, S.nrm, ws.red);
        hipLaunchKernelGGL(k_rank1_final, dim3(T.n_inst, NV), dim3(256), 0, side_, ws.red, S.n_rch, S.inst_ch,
                           T.n_inst, ws.rank1);
        FMMHP_HIP(hipGetLastError());
    }
    if (mk_.on) FMMHP_HIP(hipEventRecord(mk_.near1, side_));
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_p2m<PB, DIP>), dim3(nblk((int64_t)T.nleaf * kP2MSplit, 256), NV), dim3(256),
                       0, s, S.inst_info, T.inst, S.leaves, T.nleaf, nbox, NV, T.level, T.bx, T.by, T.first, T.count,
                       T.xs, T.ys, ws.qs, S.nrm, ws.W);
    FMMHP_HIP(hipGetLastError());
    FMMHP_CHECK(mk_.mark(FMMHP_PHASE_M2M, s));
    // M2L (+ image M2L, P2L) over the levels [l0, l1) of the tree on stream st
    auto far_levels = [&](int l0, int l1, hipStream_t st, bool deep) -> fmmhp_status {
        const int t0 = S.tile_lev[l0], t1 = S.tile_lev[l1];
        if (t1 > t0) {
            constexpr int CH = m2l_chunk(PB);
            static_assert(m2l_waves(PB) * CH >= PB + 1, "M2L waves must cover all output coefficients");
            const int which = deep ? 0 : 1;
            if (S.m2l_fp32) {
                // FP32 rows of the sources (V sources are boxes of the same levels); the event pair
                // brackets the conversion and the matrix-core M2L together
                const int b0 = T.lev_start[l0], b1 = T.lev_start[l1];
                FMMHP_CHECK(mk_.km_mark(which, 0, st));
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_w_f32<PB>), dim3(nblk(b1 - b0, 256), NV), dim3(256), 0, st, b0, b1,
                                   nbox, S.fact, ws.W, ws.Wf);
                M2L32Args ma{nbox,    t0,        S.tiles, S.tile_src_off, S.tile_src, S.tile_slot, S.tile_mask,
                             S.Bf32,  S.Lfree,   S.logside, S.fact,       ws.Wf,       ws.Lam,       S.nloc};
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_m2l_f32<PB>), dim3(t1 - t0, NV), dim3(128 * (m2l32_np(PB) / 16)),
                                   0, st, ma);
                FMMHP_CHECK(mk_.km_mark(which, 1, st));
            } else {
                M2LArgs ma{nbox,    t0,      S.tiles,   S.tile_level, S.tile_src_off, S.tile_src, S.tile_slot,
                           S.tile_mask, S.Tfree, S.Lfree, S.logside,  ws.W,            ws.Lam,      S.nloc};
                FMMHP_CHECK(mk_.km_mark(which, 0, st));
                if (S.m2l_form != 2)
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_m2l<PB, CH>), dim3(t1 - t0, NV), dim3(64 * m2l_waves(PB)),
                                       0, st, ma);
                else
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_m2l_mf<PB, kMfSteps>), dim3(t1 - t0, NV),
                                       dim3(64 * mf_ncb(PB)), 0, st, ma);
                FMMHP_CHECK(mk_.km_mark(which, 1, st));
            }
        }
        const int i0 = S.ibox_lev[l0], i1 = S.ibox_lev[l1];
        if (i1 > i0)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_m2l_img<PB, NV>), dim3(i1 - i0), dim3(img_threads(NV)), 0, st, S.ibox + i0, nbox,
                               S.nloc, S.ibase, S.vimg_off, S.vimg_ent, S.TimgH, S.TimgG, S.Limg, S.logside,
                               S.bc == 2 ? -1.0 : 1.0, ws.W, ws.Lam);
        const int x0 = S.xgrp_lev[l0], x1 = S.xgrp_lev[l1];
        if (x1 > x0)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_p2l<PB, DIP, NV>), dim3(x1 - x0), dim3(64), 0, st, S.inst_info, T.inst,
                               S.nloc, S.xgrp + x0, S.xgent, S.xbox, S.xgeo, nbox, T.xs, T.ys, ws.qs, S.nrm, S.fact,
                               ws.Lam);
        FMMHP_HIP(hipGetLastError());
        return FMMHP_OK;
    };
    // the deep levels [ld, depth] start on the second stream once their multipoles exist
    const int ld = S.deep_level;
    auto fork_deep = [&]() -> fmmhp_status {
        FMMHP_HIP(hipEventRecord(S.ev_deep_ready, s));
        FMMHP_HIP(hipStreamWaitEvent(side2_, S.ev_deep_ready, 0));
        if (mk_.on) FMMHP_HIP(hipEventRecord(mk_.deep0, side2_));
        FMMHP_CHECK(far_levels(ld, T.depth + 1, side2_, true));
        if (mk_.on) FMMHP_HIP(hipEventRecord(mk_.deep1, side2_));
        FMMHP_HIP(hipEventRecord(S.ev_deep_done, side2_));
        return FMMHP_OK;
    };
    // fork point: once the deep multipoles exist, or (S.fork_late) after the whole upward pass
    const int lc = S.sub_level;
    int lf = S.fork_late ? 2 : ld;
    if (lc > 0 && lf >= lc) lf = T.depth;  // inside the subtree pass: fork right after it
    if (lc > 0) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_m2m_sub<PB>), dim3(S.n_sub, NV), dim3(256),
                           (PB + 1) * S.sub_ld_m2m * sizeof(cplx), s, S.sub_nlev, S.sub_rng, S.sub_ld_m2m, 1, nbox,
                           T.leaf, T.child_first, T.nchild, T.bx, T.by, S.E_m2m, ws.W);
        // the subtrees too large for LDS: one launch per parent level, deepest first
        for (int l = T.depth - 1; l >= lc; --l) {
            const int c0 = S.m2m_ch_lev[l], c1 = S.m2m_ch_lev[l + 1];
            if (c1 > c0)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_m2m_chunks<PB>), dim3(c1 - c0, NV), dim3(256),
                                   (PB + 1) * 4 * kM2MParents * sizeof(cplx), s, S.m2m_ch + c0, nbox, T.leaf,
                                   T.child_first, T.nchild, T.bx, T.by, S.E_m2m, ws.W);
        }
    }
    if (ld > 0 && lf > T.depth - 1) FMMHP_CHECK(fork_deep());
    // above the cut: with a top subtree pass, the parents of levels 3..lc-1 in one launch (subtrees
    // rooted at level 3, the cut level's multipoles their inputs), then level 2
    int l_top = (lc > 0 ? lc : T.depth) - 1;
    if (S.n_top > 0) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_m2m_sub<PB>), dim3(S.n_top, NV), dim3(256),
                           (PB + 1) * S.top_ld_m2m * sizeof(cplx), s, S.top_nlev, S.top_rng, S.top_ld_m2m, 0, nbox,
                           T.leaf, T.child_first, T.nchild, T.bx, T.by, S.E_m2m, ws.W);
        if (ld > 0 && lf >= 3 && lf <= l_top) FMMHP_CHECK(fork_deep());
        l_top = 2;
    }
    for (int l = l_top; l >= 2; --l) {
        const int lo = T.lev_start[l], nb = T.lev_start[l + 1] - lo;
        if (nb > 0)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_m2m<PB>), dim3(nblk(nb, kM2MParents), NV), dim3(256),
                               (PB + 1) * 4 * kM2MParents * sizeof(cplx), s, lo, nb,
                               nbox, T.leaf, T.child_first, T.nchild, T.bx, T.by, S.E_m2m, ws.W);
        if (ld > 0 && l == lf) FMMHP_CHECK(fork_deep());
    }
    FMMHP_HIP(hipGetLastError());
    // the W list (M2P) needs every multipole and adds into the near-field sums.  With the plain
    // near-field walk (chosen when the far field dominates, so the near-field stream has slack) it
    // runs on that stream once the upward pass is done; otherwise on the main stream before k_leaf.
    const bool w_side = S.n_wpts > 0 && S.near_walk == 2;
    if (w_side) {
        FMMHP_HIP(hipEventRecord(S.ev_up, s));
        FMMHP_HIP(hipStreamWaitEvent(side_, S.ev_up, 0));
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_leaf_w<PB, LM, NV>), dim3(nblk(S.n_wpts, 128)), dim3(128), 0, side_,
                           la);
        FMMHP_HIP(hipGetLastError());
    }
    FMMHP_HIP(hipEventRecord(S.ev_join, side_));
    FMMHP_CHECK(mk_.mark(FMMHP_PHASE_M2L, s));
    {
        const int lo = T.lev_start[1], hi = T.lev_start[2];
        const int64_t tot = (int64_t)(hi - lo) * (PB + 1) * S.nloc * NV;
        if (tot > 0)
            hipLaunchKernelGGL(k_zero_lam, dim3(nblk(tot, 256)), dim3(256), 0, s, lo, hi, nbox, PB + 1, S.nloc * NV,
                               ws.Lam);
    }
    FMMHP_CHECK(far_levels(2, ld > 0 ? ld : T.depth + 1, s, false));
    FMMHP_CHECK(mk_.mark(FMMHP_PHASE_P2L, s));
    FMMHP_CHECK(mk_.mark(FMMHP_PHASE_L2L, s));
    const int l2l_end = lc > 0 ? lc : T.depth;
    // with a top subtree pass, levels 4..lc run in one launch after level 3's
    const int l2l_last = S.n_top > 0 ? 3 : l2l_end;
    if (S.n_top > 0 && ld > 0 && ld <= l2l_end) FMMHP_HIP(hipStreamWaitEvent(s, S.ev_deep_done, 0));
    for (int l = 3; l <= l2l_last; ++l) {
        if (S.n_top == 0 && ld > 0 && l == ld) FMMHP_HIP(hipStreamWaitEvent(s, S.ev_deep_done, 0));
        const int lo = T.lev_start[l], nb = T.lev_start[l + 1] - lo;
        if (nb > 0)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_l2l<PB>), dim3(nblk(nb, kL2LChildren), NV), dim3(256),
                               (PB + 1) * kL2LChildren * sizeof(cplx), s, lo, nb,
                               nbox, S.nloc, T.parent, T.bx, T.by, S.E_l2l, ws.Lam);
    }
    if (S.n_top > 0)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_l2l_sub<PB>), dim3(S.n_top, NV), dim3(256),
                           (PB + 1) * S.top_ld_l2l * sizeof(cplx), s, S.top_nlev, S.top_rng, S.top_ld_l2l, 0, nbox,
                           S.nloc, T.parent, T.bx, T.by, S.E_l2l, ws.Lam);
    if (ld > 0 && ld > l2l_end) FMMHP_HIP(hipStreamWaitEvent(s, S.ev_deep_done, 0));
    if (lc > 0) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_l2l_sub<PB>), dim3(S.n_sub, NV), dim3(256),
                           (PB + 1) * S.sub_ld_l2l * sizeof(cplx), s, S.sub_nlev, S.sub_rng, S.sub_ld_l2l, 1, nbox,
                           S.nloc, T.parent, T.bx, T.by, S.E_l2l, ws.Lam);
        // the subtrees too large for LDS: one launch per child level, top level first
        for (int l = lc + 1; l <= T.depth; ++l) {
            const int c0 = S.l2l_ch_lev[l], c1 = S.l2l_ch_lev[l + 1];
            if (c1 > c0)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_l2l_chunks<PB>), dim3(c1 - c0, NV), dim3(256),
                                   (PB + 1) * kL2LChildren * sizeof(cplx), s, S.l2l_ch + c0, nbox, S.nloc, T.parent,
                                   T.bx, T.by, S.E_l2l, ws.Lam);
        }
    }
    if (mk_.on && ld == 0) {
        FMMHP_HIP(hipEventRecord(mk_.deep0, s));
        FMMHP_HIP(hipEventRecord(mk_.deep1, s));
    }
    FMMHP_HIP(hipGetLastError());
    FMMHP_CHECK(mk_.mark(FMMHP_PHASE_SURF, s));
    if (S.nloc == 1 && S.bc == 0 && !S.rank1_side) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rank1_partial<DIP>), dim3(S.n_rch, NV), dim3(256), 0, s, T.xs, T.ys,
                           ws.qs, NV, S.rch, S.n_rch, S.inst_info, S.nrm, ws.red);
        hipLaunchKernelGGL(k_rank1_final, dim3(T.n_inst, NV), dim3(256), 0, s, ws.red, S.n_rch, S.inst_ch, T.n_inst,
                           ws.rank1);
        FMMHP_HIP(hipGetLastError());
    }
    FMMHP_HIP(hipStreamWaitEvent(s, S.ev_join, 0));
    FMMHP_CHECK(mk_.mark(FMMHP_PHASE_LEAF, s));
    if (S.n_wpts > 0 && !w_side)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_leaf_w<PB, LM, NV>), dim3(nblk(S.n_wpts, 128)), dim3(128), 0, s, la);
    // dipoles differ from charges only in the source terms: the L2P and M2P kernels are the potential's
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_leaf<PB, LM>), dim3(nblk(T.n, 256), NV), dim3(256), 0, s, la);
    FMMHP_HIP(hipGetLastError());
    FMMHP_CHECK(mk_.mark(FMMHP_PHASE_NEAR, s));
    FMMHP_CHECK(mk_.mark(FMMHP_NUM_PHASES, s));
    FMMHP_CHECK(mk_.commit(S, s));
    return FMMHP_OK;
}

template <int MODE, int NV>
static fmmhp_status run_pass(const Tree &T, const Sched &S, const VecWs &ws, const double *q, const PassOut &out,
                             hipStream_t s) {
    switch (S.PB) {
        case 5: return eval_pass<5, MODE, NV>(T, S, ws, q, out, s);
        case 10: return eval_pass<10, MODE, NV>(T, S, ws, q, out, s);
        case 15: return eval_pass<15, MODE, NV>(T, S, ws, q, out, s);
        case 20: return eval_pass<20, MODE, NV>(T, S, ws, q, out, s);
        case 25: return eval_pass<25, MODE, NV>(T, S, ws, q, out, s);
        case 30: return eval_pass<30, MODE, NV>(T, S, ws, q, out, s);
        case 35: return eval_pass<35, MODE, NV>(T, S, ws, q, out, s);
        case 40: return eval_pass<40, MODE, NV>(T, S, ws, q, out, s);
        default:
            set_error("internal: no kernels compiled for p = %d", S.PB);
            return FMMHP_EUNSUPPORTED;
    }
}


// Per-vector workspace (multipoles, locals, sorted charges, near-field sums, surface sums) for nv
// vectors at once; grown on demand, owned by the plan.
static fmmhp_status ensure_vec_ws(Arena &A, const Tree &T, Sched &S, int nv) {
    VecWs &w = S.ws;
    if (w.cap >= nv) return FMMHP_OK;
    const size_t nb = (size_t)T.nbox, P1 = (size_t)S.PB + 1;
    FMMHP_CHECK(A.alloc_n(&w.W, nv * P1 * nb, "multipoles"));
    FMMHP_CHECK(A.alloc_n(&w.Lam, nv * (size_t)S.nloc * P1 * nb, "locals"));
    FMMHP_CHECK(A.alloc_n(&w.qs, nv * (size_t)T.n, "sorted charges"));
    FMMHP_CHECK(A.alloc_n(&w.near, nv * (size_t)T.n, "near-field sums"));
    FMMHP_CHECK(A.alloc_n(&w.red, nv * (size_t)S.n_rch, "surface partial sums"));
    FMMHP_CHECK(A.alloc_n(&w.rank1, nv * (size_t)T.n_inst, "surface sums"));
    if (S.m2l_fp32) FMMHP_CHECK(A.alloc_n(&w.Wf, nv * nb * (size_t)m2l32_kp(S.PB), "FP32 M2L source rows"));
    w.part = nullptr;  // the symmetric walk's partial sums come with the walk (ensure_sym_part)
    w.cap = nv;
    return FMMHP_OK;
}

// Partial sums of the symmetric near-field walk for the plan's workspace, allocated when the walk is
// in use (walk 3 or 4 on a plan whose lists allow it).
static fmmhp_status ensure_sym_part(Arena &A, Sched &S) {
    if (!((S.near_walk == 3 || S.near_walk == 4) && S.sym_ok) || S.ws.part) return FMMHP_OK;
    return A.alloc_n(&S.ws.part, (size_t)S.ws.cap * S.sym_npart, "near-field pair partial sums");
}

static fmmhp_status enqueue_eval(const Tree &T, const Sched &S, int nvec, const double *q, double *phi,
                                 hipStream_t s) {
    int v = 0;
    for (; v + kVecChunk <= nvec; v += kVecChunk) {
        PassOut o;
        o.phi = phi + (int64_t)v * 2 * T.n;
        FMMHP_CHECK((run_pass<kPhi, kVecChunk>(T, S, S.ws, q + (int64_t)v * T.n, o, s)));
    }
    for (; v < nvec; ++v) {
        PassOut o;
        o.phi = phi + (int64_t)v * 2 * T.n;
        FMMHP_CHECK((run_pass<kPhi, 1>(T, S, S.ws, q + (int64_t)v * T.n, o, s)));
    }
    return FMMHP_OK;
}

// ---------------------------------------------------------------------------------------------
// Evaluation without allocation (fmmhp_eval_noalloc).  The per-vector workspace of each pass is
// carved from a file-scope device array instead of the plan's arena.  Host code never uses the
// array's name as an address: hipGetSymbolAddress gives its address on each device once, and that
// pointer is what the kernels receive.  Every evaluation fully overwrites the workspace it reads
// (P2M and M2M write every multipole, the M2L writes the locals of every box of levels >= 2 and
// level 1 is cleared, the near-field and surface kernels write every sum), so nothing needs clearing
// between calls.  Calls that overlap on one device share the array and race.
// ---------------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Address of the scratch array on device dev (the current device), looked up once per device.
static fmmhp_status scratch_on(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d outside the no-allocation scratch table (0..%d)", dev, kMaxDevices - 1);
        return FMMHP_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error("hipGetSymbolAddress of the no-allocation scratch failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return FMMHP_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = (unsigned char *)g_scratch_ptr[dev];
    return FMMHP_OK;
}

// Bytes of a pass workspace for nv vectors (each array aligned to 256 bytes); carves it from base
// when base is given.
static size_t vec_ws_layout(const Tree &T, const Sched &S, int nv, unsigned char *base, VecWs *w) {
    const size_t nb = (size_t)T.nbox, P1 = (size_t)S.PB + 1;
    const size_t sizes[8] = {nv * P1 * nb * sizeof(cplx), nv * (size_t)S.nloc * P1 * nb * sizeof(cplx),
                             nv * (size_t)T.n * sizeof(double), nv * (size_t)T.n * sizeof(double2),
                             nv * (size_t)S.n_rch * sizeof(cplx), nv * (size_t)T.n_inst * sizeof(cplx),
                             S.m2l_fp32 ? nv * nb * (size_t)m2l32_kp(S.PB) * sizeof(float) : 0,
                             S.sym_ok && (S.near_walk == 3 || S.near_walk == 4) ? nv * (size_t)S.sym_npart * sizeof(double) : 0};
    size_t off[8], at = 0;
    for (int k = 0; k < 8; ++k) {
        off[k] = at;
        at += (sizes[k] + 255) / 256 * 256;
    }
    if (base) {
        w->cap = nv;
        w->W = (cplx *)(base + off[0]);
        w->Lam = (cplx *)(base + off[1]);
        w->qs = (double *)(base + off[2]);
        w->near = (double2 *)(base + off[3]);
        w->red = (cplx *)(base + off[4]);
        w->rank1 = (cplx *)(base + off[5]);
        w->Wf = S.m2l_fp32 ? (float *)(base + off[6]) : nullptr;
        w->part = S.sym_ok && (S.near_walk == 3 || S.near_walk == 4) ? (double *)(base + off[7]) : nullptr;
    }
    return at;
}

fmmhp_status run_eval_noalloc(const Tree &T, const Sched &S, int device, int nvec, const double *q, double *phi,
                              hipStream_t s) {
    if (S.timing) {
        set_error("fmmhp_eval_noalloc: phase timing is on for this plan (its events would be created per call)");
        return FMMHP_ESTATE;
    }
    const size_t one = vec_ws_layout(T, S, 1, nullptr, nullptr);
    if (one > kNoAllocScratchBytes) {
        set_error("fmmhp_eval_noalloc: the plan needs %zu bytes of workspace per charge vector, more than the %zu "
                  "bytes of the no-allocation scratch",
                  one, (size_t)kNoAllocScratchBytes);
        return FMMHP_EINVAL;
    }
    unsigned char *base = nullptr;
    FMMHP_CHECK(scratch_on(device, &base));
    VecWs w1, w8;
    vec_ws_layout(T, S, 1, base, &w1);
    const bool wide = nvec >= kVecChunk && vec_ws_layout(T, S, kVecChunk, nullptr, nullptr) <= kNoAllocScratchBytes;
    if (wide) vec_ws_layout(T, S, kVecChunk, base, &w8);
    int v = 0;
    if (wide)
        for (; v + kVecChunk <= nvec; v += kVecChunk) {
            PassOut o;
            o.phi = phi + (int64_t)v * 2 * T.n;
            FMMHP_CHECK((run_pass<kPhi, kVecChunk>(T, S, w8, q + (int64_t)v * T.n, o, s)));
        }
    for (; v < nvec; ++v) {
        PassOut o;
        o.phi = phi + (int64_t)v * 2 * T.n;
        FMMHP_CHECK((run_pass<kPhi, 1>(T, S, w1, q + (int64_t)v * T.n, o, s)));
    }
    return FMMHP_OK;
}

fmmhp_status run_eval(Arena &A, const Tree &T, Sched &S, int nvec, const double *q, double *phi, hipStream_t s) {
    if (nvec >= kVecChunk) FMMHP_CHECK(ensure_vec_ws(A, T, S, kVecChunk));
    FMMHP_CHECK(ensure_sym_part(A, S));
    if (!S.use_graph || S.timing || s == nullptr) return enqueue_eval(T, S, nvec, q, phi, s);
    auto &G = S.graph;
    if (!(G.exec && G.q == q && G.phi == phi && G.nvec == nvec && G.stream == s)) {
        if (G.exec) {
            FMMHP_HIP(hipGraphExecDestroy(G.exec));
            G.exec = nullptr;
        }
        FMMHP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const fmmhp_status st = enqueue_eval(T, S, nvec, q, phi, s);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &graph);
        if (st != FMMHP_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        FMMHP_HIP(e);
        const hipError_t ei = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        FMMHP_HIP(ei);
        G.q = q;
        G.phi = phi;
        G.nvec = nvec;
        G.stream = s;
    }
    FMMHP_HIP(hipGraphLaunch(G.exec, s));
    return FMMHP_OK;
}

// ---------------------------------------------------------------------------------------------
// Complex charges: phi[q_re + i q_im] = phi[q_re] + i phi[q_im] (the operator is real-linear in the
// charges), evaluated as two real vectors and combined on the device.
// ---------------------------------------------------------------------------------------------
__global__ void k_split_complex(const double *__restrict__ q, int64_t n, double *__restrict__ qr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    qr[i] = q[2 * i];
    qr[n + i] = q[2 * i + 1];
}

__global__ void k_combine_complex(const double *__restrict__ p2, int64_t n, double *__restrict__ phi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // p2 = [phi[q_re]; phi[q_im]], each [n][2]
    phi[2 * i] = p2[2 * i] - p2[2 * n + 2 * i + 1];
    phi[2 * i + 1] = p2[2 * i + 1] + p2[2 * n + 2 * i];
}

fmmhp_status run_eval_complex(Arena &A, const Tree &T, Sched &S, int nvec, const double *q, double *phi,
                              hipStream_t s) {
    if (!S.cq) {
        FMMHP_CHECK(A.alloc_n(&S.cq, (size_t)2 * T.n, "complex-charge split"));
        FMMHP_CHECK(A.alloc_n(&S.cphi, (size_t)4 * T.n, "complex-charge potentials"));
    }
    for (int v = 0; v < nvec; ++v) {
        hipLaunchKernelGGL(k_split_complex, dim3(nblk(T.n, 256)), dim3(256), 0, s, q + (int64_t)v * 2 * T.n, T.n,
                           S.cq);
        FMMHP_HIP(hipGetLastError());
        FMMHP_CHECK(run_eval(A, T, S, 2, S.cq, S.cphi, s));
        hipLaunchKernelGGL(k_combine_complex, dim3(nblk(T.n, 256)), dim3(256), 0, s, S.cphi, T.n,
                           phi + (int64_t)v * 2 * T.n);
        FMMHP_HIP(hipGetLastError());
    }
    return FMMHP_OK;
}

// ---------------------------------------------------------------------------------------------
// Double-layer potential: dipole densities with normals, one vector per pass (the kDip mode of the
// source kernels; every translation is shared with the potential).  Complex densities are split
// into two real vectors as for complex charges.
// ---------------------------------------------------------------------------------------------
__global__ void k_gather_nrm(const double *__restrict__ nx, const double *__restrict__ ny,
                             const int32_t *__restrict__ perm, int64_t n, double2 *__restrict__ nrm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i];
    nrm[i] = make_double2(nx[o], ny[o]);
}

fmmhp_status run_eval_dlp(Arena &A, const Tree &T, Sched &S, int nvec, const double *mu, int w, const double *nx,
                          const double *ny, double *phi, hipStream_t s) {
    if (!S.nrm) FMMHP_CHECK(A.alloc_n(&S.nrm, (size_t)T.n, "sorted normals"));
    hipLaunchKernelGGL(k_gather_nrm, dim3(nblk(T.n, 256)), dim3(256), 0, s, nx, ny, T.perm, T.n, S.nrm);
    FMMHP_HIP(hipGetLastError());
    if (w == 2 && !S.cq) {
        FMMHP_CHECK(A.alloc_n(&S.cq, (size_t)2 * T.n, "complex-charge split"));
        FMMHP_CHECK(A.alloc_n(&S.cphi, (size_t)4 * T.n, "complex-charge potentials"));
    }
    for (int v = 0; v < nvec; ++v) {
        if (w == 1) {
            PassOut o;
            o.phi = phi + (int64_t)v * 2 * T.n;
            FMMHP_CHECK((run_pass<kDip, 1>(T, S, S.ws, mu + (int64_t)v * T.n, o, s)));
            continue;
        }
        hipLaunchKernelGGL(k_split_complex, dim3(nblk(T.n, 256)), dim3(256), 0, s, mu + (int64_t)v * 2 * T.n, T.n,
                           S.cq);
        FMMHP_HIP(hipGetLastError());
        for (int h = 0; h < 2; ++h) {
            PassOut o;
            o.phi = S.cphi + (int64_t)h * 2 * T.n;
            FMMHP_CHECK((run_pass<kDip, 1>(T, S, S.ws, S.cq + (int64_t)h * T.n, o, s)));
        }
        hipLaunchKernelGGL(k_combine_complex, dim3(nblk(T.n, 256)), dim3(256), 0, s, S.cphi, T.n,
                           phi + (int64_t)v * 2 * T.n);
        FMMHP_HIP(hipGetLastError());
    }
    return FMMHP_OK;
}

// ---------------------------------------------------------------------------------------------
// Adjoint.  For a real loss l of the complex potential, with incoming g_i = dl/dRe phi_i +
// i dl/dIm phi_i (so l = sum_i Re(conj(g_i) phi_i) to first order) and c = conj(g):
//   dl/dq_j = Re Phi[c](r_j)                                  (G(r, r') = G(r', r), eq. (greensfunsymm))
//   dl/dx_k = Re D_x(k),  D_x(k) = c_k d_x Phi[q](r_k) + q_k d_x Phi[c](r_k)     (alike in y)
// with Phi[c](r) = sum_j c_j G(r, r_j).  Phi[c] = Phi[Re c] + i Phi[Im c] uses two real passes.
// The impedance gradient comes from the scale homogeneity of the Green's function: the two log
// terms are invariant under r -> s r in pairs and the reaction term depends on Z and the
// coordinates only through Z (y - i x), so G_Z(s r, s r') = G_{sZ}(r, r') up to (1/2pi) log s per
// skipped coincident pair, and
//   Z dl_c/dZ = sum_k [(x_k - x0) D_x(k) + y_k D_y(k)] - (1/2pi) sum_{r_i == r_j} c_i q_j,
// l_c = sum_i c_i phi_i, for any x0 (translation invariance in x; the root centre is used).
// dl/dZ is reported as dl/dRe Z + i dl/dIm Z = conj(dl_c/dZ) (phi is holomorphic in Z).
// ---------------------------------------------------------------------------------------------
// q3 = [q; Re conj(g); Im conj(g)], [3][n] caller order: the three charge vectors of the adjoint
__global__ void k_stack3(const double *__restrict__ q, const double *__restrict__ g, int64_t n,
                         double *__restrict__ q3) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o < n) {
        q3[o] = q[o];
        q3[n + o] = g[2 * o];
        q3[2 * n + o] = -g[2 * o + 1];
    }
}

struct BwdArgs {
    const InstInfo *ii;
    const PtChunk *ch;           // point chunks, each within one instance
    const double *xs, *ys;
    const int32_t *perm;
    const double *q3;            // [n][3] (q, Re c, Im c), c = conj(g), sorted
    const cplx *phr, *phi_i;     // Phi[Re c], Phi[Im c]            (sorted)
    const cplx *gxq, *gyq;       // grad Phi[q]                     (sorted)
    const cplx *gxr, *gyr, *gxi, *gyi;  // grad Phi[Re c], grad Phi[Im c] (sorted)
    const double *qc;            // sorted
    double *grad_q, *grad_x, *grad_y;
    cplx *part;                  // [n chunks] partial sums of the impedance identity
    int want_pos;
};

// One block per point chunk; the impedance identity is summed per instance (x0 = the instance's
// root centre).
__global__ __launch_bounds__(256) void k_bwd_combine(BwdArgs a) {
    const PtChunk ch = a.ch[blockIdx.x];
    const double x0 = a.ii[ch.inst].x_lo + 0.5 * a.ii[ch.inst].S;
    double ar = 0.0, ai = 0.0;
    // every input in sorted order (contiguous); only the gradients are scattered to caller order
    for (int64_t i = ch.start + threadIdx.x; i < ch.end; i += 256) {
        const int64_t o = a.perm[i];
        if (a.grad_q) a.grad_q[o] = a.phr[i].re - a.phi_i[i].im;
        if (!a.want_pos) continue;
        const cplx c = mk(a.q3[3 * i + 1], a.q3[3 * i + 2]);
        const double qv = a.q3[3 * i];
        const cplx gcx = a.gxr[i] + mul_ipow(a.gxi[i], 1);
        const cplx gcy = a.gyr[i] + mul_ipow(a.gyi[i], 1);
        const cplx Dx = c * a.gxq[i] + qv * gcx;
        const cplx Dy = c * a.gyq[i] + qv * gcy;
        if (a.grad_x) a.grad_x[o] = Dx.re;
        if (a.grad_y) a.grad_y[o] = Dy.re;
        const cplx v = (a.xs[i] - x0) * Dx + a.ys[i] * Dy - kInv2Pi * (a.qc[i] * c);
        ar += v.re;
        ai += v.im;
    }
    const cplx t = block_sum(mk(ar, ai));
    if (threadIdx.x == 0) a.part[blockIdx.x] = t;
}

static fmmhp_status ensure_bwd(Arena &A, const Tree &T, Sched &S) {
    if (S.bw.ready) return FMMHP_OK;
    const size_t n = (size_t)T.n;
    BwdWork &b = S.bw;
    FMMHP_CHECK(A.alloc_n(&b.q3, 3 * n, "adjoint charge vectors"));
    FMMHP_CHECK(A.alloc_n(&b.qc, n, "coincident charge sums"));
    cplx **bufs[] = {&b.phi3, &b.gx3, &b.gy3, &b.near_gx, &b.near_gy};
    for (cplx **pp : bufs) FMMHP_CHECK(A.alloc_n(pp, 3 * n, "adjoint fields"));
    FMMHP_CHECK(A.alloc_n(&b.red, (size_t)S.n_rch + T.n_inst, "adjoint reduction"));
    b.ready = true;
    return FMMHP_OK;
}

__global__ void k_zero_f64(double *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Clears n doubles with a kernel (safe under graph capture, unlike a memset node).
fmmhp_status zero_f64(double *p, int64_t n, hipStream_t s) {
    if (n <= 0) return FMMHP_OK;
    hipLaunchKernelGGL(k_zero_f64, dim3(nblk(n, 256)), dim3(256), 0, s, p, n);
    FMMHP_HIP(hipGetLastError());
    return FMMHP_OK;
}

// (dl/dRe Z_k, dl/dIm Z_k) = (Re, -Im) of zsum_k / Z_k per instance (the homogeneity sums of the adjoint)
__global__ void k_dl_dz(const cplx *__restrict__ zsum, const InstInfo *__restrict__ ii, int n_inst,
                        double *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_inst) return;
    const cplx d = zsum[k] * inv(ii[k].Z);
    out[2 * k] = d.re;
    out[2 * k + 1] = -d.im;
}

fmmhp_status run_backward(Arena &A, const Tree &T, Sched &S, const double *q, const double *g, double *grad_q,
                          double *grad_x, double *grad_y, cplx *zsum_host, double *dlz_dev, hipStream_t s) {
    FMMHP_CHECK(ensure_bwd(A, T, S));
    FMMHP_CHECK(ensure_vec_ws(A, T, S, 3));  // multipoles, locals, sums for the three vectors
    BwdWork &b = S.bw;
    const bool pos = grad_x || grad_y || zsum_host || dlz_dev;
    if (!pos && !grad_q) return FMMHP_OK;
    const int64_t n = T.n;
    hipLaunchKernelGGL(k_stack3, dim3(nblk(n, 256)), dim3(256), 0, s, q, g, n, b.q3);
    FMMHP_HIP(hipGetLastError());
    if (pos) {
        // one pass over the three vectors: potential and gradient, the near field shared by all three
        PassOut po;
        po.phi = (double *)b.phi3;
        po.gx = b.gx3;
        po.gy = b.gy3;
        po.qc = b.qc;
        po.sorted = true;
        FMMHP_CHECK((run_pass<kPhiGrad, 3>(T, S, S.ws, b.q3, po, s)));
    } else {
        // dl/dq only: the potentials of Re conj(g) and Im conj(g)
        for (int v = 1; v < 3; ++v) {
            PassOut po;
            po.phi = (double *)(b.phi3 + v * n);
            po.sorted = true;
            FMMHP_CHECK((run_pass<kPhi, 1>(T, S, S.ws, b.q3 + v * n, po, s)));
        }
    }
    // the pass left its charges sorted and interleaved in S.ws.qs: (q, Re c, Im c) per point
    BwdArgs ba{S.inst_info, S.rch,         T.xs,          T.ys,          T.perm,    S.ws.qs,
               b.phi3 + n,  b.phi3 + 2 * n, b.gx3,         b.gy3,         b.gx3 + n, b.gy3 + n,
               b.gx3 + 2 * n, b.gy3 + 2 * n, b.qc,         grad_q,        grad_x,    grad_y, b.red,
               pos ? 1 : 0};
    hipLaunchKernelGGL(k_bwd_combine, dim3(S.n_rch), dim3(256), 0, s, ba);
    FMMHP_HIP(hipGetLastError());
    if (zsum_host || dlz_dev) {
        hipLaunchKernelGGL(k_rank1_final, dim3(T.n_inst, 1), dim3(256), 0, s, b.red, S.n_rch, S.inst_ch, T.n_inst,
                           b.red + S.n_rch);
        FMMHP_HIP(hipGetLastError());
    }
    if (dlz_dev) {
        hipLaunchKernelGGL(k_dl_dz, dim3(nblk(T.n_inst, 256)), dim3(256), 0, s, b.red + S.n_rch, S.inst_info,
                           T.n_inst, dlz_dev);
        FMMHP_HIP(hipGetLastError());
    }
    if (zsum_host) {
        FMMHP_HIP(hipMemcpyAsync(zsum_host, b.red + S.n_rch, T.n_inst * sizeof(cplx), hipMemcpyDeviceToHost, s));
        FMMHP_HIP(hipStreamSynchronize(s));
    }
    return FMMHP_OK;
}

// Potential and gradient (d_x phi, d_y phi) of one real charge vector at every point, caller order:
// the forward pass in its gradient mode (the same expansions, differentiated in the target).
fmmhp_status run_field(Arena &A, const Tree &T, Sched &S, const double *q, double *phi, cplx *gx, cplx *gy,
                       hipStream_t s) {
    FMMHP_CHECK(ensure_bwd(A, T, S));  // near-field gradient sums
    PassOut po;
    po.phi = phi;
    po.gx = gx;
    po.gy = gy;
    return run_pass<kPhiGrad, 1>(T, S, S.ws, q, po, s);
}

fmmhp_status collect_phase_times(Sched &S) {
    if (!S.events) return FMMHP_OK;
    auto &ev = *S.events;
    // group: main-stream boundaries [0, NUM_PHASES], near pair, deep-M2L pair, k_m2l pairs
    const int G = FMMHP_NUM_PHASES + 9;
    for (size_t g0 = 0, gi = 0; g0 + G <= ev.size(); g0 += G, ++gi) {
        const size_t n0 = g0 + FMMHP_NUM_PHASES + 1, d0 = n0 + 2;
        FMMHP_HIP(hipEventSynchronize(ev[g0 + FMMHP_NUM_PHASES]));
        FMMHP_HIP(hipEventSynchronize(ev[n0 + 1]));
        FMMHP_HIP(hipEventSynchronize(ev[d0 + 1]));
        for (int k = 0; k < FMMHP_NUM_PHASES; ++k) {
            float ms = 0.f;
            if (k == FMMHP_PHASE_NEAR)
                FMMHP_HIP(hipEventElapsedTime(&ms, ev[n0], ev[n0 + 1]));
            else if (k < FMMHP_PHASE_NEAR)
                FMMHP_HIP(hipEventElapsedTime(&ms, ev[g0 + k], ev[g0 + k + 1]));
            if (k == FMMHP_PHASE_M2L) {
                float md = 0.f;
                FMMHP_HIP(hipEventElapsedTime(&md, ev[d0], ev[d0 + 1]));
                ms += md;
            }
            S.phase_ms[k] += ms;
        }
        S.timed_evals += 1;
        const size_t k0 = d0 + 2;
        for (int k = 0; k < 2; ++k) {
            FMMHP_HIP(hipEventSynchronize(ev[k0 + 2 * k + 1]));
            float ms = 0.f;
            FMMHP_HIP(hipEventElapsedTime(&ms, ev[k0 + 2 * k], ev[k0 + 2 * k + 1]));
            S.m2l_kernel_ms += ms;
        }
        S.m2l_launches += (*S.m2l_n)[gi];
    }
    for (auto e : ev) (void)hipEventDestroy(e);
    ev.clear();
    S.m2l_n->clear();
    return FMMHP_OK;
}

}  // namespace fmmhp
