// C-ABI entry points of libfmmhp (declared in include/fmmhp.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "internal.hpp"

namespace fmmhp {

static thread_local char g_msg[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
}

constexpr uint64_t kMagic = 0x66'6d'6d'68'70'6c'61'6eull;  // "fmmhplan"
constexpr uint64_t kDead = 0xdeadull;

static fmmhp_status check_plan(fmmhp_plan_t p) {
    if (!p) {
        set_error("plan is NULL");
        return FMMHP_ESTATE;
    }
    if (p->magic != kMagic) {
        set_error("plan handle is not a live plan (destroyed or corrupted)");
        return FMMHP_ESTATE;
    }
    int dev = -1;
    FMMHP_HIP(hipGetDevice(&dev));
    if (dev != p->device) {
        set_error("plan was created on device %d but device %d is current", p->device, dev);
        return FMMHP_EINVAL;
    }
    return FMMHP_OK;
}

// Dirichlet and Neumann plans ignore the impedance.
static bool no_impedance(const fmmhp_opts *opts) {
    return opts && (opts->flags & (FMMHP_FLAG_DIRICHLET | FMMHP_FLAG_NEUMANN)) != 0;
}

static fmmhp_status check_impedance(double re, double im) {
    if (!isfinite(re) || !isfinite(im)) {
        set_error("impedance is not finite");
        return FMMHP_EINVAL;
    }
    if (!(re > 0.0) || im < 0.0) {
        set_error("impedance %g%+gi is outside Re > 0, Im >= 0", re, im);
        return FMMHP_EDOMAIN;
    }
    return FMMHP_OK;
}

}  // namespace fmmhp

using namespace fmmhp;

extern "C" {

const char *fmmhp_status_string(fmmhp_status s) {
    switch (s) {
        case FMMHP_OK: return "FMMHP_OK";
        case FMMHP_EINVAL: return "FMMHP_EINVAL";
        case FMMHP_EDOMAIN: return "FMMHP_EDOMAIN";
        case FMMHP_ENOMEM: return "FMMHP_ENOMEM";
        case FMMHP_EHIP: return "FMMHP_EHIP";
        case FMMHP_ESTATE: return "FMMHP_ESTATE";
        case FMMHP_EUNSUPPORTED: return "FMMHP_EUNSUPPORTED";
        default: return "unknown status";
    }
}

const char *fmmhp_last_error_message(void) { return g_msg; }

// Shared by the plain and batched plan builders: n_inst instances, point ranges off[0..n_inst].
static fmmhp_status create_plan(int n_inst, const int64_t *off, const double *x, const double *y,
                                const double *img_x, const double *img_y, int64_t src_end, const cplx *Zs,
                                const fmmhp_opts *opts, hipStream_t stream, fmmhp_plan_t *plan_out) {
    const int lb = n_inst == 1 ? kLBits : kLBitsForest;
    fmmhp_opts o{20, 40, lb, 0, 0, 0};
    if (opts) o = *opts;
    if (o.max_level == 0) o.max_level = lb;
    if (o.p < 1 || o.p > FMMHP_MAX_P || o.leaf_size < 1 || o.max_level < 1 || o.max_level > lb ||
        (o.flags & ~(FMMHP_FLAG_GRAPH | FMMHP_FLAG_M2L_FP32 | FMMHP_FLAG_DIRICHLET | FMMHP_FLAG_NEUMANN |
                     FMMHP_FLAG_SERIAL | FMMHP_FLAG_M2L_VECTOR | FMMHP_FLAG_M2L_MFMA)) != 0 ||
        (o.flags & FMMHP_FLAG_DIRICHLET && o.flags & FMMHP_FLAG_NEUMANN) ||
        (o.flags & FMMHP_FLAG_M2L_VECTOR && o.flags & FMMHP_FLAG_M2L_MFMA) || o.near_walk < 0 || o.near_walk > 4 ||
        o.near_groups < 0 || o.near_groups > 16) {
        set_error("options out of range: p=%d (1..%d), leaf_size=%d (>=1), max_level=%d (1..%d), flags=%u (FMMHP_FLAG_* bits, "
                  "not both DIRICHLET and NEUMANN, not both M2L_VECTOR and M2L_MFMA), "
                  "near_walk=%d (0..4), near_groups=%d (0..16)",
                  o.p, FMMHP_MAX_P, o.leaf_size, o.max_level, lb, o.flags, o.near_walk, o.near_groups);
        return FMMHP_EINVAL;
    }
    fmmhp_plan_s *p = new (std::nothrow) fmmhp_plan_s();
    if (!p) {
        set_error("host allocation of the plan failed");
        return FMMHP_ENOMEM;
    }
    p->magic = kMagic;
    p->p_req = o.p;
    p->leaf_size = o.leaf_size;
    p->max_level = o.max_level;
    p->lambda_re = Zs[0].re;
    p->lambda_im = Zs[0].im;
    p->Zs.assign(Zs, Zs + n_inst);
    fmmhp_status st = FMMHP_OK;
    if (hipGetDevice(&p->device) != hipSuccess) {
        set_error("hipGetDevice failed");
        st = FMMHP_EHIP;
    }
    if (st == FMMHP_OK)
        st = build_tree(p->arena, p->tree, n_inst, off, x, y, img_x, img_y, src_end, o.leaf_size, o.max_level,
                        stream);
    p->sched.m2l_fp32 = (o.flags & FMMHP_FLAG_M2L_FP32) != 0;
    p->sched.serial = (o.flags & FMMHP_FLAG_SERIAL) != 0;
    p->sched.m2l_form = (o.flags & FMMHP_FLAG_M2L_VECTOR) ? 1 : (o.flags & FMMHP_FLAG_M2L_MFMA) ? 2 : 0;
    p->sched.bc = (o.flags & FMMHP_FLAG_DIRICHLET) ? 1 : (o.flags & FMMHP_FLAG_NEUMANN) ? 2 : 0;
    if (st == FMMHP_OK) st = build_schedule(p->arena, p->tree, p->sched, pick_bucket(o.p), Zs, stream);
    if (st == FMMHP_OK) st = apply_launch_shape(p->arena, p->tree, p->sched, o.near_walk, o.near_groups, stream);
    p->sched.use_graph = (o.flags & FMMHP_FLAG_GRAPH) != 0;
    if (st == FMMHP_OK) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            set_error("plan build failed on the device: %s", hipGetErrorString(e));
            st = FMMHP_EHIP;
        }
    }
    if (st != FMMHP_OK) {
        (void)hipStreamSynchronize(stream);
        if (p->sched.ev_fork) (void)hipEventDestroy(p->sched.ev_fork);
        if (p->sched.ev_join) (void)hipEventDestroy(p->sched.ev_join);
        if (p->sched.ev_up) (void)hipEventDestroy(p->sched.ev_up);

        if (p->sched.side) (void)hipStreamDestroy(p->sched.side);
        if (p->sched.side2) (void)hipStreamDestroy(p->sched.side2);
        if (p->sched.ev_deep_ready) (void)hipEventDestroy(p->sched.ev_deep_ready);
        if (p->sched.ev_deep_done) (void)hipEventDestroy(p->sched.ev_deep_done);
        p->arena.release();
        p->magic = kDead;
        delete p;
        return st;
    }
    *plan_out = p;
    return FMMHP_OK;
}

fmmhp_status fmmhp_plan_create(int64_t n, const double *x, const double *y, const double *img_x,
                               const double *img_y, double lambda_re, double lambda_im, const fmmhp_opts *opts,
                               hipStream_t stream, fmmhp_plan_t *plan_out) {
    g_msg[0] = 0;
    if (!plan_out) {
        set_error("plan_out is NULL");
        return FMMHP_EINVAL;
    }
    *plan_out = nullptr;
    if (n < 1 || n >= ((int64_t)1 << 31)) {
        set_error("n = %lld outside [1, 2^31)", (long long)n);
        return FMMHP_EINVAL;
    }
    if (!x || !y) {
        set_error("x or y is NULL");
        return FMMHP_EINVAL;
    }
    if ((img_x == nullptr) != (img_y == nullptr)) {
        set_error("img_x and img_y must both be NULL or both be given");
        return FMMHP_EINVAL;
    }
    if (!no_impedance(opts)) FMMHP_CHECK(check_impedance(lambda_re, lambda_im));
    const int64_t off[2] = {0, n};
    const cplx Z = no_impedance(opts) ? mk(1.0, 0.0) : mk(lambda_re, lambda_im);
    return create_plan(1, off, x, y, img_x, img_y, n, &Z, opts, stream, plan_out);
}

fmmhp_status fmmhp_plan_create_targets(int64_t n_src, const double *xs, const double *ys, int64_t n_tgt,
                                       const double *xt, const double *yt, double lambda_re, double lambda_im,
                                       const fmmhp_opts *opts, hipStream_t stream, fmmhp_plan_t *plan_out) {
    g_msg[0] = 0;
    if (!plan_out) {
        set_error("plan_out is NULL");
        return FMMHP_EINVAL;
    }
    *plan_out = nullptr;
    if (n_src < 1 || n_tgt < 1 || n_src + n_tgt >= ((int64_t)1 << 31)) {
        set_error("n_src = %lld, n_tgt = %lld: both >= 1 and their sum < 2^31", (long long)n_src,
                  (long long)n_tgt);
        return FMMHP_EINVAL;
    }
    if (!xs || !ys || !xt || !yt) {
        set_error("xs, ys, xt and yt must be non-NULL");
        return FMMHP_EINVAL;
    }
    if (!no_impedance(opts)) FMMHP_CHECK(check_impedance(lambda_re, lambda_im));
    // one point set: the sources, then the targets (the tree is built over both)
    const int64_t n = n_src + n_tgt;
    double *xy = nullptr;
    if (hipMalloc(&xy, 2 * (size_t)n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation of %lld bytes for the combined points failed", (long long)(16 * n));
        return FMMHP_ENOMEM;
    }
    fmmhp_status st = FMMHP_OK;
    const hipMemcpyKind d2d = hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(xy, xs, n_src * sizeof(double), d2d, stream) != hipSuccess ||
        hipMemcpyAsync(xy + n_src, xt, n_tgt * sizeof(double), d2d, stream) != hipSuccess ||
        hipMemcpyAsync(xy + n, ys, n_src * sizeof(double), d2d, stream) != hipSuccess ||
        hipMemcpyAsync(xy + n + n_src, yt, n_tgt * sizeof(double), d2d, stream) != hipSuccess) {
        set_error("copy of the points failed");
        st = FMMHP_EHIP;
    }
    const int64_t off[2] = {0, n};
    const cplx Z = no_impedance(opts) ? mk(1.0, 0.0) : mk(lambda_re, lambda_im);
    if (st == FMMHP_OK) st = create_plan(1, off, xy, xy + n, nullptr, nullptr, n_src, &Z, opts, stream, plan_out);
    (void)hipStreamSynchronize(stream);
    (void)hipFree(xy);
    if (st == FMMHP_OK) (*plan_out)->n_src = n_src;
    return st;
}

fmmhp_status fmmhp_batch_plan_create(int n_inst, const int64_t *offsets, const double *x, const double *y,
                                     const double *lambda, const fmmhp_opts *opts, hipStream_t stream,
                                     fmmhp_plan_t *plan_out) {
    g_msg[0] = 0;
    if (!plan_out) {
        set_error("plan_out is NULL");
        return FMMHP_EINVAL;
    }
    *plan_out = nullptr;
    if (n_inst < 1 || n_inst > kMaxInstances) {
        set_error("n_inst = %d outside [1, %d]", n_inst, kMaxInstances);
        return FMMHP_EINVAL;
    }
    if (!offsets || !x || !y || !lambda) {
        set_error("offsets, x, y and lambda must be non-NULL");
        return FMMHP_EINVAL;
    }
    if (offsets[0] != 0) {
        set_error("offsets[0] must be 0");
        return FMMHP_EINVAL;
    }
    for (int k = 0; k < n_inst; ++k)
        if (offsets[k + 1] <= offsets[k]) {
            set_error("instance %d is empty or offsets decrease", k);
            return FMMHP_EINVAL;
        }
    if (offsets[n_inst] >= ((int64_t)1 << 31)) {
        set_error("total point count %lld outside [1, 2^31)", (long long)offsets[n_inst]);
        return FMMHP_EINVAL;
    }
    std::vector<cplx> Zs(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        if (no_impedance(opts)) {
            Zs[k] = mk(1.0, 0.0);
            continue;
        }
        FMMHP_CHECK(check_impedance(lambda[2 * k], lambda[2 * k + 1]));
        Zs[k] = mk(lambda[2 * k], lambda[2 * k + 1]);
    }
    return create_plan(n_inst, offsets, x, y, nullptr, nullptr, offsets[n_inst], Zs.data(), opts, stream, plan_out);
}

// q [nv][n_src][w] -> qp [nv][n][w] (zero charges on the target-only points)
__global__ void k_pad_charges(const double *__restrict__ q, int64_t ns, int64_t n, int w, int nv,
                              double *__restrict__ qp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * w) return;
    for (int v = 0; v < nv; ++v) qp[(int64_t)v * n * w + i] = i < ns * w ? q[(int64_t)v * ns * w + i] : 0.0;
}

// pp [nv][n][2] -> phi [nv][n - ns][2] (the targets' potentials)
__global__ void k_take_targets(const double *__restrict__ pp, int64_t ns, int64_t n, int nv, double *__restrict__ phi) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nt = n - ns;
    if (t >= 2 * nt) return;
    for (int v = 0; v < nv; ++v) phi[(int64_t)v * 2 * nt + t] = pp[(int64_t)v * 2 * n + 2 * ns + t];
}

// Evaluation on a plan with separate targets: charges padded to all tree points, potentials of
// the targets kept.  w = 1 (real charges) or 2 (complex).
static fmmhp_status eval_targets(fmmhp_plan_t plan, int n_vec, const double *q, double *phi, int w,
                                 hipStream_t stream) {
    const int64_t n = plan->tree.n, ns = plan->n_src;
    if (plan->pad_cap < n_vec) {
        FMMHP_CHECK(plan->arena.alloc_n(&plan->qpad, (size_t)n_vec * n * 2, "padded charges"));
        FMMHP_CHECK(plan->arena.alloc_n(&plan->phipad, (size_t)n_vec * n * 2, "potentials at all points"));
        plan->pad_cap = n_vec;
    }
    const unsigned nb = (unsigned)((n * w + 255) / 256);
    hipLaunchKernelGGL(k_pad_charges, dim3(nb), dim3(256), 0, stream, q, ns, n, w, n_vec, plan->qpad);
    FMMHP_HIP(hipGetLastError());
    if (w == 1)
        FMMHP_CHECK(run_eval(plan->arena, plan->tree, plan->sched, n_vec, plan->qpad, plan->phipad, stream));
    else
        FMMHP_CHECK(run_eval_complex(plan->arena, plan->tree, plan->sched, n_vec, plan->qpad, plan->phipad, stream));
    hipLaunchKernelGGL(k_take_targets, dim3((unsigned)((2 * (n - ns) + 255) / 256)), dim3(256), 0, stream,
                       plan->phipad, ns, n, n_vec, phi);
    FMMHP_HIP(hipGetLastError());
    return FMMHP_OK;
}

fmmhp_status fmmhp_eval(fmmhp_plan_t plan, int n_vec, const double *q, double *phi, hipStream_t stream) {
    FMMHP_CHECK(check_plan(plan));
    if (n_vec < 1 || !q || !phi) {
        set_error("n_vec must be >= 1 and q, phi non-NULL");
        return FMMHP_EINVAL;
    }
    if (plan->n_src > 0) return eval_targets(plan, n_vec, q, phi, 1, stream);
    return run_eval(plan->arena, plan->tree, plan->sched, n_vec, q, phi, stream);
}

fmmhp_status fmmhp_eval_noalloc(fmmhp_plan_t plan, int n_vec, const double *q, double *phi, hipStream_t stream) {
    FMMHP_CHECK(check_plan(plan));
    if (n_vec < 1 || !q || !phi) {
        set_error("n_vec must be >= 1 and q, phi non-NULL");
        return FMMHP_EINVAL;
    }
    if (plan->n_src > 0) {
        set_error("fmmhp_eval_noalloc: plans with separate targets are not supported");
        return FMMHP_EUNSUPPORTED;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) {
        (void)hipGetLastError();
        set_error("fmmhp_eval_noalloc: the plan's device %d is not the current device (%d)", plan->device, dev);
        return FMMHP_ESTATE;
    }
    return run_eval_noalloc(plan->tree, plan->sched, dev, n_vec, q, phi, stream);
}

fmmhp_status fmmhp_eval_complex(fmmhp_plan_t plan, int n_vec, const double *q, double *phi, hipStream_t stream) {
    FMMHP_CHECK(check_plan(plan));
    if (n_vec < 1 || !q || !phi) {
        set_error("n_vec must be >= 1 and q, phi non-NULL");
        return FMMHP_EINVAL;
    }
    if (plan->n_src > 0) return eval_targets(plan, n_vec, q, phi, 2, stream);
    return run_eval_complex(plan->arena, plan->tree, plan->sched, n_vec, q, phi, stream);
}

fmmhp_status fmmhp_eval_double_layer(fmmhp_plan_t plan, int n_vec, const double *mu, int mu_complex,
                                     const double *nx, const double *ny, double *phi, hipStream_t stream) {
    FMMHP_CHECK(check_plan(plan));
    if (n_vec < 1 || !mu || !nx || !ny || !phi || (mu_complex != 0 && mu_complex != 1)) {
        set_error("n_vec must be >= 1, mu_complex 0 or 1 and mu, nx, ny, phi non-NULL");
        return FMMHP_EINVAL;
    }
    const int w = mu_complex ? 2 : 1;
    if (plan->n_src == 0)
        return run_eval_dlp(plan->arena, plan->tree, plan->sched, n_vec, mu, w, nx, ny, phi, stream);
    // separate targets: densities and normals padded with zeros to all tree points
    const int64_t n = plan->tree.n, ns = plan->n_src;
    if (plan->pad_cap < n_vec) {
        FMMHP_CHECK(plan->arena.alloc_n(&plan->qpad, (size_t)n_vec * n * 2, "padded charges"));
        FMMHP_CHECK(plan->arena.alloc_n(&plan->phipad, (size_t)n_vec * n * 2, "potentials at all points"));
        plan->pad_cap = n_vec;
    }
    if (!plan->npad) FMMHP_CHECK(plan->arena.alloc_n(&plan->npad, (size_t)2 * n, "padded normals"));
    hipLaunchKernelGGL(k_pad_charges, dim3((unsigned)((n * w + 255) / 256)), dim3(256), 0, stream, mu, ns, n, w, n_vec,
                       plan->qpad);
    hipLaunchKernelGGL(k_pad_charges, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, nx, ns, n, 1, 1,
                       plan->npad);
    hipLaunchKernelGGL(k_pad_charges, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, ny, ns, n, 1, 1,
                       plan->npad + n);
    FMMHP_HIP(hipGetLastError());
    FMMHP_CHECK(run_eval_dlp(plan->arena, plan->tree, plan->sched, n_vec, plan->qpad, w, plan->npad, plan->npad + n,
                             plan->phipad, stream));
    hipLaunchKernelGGL(k_take_targets, dim3((unsigned)((2 * (n - ns) + 255) / 256)), dim3(256), 0, stream,
                       plan->phipad, ns, n, n_vec, phi);
    FMMHP_HIP(hipGetLastError());
    return FMMHP_OK;
}

// pp [n][2] -> out [n - ns][2] (one vector)
__global__ void k_take_targets2(const double *__restrict__ pp, int64_t ns, int64_t n, double *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * (n - ns)) return;
    out[t] = pp[2 * ns + t];
}

fmmhp_status fmmhp_eval_field(fmmhp_plan_t plan, const double *q, double *phi, double *grad_x, double *grad_y,
                              hipStream_t stream) {
    FMMHP_CHECK(check_plan(plan));
    if (!q || !phi || !grad_x || !grad_y) {
        set_error("q, phi, grad_x and grad_y must be non-NULL");
        return FMMHP_EINVAL;
    }
    if (plan->n_src == 0)
        return run_field(plan->arena, plan->tree, plan->sched, q, phi, (cplx *)grad_x, (cplx *)grad_y, stream);
    // separate targets: charges padded to all tree points, the targets' values kept
    const int64_t n = plan->tree.n, ns = plan->n_src;
    if (plan->pad_cap < 1) {
        FMMHP_CHECK(plan->arena.alloc_n(&plan->qpad, (size_t)n * 2, "padded charges"));
        FMMHP_CHECK(plan->arena.alloc_n(&plan->phipad, (size_t)n * 2, "potentials at all points"));
        plan->pad_cap = 1;
    }
    if (!plan->gpad) FMMHP_CHECK(plan->arena.alloc_n(&plan->gpad, (size_t)n * 4, "gradients at all points"));
    hipLaunchKernelGGL(k_pad_charges, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, q, ns, n, 1, 1,
                       plan->qpad);
    FMMHP_HIP(hipGetLastError());
    FMMHP_CHECK(run_field(plan->arena, plan->tree, plan->sched, plan->qpad, plan->phipad, (cplx *)plan->gpad,
                          (cplx *)(plan->gpad + 2 * n), stream));
    const dim3 g((unsigned)((2 * (n - ns) + 255) / 256));
    hipLaunchKernelGGL(k_take_targets2, g, dim3(256), 0, stream, plan->phipad, ns, n, phi);
    hipLaunchKernelGGL(k_take_targets2, g, dim3(256), 0, stream, plan->gpad, ns, n, grad_x);
    hipLaunchKernelGGL(k_take_targets2, g, dim3(256), 0, stream, plan->gpad + 2 * n, ns, n, grad_y);
    FMMHP_HIP(hipGetLastError());
    return FMMHP_OK;
}

// dphi[i] = nx[i] g[0][i] + ny[i] g[1][i] (complex, [n][2])
__global__ void k_normal_combine(const double *__restrict__ gx, const double *__restrict__ gy,
                                 const double *__restrict__ nx, const double *__restrict__ ny, int64_t n,
                                 double *__restrict__ dphi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dphi[2 * i] = fma(nx[i], gx[2 * i], ny[i] * gy[2 * i]);
    dphi[2 * i + 1] = fma(nx[i], gx[2 * i + 1], ny[i] * gy[2 * i + 1]);
}

fmmhp_status fmmhp_eval_normal_derivative(fmmhp_plan_t plan, const double *q, const double *nx, const double *ny,
                                          double *dphi, hipStream_t stream) {
    FMMHP_CHECK(check_plan(plan));
    if (!q || !nx || !ny || !dphi) {
        set_error("q, nx, ny and dphi must be non-NULL");
        return FMMHP_EINVAL;
    }
    const int64_t nt = plan->tree.n - plan->n_src;
    if (!plan->ndwork) FMMHP_CHECK(plan->arena.alloc_n(&plan->ndwork, (size_t)6 * nt, "normal-derivative workspace"));
    double *w = plan->ndwork;
    FMMHP_CHECK(fmmhp_eval_field(plan, q, w, w + 2 * nt, w + 4 * nt, stream));
    hipLaunchKernelGGL(k_normal_combine, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, stream, w + 2 * nt,
                       w + 4 * nt, nx, ny, nt, dphi);
    FMMHP_HIP(hipGetLastError());
    return FMMHP_OK;
}

fmmhp_status fmmhp_backward(fmmhp_plan_t plan, const double *q, const double *grad_phi, double *grad_q,
                            double *grad_x, double *grad_y, double *grad_lambda, hipStream_t stream) {
    FMMHP_CHECK(check_plan(plan));
    if (!q || !grad_phi) {
        set_error("q and grad_phi must be non-NULL");
        return FMMHP_EINVAL;
    }
    if (plan->n_src > 0) {
        set_error("fmmhp_backward is not available for plans with separate targets");
        return FMMHP_EUNSUPPORTED;
    }
    std::vector<cplx> zsum(plan->tree.n_inst, mk(0.0, 0.0));
    // Dirichlet and Neumann kernels do not depend on an impedance: its gradient is zero
    const bool want_z = grad_lambda && plan->sched.bc == 0;
    FMMHP_CHECK(run_backward(plan->arena, plan->tree, plan->sched, q, grad_phi, grad_q, grad_x, grad_y,
                             want_z ? zsum.data() : nullptr, nullptr, stream));
    if (grad_lambda) {
        // per instance: dl_c/dZ_k = zsum_k / Z_k;  (dl/dRe Z_k, dl/dIm Z_k) = (Re, -Im) of it
        for (int k = 0; k < plan->tree.n_inst; ++k) {
            const cplx d = zsum[k] * inv(plan->Zs[k]);
            grad_lambda[2 * k] = d.re;
            grad_lambda[2 * k + 1] = -d.im;
        }
    }
    return FMMHP_OK;
}

fmmhp_status fmmhp_backward_device(fmmhp_plan_t plan, const double *q, const double *grad_phi, double *grad_q,
                                   double *grad_x, double *grad_y, double *grad_lambda, hipStream_t stream) {
    FMMHP_CHECK(check_plan(plan));
    if (!q || !grad_phi) {
        set_error("q and grad_phi must be non-NULL");
        return FMMHP_EINVAL;
    }
    if (plan->n_src > 0) {
        set_error("fmmhp_backward_device is not available for plans with separate targets");
        return FMMHP_EUNSUPPORTED;
    }
    if (grad_lambda && plan->sched.bc != 0) {
        // Dirichlet and Neumann kernels do not depend on an impedance: its gradient is zero
        FMMHP_CHECK(zero_f64(grad_lambda, 2 * (int64_t)plan->tree.n_inst, stream));
        grad_lambda = nullptr;
    }
    return run_backward(plan->arena, plan->tree, plan->sched, q, grad_phi, grad_q, grad_x, grad_y, nullptr,
                        grad_lambda, stream);
}

fmmhp_status fmmhp_plan_info(fmmhp_plan_t plan, fmmhp_plan_stats *st) {
    FMMHP_CHECK(check_plan(plan));
    if (!st) {
        set_error("stats is NULL");
        return FMMHP_EINVAL;
    }
    const Tree &T = plan->tree;
    memset(st, 0, sizeof(*st));
    st->n = T.n;
    st->p = plan->sched.PB;
    st->leaf_size = plan->leaf_size;
    st->max_level = plan->max_level;
    st->depth = T.depth;
    st->nbox = T.nbox;
    st->nleaf = T.nleaf;
    for (int k = 0; k < 4; ++k) st->list_len[k] = T.len[k];
    st->x_lo = T.x_lo;
    st->S = T.S;
    st->scale = T.scale;
    st->lambda_re = plan->lambda_re;
    st->lambda_im = plan->lambda_im;
    st->real_impedance = plan->sched.real_Z ? 1 : 0;
    st->device_bytes = plan->arena.bytes;
    st->n_inst = T.n_inst;
    st->n_sources = plan->n_src > 0 ? plan->n_src : T.n;
    st->near_walk = plan->sched.near_walk;
    st->near_groups = (int32_t)(plan->sched.near_blocks / std::max(1, plan->sched.cus));
    for (int k = 0; k < 2; ++k) {
        st->p2p_pairs[k] = plan->sched.p2p_pairs[k];
        st->m2l_pairs[k] = plan->sched.m2l_pairs[k];
    }
    return FMMHP_OK;
}

fmmhp_status fmmhp_plan_set_timing(fmmhp_plan_t plan, int enable) {
    FMMHP_CHECK(check_plan(plan));
    Sched &S = plan->sched;
    if (!S.events) {
        S.events = new (std::nothrow) std::vector<hipEvent_t>();
        S.m2l_n = new (std::nothrow) std::vector<int>();
        if (!S.events || !S.m2l_n) {
            set_error("host allocation failed");
            return FMMHP_ENOMEM;
        }
    }
    FMMHP_CHECK(collect_phase_times(S));
    for (double &v : S.phase_ms) v = 0.0;
    S.timed_evals = 0;
    S.m2l_kernel_ms = 0.0;
    S.m2l_launches = 0;
    S.timing = enable != 0;
    return FMMHP_OK;
}

fmmhp_status fmmhp_plan_phase_times(fmmhp_plan_t plan, double *ms, int64_t *n_evals) {
    FMMHP_CHECK(check_plan(plan));
    if (!ms) {
        set_error("ms is NULL");
        return FMMHP_EINVAL;
    }
    FMMHP_CHECK(collect_phase_times(plan->sched));
    for (int k = 0; k < FMMHP_NUM_PHASES; ++k) ms[k] = plan->sched.phase_ms[k];
    if (n_evals) *n_evals = plan->sched.timed_evals;
    return FMMHP_OK;
}

fmmhp_status fmmhp_plan_m2l_kernel_times(fmmhp_plan_t plan, double *ms, int64_t *n_launches) {
    FMMHP_CHECK(check_plan(plan));
    if (!ms) {
        set_error("ms is NULL");
        return FMMHP_EINVAL;
    }
    FMMHP_CHECK(collect_phase_times(plan->sched));
    *ms = plan->sched.m2l_kernel_ms;
    if (n_launches) *n_launches = plan->sched.m2l_launches;
    return FMMHP_OK;
}

fmmhp_status fmmhp_plan_export_tree(fmmhp_plan_t plan, int32_t *level, int32_t *bx, int32_t *by, int32_t *first,
                                    int32_t *count, int32_t *parent, int32_t *leaf, int32_t *child_first,
                                    int32_t *nchild, int64_t *perm, int64_t *u_off, int32_t *u_ent, int64_t *v_off,
                                    int32_t *v_ent, int64_t *w_off, int32_t *w_ent, int64_t *x_off,
                                    int32_t *x_ent) {
    FMMHP_CHECK(check_plan(plan));
    const Tree &T = plan->tree;
    const size_t nb = (size_t)T.nbox;
    struct Item {
        void *dst;
        const void *src;
        size_t bytes;
    } items[] = {
        {level, T.level, nb * 4}, {bx, T.bx, nb * 4},         {by, T.by, nb * 4},
        {first, T.first, nb * 4}, {count, T.count, nb * 4},   {parent, T.parent, nb * 4},
        {leaf, T.leaf, nb * 4},   {child_first, T.child_first, nb * 4}, {nchild, T.nchild, nb * 4},
        {u_ent, T.ent[0], (size_t)T.len[0] * 4}, {v_ent, T.ent[1], (size_t)T.len[1] * 4},
        {w_ent, T.ent[2], (size_t)T.len[2] * 4}, {x_ent, T.ent[3], (size_t)T.len[3] * 4},
    };
    for (auto &it : items)
        if (it.dst && it.bytes) FMMHP_HIP(hipMemcpy(it.dst, it.src, it.bytes, hipMemcpyDeviceToHost));
    int64_t *offs[4] = {u_off, v_off, w_off, x_off};
    std::vector<int32_t> tmp(nb + 1);
    for (int k = 0; k < 4; ++k) {
        if (!offs[k]) continue;
        FMMHP_HIP(hipMemcpy(tmp.data(), T.off[k], (nb + 1) * 4, hipMemcpyDeviceToHost));
        for (size_t i = 0; i <= nb; ++i) offs[k][i] = tmp[i];
    }
    if (perm) {
        std::vector<int32_t> pp((size_t)T.n);
        FMMHP_HIP(hipMemcpy(pp.data(), T.perm, (size_t)T.n * 4, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < T.n; ++i) perm[i] = pp[i];
    }
    return FMMHP_OK;
}

fmmhp_status fmmhp_plan_destroy(fmmhp_plan_t plan) {
    if (!plan) return FMMHP_OK;
    if (plan->magic != kMagic) {
        set_error("plan handle is not a live plan (destroyed or corrupted)");
        return FMMHP_ESTATE;
    }
    (void)hipDeviceSynchronize();
    if (plan->sched.events) {
        for (auto e : *plan->sched.events) (void)hipEventDestroy(e);
        delete plan->sched.events;
        plan->sched.events = nullptr;
    }
    delete plan->sched.m2l_n;
    plan->sched.m2l_n = nullptr;
    if (plan->sched.ev_fork) (void)hipEventDestroy(plan->sched.ev_fork);
    if (plan->sched.ev_join) (void)hipEventDestroy(plan->sched.ev_join);
    if (plan->sched.ev_up) (void)hipEventDestroy(plan->sched.ev_up);

    if (plan->sched.side) (void)hipStreamDestroy(plan->sched.side);
    if (plan->sched.side2) (void)hipStreamDestroy(plan->sched.side2);
    if (plan->sched.ev_deep_ready) (void)hipEventDestroy(plan->sched.ev_deep_ready);
    if (plan->sched.ev_deep_done) (void)hipEventDestroy(plan->sched.ev_deep_done);
    if (plan->sched.graph.exec) (void)hipGraphExecDestroy(plan->sched.graph.exec);
    plan->arena.release();
    plan->magic = kDead;
    delete plan;
    return FMMHP_OK;
}

fmmhp_status fmmhp_direct_eval(int64_t n_src, const double *src_x, const double *src_y, int n_vec, const double *q,
                               int64_t n_tgt, const double *tgt_x, const double *tgt_y, double lambda_re,
                               double lambda_im, double *phi, hipStream_t stream) {
    g_msg[0] = 0;
    if (n_src < 1 || n_tgt < 1 || n_vec < 1 || !src_x || !src_y || !q || !tgt_x || !tgt_y || !phi) {
        set_error("sizes must be >= 1 and pointers non-NULL");
        return FMMHP_EINVAL;
    }
    FMMHP_CHECK(check_impedance(lambda_re, lambda_im));
    return run_direct(n_src, src_x, src_y, n_vec, q, n_tgt, tgt_x, tgt_y, mk(lambda_re, lambda_im), phi, stream);
}

fmmhp_status fmmhp_reaction_integrals(int64_t m, const double *x, const double *y, int nmax, double lambda_re,
                                      double lambda_im, double *out, hipStream_t stream) {
    g_msg[0] = 0;
    if (m < 1 || !x || !y || !out || nmax < 0 || nmax > 2 * FMMHP_MAX_P) {
        set_error("m must be >= 1, pointers non-NULL, 0 <= nmax <= %d", 2 * FMMHP_MAX_P);
        return FMMHP_EINVAL;
    }
    FMMHP_CHECK(check_impedance(lambda_re, lambda_im));
    return run_reaction_integrals(m, x, y, nmax, mk(lambda_re, lambda_im), out, stream);
}

}  // extern "C"
