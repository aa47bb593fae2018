// Autotuner (declared in include/fmmhp.h): p from a measured error against the GPU direct sum,
// leaf size, the near-field launch shape and the M2L form (FP64 or FP32 matrix cores) from measured
// eval time.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace fmmhp {

__global__ void k_gather_sample(const double *__restrict__ x, const double *__restrict__ y, int64_t n, int m,
                                double *__restrict__ sx, double *__restrict__ sy) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int64_t i = (int64_t)((double)k * (double)n / (double)m);
    sx[k] = x[i];
    sy[k] = y[i];
}

__global__ void k_gather_phi(const double *__restrict__ phi, int64_t n, int m, double *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int64_t i = (int64_t)((double)k * (double)n / (double)m);
    out[2 * k] = phi[2 * i];
    out[2 * k + 1] = phi[2 * i + 1];
}

struct DevTmp {
    std::vector<void *> p;
    ~DevTmp() {
        for (void *q : p) (void)hipFree(q);
    }
    template <class T>
    fmmhp_status get(T **ptr, size_t n) {
        void *q = nullptr;
        if (hipMalloc(&q, (n ? n : 1) * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            set_error("autotuner: device allocation of %zu bytes failed", n * sizeof(T));
            return FMMHP_ENOMEM;
        }
        p.push_back(q);
        *ptr = (T *)q;
        return FMMHP_OK;
    }
};

// Median over three rounds of the mean time of five back-to-back evaluations (n_vec vectors),
// after one untimed evaluation: the steady state of a loop of evaluations, in which one
// evaluation's first kernels overlap the tail of the one before.
static fmmhp_status median_ms(fmmhp_plan_t plan, int n_vec, const double *q, double *phi, hipEvent_t e0,
                              hipEvent_t e1, hipStream_t s, double *med) {
    constexpr int kRounds = 3, kPerRound = 5;
    FMMHP_CHECK(fmmhp_eval(plan, n_vec, q, phi, s));
    std::vector<float> t;
    for (int r = 0; r < kRounds; ++r) {
        FMMHP_HIP(hipEventRecord(e0, s));
        for (int k = 0; k < kPerRound; ++k) FMMHP_CHECK(fmmhp_eval(plan, n_vec, q, phi, s));
        FMMHP_HIP(hipEventRecord(e1, s));
        FMMHP_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        FMMHP_HIP(hipEventElapsedTime(&ms, e0, e1));
        t.push_back(ms / kPerRound);
    }
    std::sort(t.begin(), t.end());
    *med = t[t.size() / 2];
    return FMMHP_OK;
}

// Mean time of five back-to-back evaluations after one untimed evaluation.
static fmmhp_status mean_ms(fmmhp_plan_t plan, int n_vec, const double *q, double *phi, hipEvent_t e0,
                            hipEvent_t e1, hipStream_t s, double *ms_out) {
    constexpr int kPerRound = 5;
    FMMHP_CHECK(fmmhp_eval(plan, n_vec, q, phi, s));
    FMMHP_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < kPerRound; ++k) FMMHP_CHECK(fmmhp_eval(plan, n_vec, q, phi, s));
    FMMHP_HIP(hipEventRecord(e1, s));
    FMMHP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    FMMHP_HIP(hipEventElapsedTime(&ms, e0, e1));
    *ms_out = ms / kPerRound;
    return FMMHP_OK;
}

}  // namespace fmmhp

using namespace fmmhp;

extern "C" fmmhp_status fmmhp_tune(int64_t n, const double *x, const double *y, const double *q, double lambda_re,
                                   double lambda_im, double tol, int n_vec, const int *leaf_sizes, int n_leaf,
                                   int sample, fmmhp_opts *best, double *err_out, double *ms_out, hipStream_t s) {
    if (!x || !y || !q || !best || n < 1 || !(tol > 0.0) || n_vec < 1 || (leaf_sizes && n_leaf < 1) ||
        sample < 0 || sample > n) {
        set_error("fmmhp_tune: invalid arguments");
        return FMMHP_EINVAL;
    }
    static const int kDefaultLeaves[] = {24, 32, 40, 48, 64, 96};
    if (!leaf_sizes) {
        leaf_sizes = kDefaultLeaves;
        n_leaf = 6;
    }
    const int m = sample ? sample : (int)std::min<int64_t>(n, 256);
    DevTmp tmp;
    double *sx, *sy, *ref, *phi, *got, *qv;
    FMMHP_CHECK(tmp.get(&sx, m));
    FMMHP_CHECK(tmp.get(&sy, m));
    FMMHP_CHECK(tmp.get(&ref, 2 * (size_t)m));
    FMMHP_CHECK(tmp.get(&got, 2 * (size_t)m));
    FMMHP_CHECK(tmp.get(&phi, 2 * (size_t)n * n_vec));
    FMMHP_CHECK(tmp.get(&qv, (size_t)n * n_vec));
    for (int v = 0; v < n_vec; ++v)
        FMMHP_HIP(hipMemcpyAsync(qv + (size_t)v * n, q, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_gather_sample, dim3((m + 127) / 128), dim3(128), 0, s, x, y, n, m, sx, sy);
    FMMHP_HIP(hipGetLastError());
    FMMHP_CHECK(fmmhp_direct_eval(n, x, y, 1, q, m, sx, sy, lambda_re, lambda_im, ref, s));
    std::vector<double> href(2 * (size_t)m), hgot(2 * (size_t)m);
    FMMHP_HIP(hipMemcpyAsync(href.data(), ref, href.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    FMMHP_HIP(hipStreamSynchronize(s));
    double nref = 0.0;
    for (double v : href) nref += v * v;
    nref = sqrt(nref);
    hipEvent_t e0, e1;
    FMMHP_HIP(hipEventCreate(&e0));
    FMMHP_HIP(hipEventCreate(&e1));
    double best_ms = INFINITY, best_err = 0.0;
    fmmhp_opts bo{0, 0, 0, 0, 0, 0};
    int p_start = 5;
    fmmhp_status st = FMMHP_OK;
    for (int li = 0; li < n_leaf && st == FMMHP_OK; ++li) {
        for (int p = p_start; p <= FMMHP_MAX_P && st == FMMHP_OK; p += 5) {
            fmmhp_opts o{p, leaf_sizes[li], 0, 0, 0, 0};
            fmmhp_plan_t plan = nullptr;
            st = fmmhp_plan_create(n, x, y, nullptr, nullptr, lambda_re, lambda_im, &o, s, &plan);
            if (st == FMMHP_EUNSUPPORTED) {  // e.g. tables beyond the recursion's range at this leaf size
                st = FMMHP_OK;
                break;
            }
            if (st != FMMHP_OK) break;
            st = fmmhp_eval(plan, 1, q, phi, s);
            if (st == FMMHP_OK) {
                hipLaunchKernelGGL(k_gather_phi, dim3((m + 127) / 128), dim3(128), 0, s, phi, n, m, got);
                if (hipGetLastError() != hipSuccess ||
                    hipMemcpyAsync(hgot.data(), got, hgot.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
                        hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess) {
                    set_error("autotuner: device copy failed");
                    st = FMMHP_EHIP;
                }
            }
            double e = INFINITY;
            if (st == FMMHP_OK) {
                double d = 0.0;
                for (size_t k = 0; k < hgot.size(); ++k) d += (hgot[k] - href[k]) * (hgot[k] - href[k]);
                e = sqrt(d) / nref;
            }
            if (st == FMMHP_OK && e <= tol) {
                double med = INFINITY;
                st = median_ms(plan, n_vec, qv, phi, e0, e1, s, &med);
                if (st == FMMHP_OK && med < best_ms) {
                    best_ms = med;
                    best_err = e;
                    bo = o;
                }
                (void)fmmhp_plan_destroy(plan);
                // the next leaf size rarely needs a smaller p: start one step below
                p_start = std::max(5, p - 5);
                break;
            }
            (void)fmmhp_plan_destroy(plan);
        }
    }
    // launch shape of the near field on the chosen plan: the shapes are timed in turn over three
    // rounds (so that a drift of the clocks favours none), each by the median of its rounds; another
    // shape replaces the library default only when it is more than 2% faster
    if (st == FMMHP_OK && best_ms < INFINITY) {
        fmmhp_plan_t plan = nullptr;
        st = fmmhp_plan_create(n, x, y, nullptr, nullptr, lambda_re, lambda_im, &bo, s, &plan);
        if (st == FMMHP_OK) {
            constexpr int kShapes = 6, kRounds = 3;
            static const int shapes[kShapes][2] = {{1, 2}, {1, 4}, {2, 4}, {2, 8}, {4, 4}, {4, 8}};
            const int def_walk = plan->sched.near_walk, def_groups = (int)(plan->sched.near_blocks / plan->sched.cus);
            double t[kShapes][kRounds];
            for (int r = 0; r < kRounds && st == FMMHP_OK; ++r)
                for (int k = 0; k < kShapes && st == FMMHP_OK; ++k) {
                    st = apply_launch_shape(plan->arena, plan->tree, plan->sched, shapes[k][0], shapes[k][1], s);
                    if (st == FMMHP_OK) st = mean_ms(plan, n_vec, qv, phi, e0, e1, s, &t[k][r]);
                }
            if (st == FMMHP_OK) {
                double med[kShapes];
                int kd = 0, kb = 0;
                for (int k = 0; k < kShapes; ++k) {
                    std::sort(t[k], t[k] + kRounds);
                    med[k] = t[k][kRounds / 2];
                    if (shapes[k][0] == def_walk && shapes[k][1] == def_groups) kd = k;
                    if (med[k] < med[kb]) kb = k;
                }
                const int k = med[kb] < 0.98 * med[kd] ? kb : kd;
                bo.near_walk = shapes[k][0];
                bo.near_groups = shapes[k][1];
                best_ms = med[k];
            }
            (void)fmmhp_plan_destroy(plan);
        }
    }
    // FP64 M2L form: the other of the vector-ALU and matrix-core forms on the chosen plan and launch
    // shape (the same sums in another order), kept when it is more than 2% faster
    if (st == FMMHP_OK && best_ms < INFINITY) {
        fmmhp_opts of = bo;
        fmmhp_plan_t plan = nullptr;
        st = fmmhp_plan_create(n, x, y, nullptr, nullptr, lambda_re, lambda_im, &bo, s, &plan);
        if (st == FMMHP_OK) {
            // the form the chosen plan uses
            const bool mf = plan->sched.m2l_form == 2;
            (void)fmmhp_plan_destroy(plan);
            plan = nullptr;
            of.flags = (bo.flags & ~(FMMHP_FLAG_M2L_VECTOR | FMMHP_FLAG_M2L_MFMA)) |
                       (mf ? FMMHP_FLAG_M2L_VECTOR : FMMHP_FLAG_M2L_MFMA);
            st = fmmhp_plan_create(n, x, y, nullptr, nullptr, lambda_re, lambda_im, &of, s, &plan);
        }
        if (st == FMMHP_OK) {
            double t[3];
            for (int r = 0; r < 3 && st == FMMHP_OK; ++r) st = mean_ms(plan, n_vec, qv, phi, e0, e1, s, &t[r]);
            if (st == FMMHP_OK) {
                std::sort(t, t + 3);
                if (t[1] < 0.98 * best_ms) {
                    bo = of;
                    best_ms = t[1];
                }
            }
        }
        if (plan) (void)fmmhp_plan_destroy(plan);
    }
    // M2L form: the FP32 matrix-core M2L (FMMHP_FLAG_M2L_FP32) on the chosen plan and launch shape, kept
    // when its error against the direct sum still meets the tolerance and it is more than 2% faster
    if (st == FMMHP_OK && best_ms < INFINITY) {
        fmmhp_opts o32 = bo;
        o32.flags |= FMMHP_FLAG_M2L_FP32;
        fmmhp_plan_t plan = nullptr;
        st = fmmhp_plan_create(n, x, y, nullptr, nullptr, lambda_re, lambda_im, &o32, s, &plan);
        if (st == FMMHP_OK) {
            st = fmmhp_eval(plan, 1, q, phi, s);
            if (st == FMMHP_OK) {
                hipLaunchKernelGGL(k_gather_phi, dim3((m + 127) / 128), dim3(128), 0, s, phi, n, m, got);
                if (hipGetLastError() != hipSuccess ||
                    hipMemcpyAsync(hgot.data(), got, hgot.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
                        hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess) {
                    set_error("autotuner: device copy failed");
                    st = FMMHP_EHIP;
                }
            }
            if (st == FMMHP_OK) {
                double d = 0.0;
                for (size_t k = 0; k < hgot.size(); ++k) d += (hgot[k] - href[k]) * (hgot[k] - href[k]);
                const double e32 = sqrt(d) / nref;
                if (e32 <= tol) {
                    double t[3];
                    for (int r = 0; r < 3 && st == FMMHP_OK; ++r) st = mean_ms(plan, n_vec, qv, phi, e0, e1, s, &t[r]);
                    if (st == FMMHP_OK) {
                        std::sort(t, t + 3);
                        if (t[1] < 0.98 * best_ms) {
                            bo = o32;
                            best_ms = t[1];
                            best_err = e32;
                        }
                    }
                }
            }
            (void)fmmhp_plan_destroy(plan);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FMMHP_OK) return st;
    if (!(best_ms < INFINITY)) {
        set_error("fmmhp_tune: no candidate reached rel-l2 %g at p <= %d", tol, FMMHP_MAX_P);
        return FMMHP_EUNSUPPORTED;
    }
    *best = bo;
    if (err_out) *err_out = best_err;
    if (ms_out) *ms_out = best_ms;
    return FMMHP_OK;
}
