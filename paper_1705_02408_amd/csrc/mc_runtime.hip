// Monte Carlo verification of a plan (Sec. 3, final phase; the system and
// localisation models of Sec. 4.1): many sampled flights of the plan, each a
// double integrator tracking the nominal trajectory with an LQR controller
// while a Kalman filter fuses a noisy accelerometer with position fixes taken
// where the mapped features are good enough.  One thread per flight, float64
// state, counter-based normals (Philox4x32-10), blobs and boxes in LDS.
//
// The model, fixed where the paper gives only its structure:
//  * nominal: per edge the minimum-energy cubic between its two states --
//    2D/3D roadmaps: from rest to rest over 1.5 length / speed (peak speed
//    `speed`); 6D: the roadmap's states over the steering time (the
//    fixed-time minimum-energy trajectory); with velocity and acceleration;
//    samples at t_k = k dt, k = 0..K, K = ceil(duration / dt), clamped;
//  * per axis x = (p, v), x' = A x + B a, A = [[1, dt], [0, 1]],
//    B = [dt^2 / 2, dt]; applied a = u + sigma_w xi;
//  * u = (v_nom,k+1 - v_nom,k) / dt - k_p (p_hat - p_nom) - k_v (v_hat - v_nom):
//    the nominal velocity change over the step as feed-forward, the
//    steady-state discrete LQR gain for Q = diag(q_p, q_v), R = r_u (20,000
//    Riccati steps) as feedback;
//  * Kalman prediction with the measured acceleration a + sigma_a eta and
//    covariance sigma_a^2 B B^T; a position fix z = p + (sigma_v / sqrt(q)) zeta
//    at the new true position when its feature quality q >= q_min;
//  * start: p = p_nom + sigma_0 xi_0, v = v_nom, estimate nominal, covariance
//    diag(sigma_0^2, 0);
//  * per flight: the largest |p - p_hat| over k = 0..K, and whether a true
//    position lies in a closed box.
// Normals: Philox4x32-10 keyed by the seed, counter (step, flight, draw, 0)
// (step 0xffffffff at the start), two 53-bit uniforms per call and the
// Box-Muller pair; per step 3 dim normals in the order xi, eta, zeta.
#include "device_common.h"
#include "runtime_internal.h"

namespace {

constexpr int kMcGainSteps = 20000;
constexpr unsigned kMcStartStep = 0xffffffffu;

struct McNominal {
    int K;
    int dim;          // workspace dimension (2 or 3)
    double *p, *v, *a;  // [K+1][dim]
};

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// two standard normals for counter (step, flight, draw, 0)
__device__ __forceinline__ void normal2(uint32_t k0, uint32_t k1, uint32_t step, uint32_t flight,
                                        uint32_t draw, double &z0, double &z1) {
    uint32_t c[4] = {step, flight, draw, 0u};
    philox10(c, k0, k1);
    const uint64_t a = ((uint64_t)c[0] << 32) | c[1];
    const uint64_t b = ((uint64_t)c[2] << 32) | c[3];
    const double u1 = ((double)(a >> 11) + 0.5) * 0x1p-53;
    const double u2 = ((double)(b >> 11) + 0.5) * 0x1p-53;
    const double r = sqrt(-2.0 * log(u1));
    const double t = 2.0 * 3.141592653589793 * u2;
    z0 = r * cos(t);
    z1 = r * sin(t);
}

// n normals (n <= 10) of one step into z[0..n)
__device__ __forceinline__ void normals(uint32_t k0, uint32_t k1, uint32_t step, uint32_t flight,
                                        int n, double *z) {
    for (int j = 0; 2 * j < n; ++j) {
        double a, b;
        normal2(k0, k1, step, flight, (uint32_t)j, a, b);
        z[2 * j] = a;
        if (2 * j + 1 < n) z[2 * j + 1] = b;
    }
}

// steady-state discrete LQR gain of the per-axis double integrator (one thread)
__global__ void k_mc_gain(double dt, double qp, double qv, double ru, double *gain) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const double h = 0.5 * dt * dt;
    double P00 = qp, P01 = 0.0, P11 = qv;
    double kp = 0.0, kv = 0.0;
    for (int it = 0; it <= kMcGainSteps; ++it) {
        // B^T P B, B^T P A
        const double pb0 = P00 * h + P01 * dt, pb1 = P01 * h + P11 * dt;  // P B
        const double S = ru + (h * pb0 + dt * pb1);
        const double ba0 = pb0, ba1 = pb0 * dt + pb1;  // (P B)^T A
        kp = ba0 / S;
        kv = ba1 / S;
        if (it == kMcGainSteps) break;
        // A^T P A
        const double a00 = P00, a01 = P00 * dt + P01, a11 = (P00 * dt + P01) * dt + (P01 * dt + P11);
        // P <- Q + A^T P A - (A^T P B) K
        P00 = qp + a00 - ba0 * kp;
        P01 = a01 - ba0 * kv;
        P11 = qv + a11 - ba1 * kv;
    }
    gain[0] = kp;
    gain[1] = kv;
}

// duration and cumulative start time of every plan segment (one thread):
// polyline segments length / speed, or the steering time per edge
__global__ void k_mc_times(int m, int dim, const float *pos, const int *path, double speed,
                           double horizon, double *dur_out, double *tau) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int pw = dim;
    double t = 0.0;
    tau[0] = 0.0;
    for (int i = 0; i < m; ++i) {
        double dur;
        if (horizon > 0.0) {
            dur = horizon;
        } else {
            double l2 = 0.0;
            for (int k = 0; k < pw; ++k) {
                const double d = (double)pos[(size_t)path[i + 1] * pw + k] -
                                 (double)pos[(size_t)path[i] * pw + k];
                l2 = l2 + d * d;
            }
            dur = 1.5 * sqrt(l2) / speed;
        }
        dur_out[i] = dur;
        t = t + dur;
        tau[i + 1] = t;
    }
}

// nominal state at every step (one thread per step)
__global__ void k_mc_nominal(McNominal nm, int m, const float *pos, const float *vel,
                             const int *path, const double *dur, const double *tau, double dt,
                             double horizon) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nm.K) return;
    const int d = nm.dim;
    const double total = tau[m];
    const double t = fmin((double)k * dt, total);
    double pp[3] = {0, 0, 0}, vv[3] = {0, 0, 0}, aa[3] = {0, 0, 0};
    if (horizon > 0.0) {
        const double T = horizon;
        int i = (int)floor(t / T);
        i = min(max(i, 0), m - 1);
        const double s = t - (double)i * T;
        for (int c = 0; c < d; ++c) {
            const double p0 = pos[(size_t)path[i] * d + c], p1 = pos[(size_t)path[i + 1] * d + c];
            const double v0 = vel[(size_t)path[i] * 3 + c], v1 = vel[(size_t)path[i + 1] * 3 + c];
            const double c2 = (3.0 * (p1 - p0) - (2.0 * v0 + v1) * T) / (T * T);
            const double c3 = (2.0 * (p0 - p1) + (v0 + v1) * T) / (T * T * T);
            pp[c] = p0 + v0 * s + c2 * s * s + c3 * s * s * s;
            vv[c] = v0 + 2.0 * c2 * s + 3.0 * c3 * s * s;
            aa[c] = 2.0 * c2 + 6.0 * c3 * s;
        }
    } else {
        // last segment start <= t (searchsorted right, minus one), clamped
        int lo = 0, hi = m;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (tau[mid] <= t) lo = mid + 1; else hi = mid;
        }
        int i = min(max(lo - 1, 0), m - 1);
        const double s = t - tau[i];
        const double T = dur[i];
        for (int c = 0; c < d; ++c) {
            const double p0 = pos[(size_t)path[i] * d + c], p1 = pos[(size_t)path[i + 1] * d + c];
            const double c2 = (3.0 * (p1 - p0)) / (T * T);
            const double c3 = (2.0 * (p0 - p1)) / (T * T * T);
            pp[c] = p0 + c2 * s * s + c3 * s * s * s;
            vv[c] = 2.0 * c2 * s + 3.0 * c3 * s * s;
            aa[c] = 2.0 * c2 + 6.0 * c3 * s;
        }
    }
    for (int c = 0; c < d; ++c) {
        nm.p[(size_t)k * d + c] = pp[c];
        nm.v[(size_t)k * d + c] = vv[c];
        nm.a[(size_t)k * d + c] = aa[c];
    }
}

struct McArgs {
    McNominal nm;
    int rollouts;
    double dt, sw, sa, sv, qmin, s0, bound;
    const double *gain;
    uint32_t k0, k1;
    int nblob;
    const float *mu, *sig, *amp;  // [nblob][dim], [nblob], [nblob]
    int nbox;
    const float *blo, *bhi;       // [nbox][dim]
    double *max_err;              // [rollouts]
    uint8_t *collided;            // [rollouts]
    unsigned long long *counts;   // [3]: within bound, collision free, both
    double *err_sum;              // [1]
};

__device__ __forceinline__ bool in_boxes(const double *x, int d, int nbox, const float *lo,
                                         const float *hi) {
    for (int j = 0; j < nbox; ++j) {
        bool in = true;
        for (int c = 0; c < d; ++c)
            in = in && x[c] >= (double)lo[j * d + c] && x[c] <= (double)hi[j * d + c];
        if (in) return true;
    }
    return false;
}

__device__ __forceinline__ double quality(const double *x, int d, int nblob, const float *mu,
                                          const float *sig, const float *amp) {
    double acc = 0.0;
    for (int j = 0; j < nblob; ++j) {
        double d2 = 0.0;
        for (int c = 0; c < d; ++c) {
            const double t = x[c] - (double)mu[j * d + c];
            d2 = d2 + t * t;
        }
        const double s = (double)sig[j];
        acc = acc + (double)amp[j] * exp(-d2 / (2.0 * (s * s)));
    }
    return fmin(fmax(acc, 0.0), 1.0);
}

__global__ void __launch_bounds__(256) k_mc_rollout(McArgs a) {
    extern __shared__ float env[];  // mu, sig, amp, box lo, box hi
    const int d = a.nm.dim;
    float *mu = env, *sig = mu + a.nblob * d, *amp = sig + a.nblob;
    float *blo = amp + a.nblob, *bhi = blo + a.nbox * d;
    for (int i = threadIdx.x; i < a.nblob * d; i += blockDim.x) mu[i] = a.mu[i];
    for (int i = threadIdx.x; i < a.nblob; i += blockDim.x) {
        sig[i] = a.sig[i];
        amp[i] = a.amp[i];
    }
    for (int i = threadIdx.x; i < a.nbox * d; i += blockDim.x) {
        blo[i] = a.blo[i];
        bhi[i] = a.bhi[i];
    }
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    bool within = false, free = false;
    double merr = 0.0;
    if (r < a.rollouts) {
        const double dt = a.dt, h = 0.5 * dt * dt;
        const double kp = a.gain[0], kv = a.gain[1];
        const double *pn = a.nm.p, *vn = a.nm.v;
        double p[3], v[3], ph[3], vh[3], z[10];
        normals(a.k0, a.k1, kMcStartStep, (uint32_t)r, d, z);
        double e2 = 0.0;
        for (int c = 0; c < d; ++c) {
            p[c] = pn[c] + a.s0 * z[c];
            v[c] = vn[c];
            ph[c] = pn[c];
            vh[c] = vn[c];
            const double e = p[c] - ph[c];
            e2 = e2 + e * e;
        }
        double P00 = a.s0 * a.s0, P01 = 0.0, P11 = 0.0;
        merr = sqrt(e2);
        bool hit = in_boxes(p, d, a.nbox, blo, bhi);
        const double qa = a.sa * a.sa;
        for (int k = 0; k < a.nm.K; ++k) {
            normals(a.k0, a.k1, (uint32_t)k, (uint32_t)r, 3 * d, z);
            for (int c = 0; c < d; ++c) {
                const size_t o = (size_t)k * d + c;
                const double ff = (vn[o + d] - vn[o]) / dt;
                const double u = ff - kp * (ph[c] - pn[o]) - kv * (vh[c] - vn[o]);
                const double acc = u + a.sw * z[c];
                p[c] = p[c] + v[c] * dt + h * acc;
                v[c] = v[c] + dt * acc;
                const double am = acc + a.sa * z[d + c];
                ph[c] = ph[c] + vh[c] * dt + h * am;
                vh[c] = vh[c] + dt * am;
            }
            const double n00 = P00 + 2.0 * dt * P01 + dt * dt * P11 + qa * h * h;
            const double n01 = P01 + dt * P11 + qa * h * dt;
            const double n11 = P11 + qa * dt * dt;
            P00 = n00;
            P01 = n01;
            P11 = n11;
            const double q = quality(p, d, a.nblob, mu, sig, amp);
            if (q >= a.qmin) {
                const double Rv = a.sv * a.sv / q;
                const double sd = a.sv / sqrt(q);
                const double S = P00 + Rv;
                const double K0 = P00 / S, K1 = P01 / S;
                for (int c = 0; c < d; ++c) {
                    const double zp = p[c] + sd * z[2 * d + c];
                    const double innov = zp - ph[c];
                    ph[c] = ph[c] + K0 * innov;
                    vh[c] = vh[c] + K1 * innov;
                }
                const double u00 = (1.0 - K0) * P00, u01 = (1.0 - K0) * P01,
                             u11 = P11 - K1 * P01;
                P00 = u00;
                P01 = u01;
                P11 = u11;
            }
            e2 = 0.0;
            for (int c = 0; c < d; ++c) {
                const double e = p[c] - ph[c];
                e2 = e2 + e * e;
            }
            merr = fmax(merr, sqrt(e2));
            hit = hit || in_boxes(p, d, a.nbox, blo, bhi);
        }
        a.max_err[r] = merr;
        a.collided[r] = hit ? 1 : 0;
        within = merr <= a.bound;
        free = !hit;
    }
    // counts and the sum of the largest errors, one atomic per wave
    const unsigned long long bw = __popcll(ballot64(within)), bf = __popcll(ballot64(free)),
                             bb = __popcll(ballot64(within && free));
    const double es = wave_sum(r < a.rollouts ? merr : 0.0);
    if (lane_id() == 0) {
        atomicAdd(&a.counts[0], bw);
        atomicAdd(&a.counts[1], bf);
        atomicAdd(&a.counts[2], bb);
        atomicAdd(a.err_sum, es);
    }
}

}  // namespace

extern "C" int mpap_mc_verify(const mpap_graph *g, const int32_t *nodes, int32_t n_nodes,
                              const mpap_mc_params *mp, void *stream, double *max_err,
                              uint8_t *collided, mpap_mc_stats *out) {
    if (!g || !nodes || !mp || !out) return fail(MPAP_ERR_INVAL, "null graph, plan, params or output");
    if (!g->pos || (g->dim != 2 && g->dim != 3 && g->dim != 6) || g->nq != 1)
        return fail(MPAP_ERR_INVAL, "a roadmap built by mpap_build_graph (one query)");
    if (mp->rollouts < 1) return fail(MPAP_ERR_INVAL, "rollouts must be >= 1");
    const float fpos[] = {mp->dt, mp->speed, mp->sigma_v, mp->r_u};
    for (float x : fpos)
        if (!(x > 0.0f) || !std::isfinite(x)) return fail(MPAP_ERR_INVAL, "dt, speed, sigma_v, r_u must be > 0");
    const float fnn[] = {mp->sigma_w, mp->sigma_a, mp->sigma0, mp->q_p, mp->q_v, mp->err_bound,
                         mp->q_min};
    for (float x : fnn)
        if (!(x >= 0.0f) || !std::isfinite(x))
            return fail(MPAP_ERR_INVAL, "noise levels, weights, bound and q_min must be >= 0");
    if (n_nodes < 2) return fail(MPAP_ERR_INVAL, "the plan has no edge");
    for (int32_t i = 0; i < n_nodes; ++i)
        if (nodes[i] < 0 || nodes[i] >= g->n) return fail(MPAP_ERR_INVAL, "plan node out of range");
    const int len = n_nodes;
    const int32_t *path_h = nodes;
    const int m = len - 1;
    const int d = g->dim == 6 ? 3 : g->dim;
    const double dt = mp->dt, speed = mp->speed;
    const double horizon = g->dim == 6 ? (double)g->horizon : 0.0;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int *d_path = nullptr;
    double *segdur = nullptr;
    double *tau = nullptr, *gain = nullptr, *np_ = nullptr, *nv = nullptr, *na = nullptr,
           *merr = nullptr, *esum = nullptr;
    uint8_t *col = nullptr;
    unsigned long long *cnt = nullptr;
    auto cleanup = [&]() {
        dfree(d_path); dfree(segdur); dfree(tau); dfree(gain); dfree(np_); dfree(nv); dfree(na); dfree(merr);
        dfree(esum); dfree(col); dfree(cnt);
    };
    int rc;
    if ((rc = dalloc(&d_path, len)) || (rc = dalloc(&segdur, m)) || (rc = dalloc(&tau, m + 1)) ||
        (rc = dalloc(&gain, 2))) {
        cleanup();
        return rc;
    }
    HIP_TRY(hipMemcpyAsync(d_path, path_h, sizeof(int32_t) * len, hipMemcpyHostToDevice, s));
    k_mc_times<<<1, 64, 0, s>>>(m, d, g->pos, d_path, speed, horizon, segdur, tau);
    k_mc_gain<<<1, 64, 0, s>>>(dt, (double)mp->q_p, (double)mp->q_v, (double)mp->r_u, gain);
    double total = 0.0;
    HIP_TRY(hipMemcpyAsync(&total, tau + m, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double kd = std::ceil(total / dt);
    if (!(kd < 1e8)) {
        cleanup();
        return fail(MPAP_ERR_INVAL, "the plan needs more than 1e8 time steps");
    }
    const int K = std::max(1, (int)kd);
    const int R = mp->rollouts;
    if ((rc = dalloc(&np_, (size_t)(K + 1) * d)) || (rc = dalloc(&nv, (size_t)(K + 1) * d)) ||
        (rc = dalloc(&na, (size_t)(K + 1) * d)) || (rc = dalloc(&merr, R)) ||
        (rc = dalloc(&col, R)) || (rc = dalloc(&cnt, 3)) || (rc = dalloc(&esum, 1))) {
        cleanup();
        return rc;
    }
    McNominal nm{K, d, np_, nv, na};
    k_mc_nominal<<<div_up(K + 1, 256), 256, 0, s>>>(nm, m, g->pos, g->vel, d_path, segdur, tau,
                                                     dt, horizon);
    k_zero_i32<<<1, 64, 0, s>>>(reinterpret_cast<int *>(cnt), 6);
    k_zero_i32<<<1, 64, 0, s>>>(reinterpret_cast<int *>(esum), 2);
    McArgs a{};
    a.nm = nm;
    a.rollouts = R;
    a.dt = dt;
    a.sw = mp->sigma_w; a.sa = mp->sigma_a; a.sv = mp->sigma_v; a.qmin = mp->q_min;
    a.s0 = mp->sigma0; a.bound = mp->err_bound;
    a.gain = gain;
    a.k0 = (uint32_t)(mp->seed & 0xffffffffu);
    a.k1 = (uint32_t)(mp->seed >> 32);
    a.nblob = g->nblob; a.mu = g->bmu; a.sig = g->bsig; a.amp = g->bamp;
    a.nbox = g->nbox; a.blo = g->blo; a.bhi = g->bhi;
    a.max_err = merr; a.collided = col; a.counts = cnt; a.err_sum = esum;
    const size_t lds = sizeof(float) * ((size_t)g->nblob * (d + 2) + (size_t)g->nbox * 2 * d);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s));
    k_mc_rollout<<<div_up(R, 256), 256, lds, s>>>(a);
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipGetLastError());
    unsigned long long hc[3] = {0, 0, 0};
    double hs = 0.0, hg[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hs, esum, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hg, gain, sizeof(hg), hipMemcpyDeviceToHost, s));
    if (max_err) HIP_TRY(hipMemcpyAsync(max_err, merr, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    if (collided) HIP_TRY(hipMemcpyAsync(collided, col, R, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the largest error over all flights (host, from the per-flight values
    // when they were asked for; else a device pass would be needed)
    double mx = 0.0;
    if (max_err)
        for (int i = 0; i < R; ++i) mx = std::max(mx, max_err[i]);
    out->rollouts = R;
    out->within_bound = (int64_t)hc[0];
    out->collision_free = (int64_t)hc[1];
    out->success = (int64_t)hc[2];
    out->steps = K;
    out->duration = total;
    out->mean_max_err = hs / R;
    out->max_max_err = max_err ? mx : -1.0;
    out->gain_p = hg[0];
    out->gain_v = hg[1];
    out->gpu_ms = ms;
    cleanup();
    return MPAP_OK;
}
