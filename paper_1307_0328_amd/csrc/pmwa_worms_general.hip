// pmwa_worms_general.hip -- worms of many intervals for a general local
// operator Q = sum_alpha Q_alpha (paper: "Worm creation and annihilation",
// Eq. (worm) in its general form and the sequence rule after it): soft-core
// bosons (b, b^+ with sqrt(n) elements), spin S (S^-, S^+), or any set of
// nonnegative operator types on up to 8 local states.
//
// One lane per interval.  The law of one interval, with x = lam * ell:
//   1. f_qp = <q|exp(x Q)|p> as the series of u_j = (x/j) Q u_{j-1}, u_0 =
//      |p>, stopped after term j once j + 2 >= 2y (y = x * max column sum
//      of Q) and 2 y |u_j|_1 / (j + 1) <= 2^-60 S_j (or u_j = 0); then the
//      count n by inversion of the partial sums S_j against U * f (a new U
//      when U * f rounds to f or n exceeds the free slots);
//   2. n distinct uniform slots, sorted;
//   3. the types and intermediate states from the last worm back to the
//      first: given the state s_k above worm k, (alpha_k, s_{k-1}) with
//      weight <s_k|Q_alpha|s_{k-1}> u_{k-1}[s_{k-1}];
//   4. one direction bit per worm in slot order.
// Every floating-point expression is evaluated in the order written (the
// library is built without contraction), so the draws are reproducible
// bit for bit from the stream words.
//
// Layout: outputs are slot-major (worm k of interval i at k * n_int + i),
// so a wavefront's stores of one worm index are contiguous.  The scaled
// vectors u_0..u_min(J,cap) of a lane live in a device workspace, vector
// component-major ((j * d + s) * lanes + lane), read back in reverse order
// by step 3.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "pmwa.h"
#include "pmwa_device.h"

namespace pmwa {

constexpr int GQ_D = PMWA_GQ_DMAX;
constexpr int GQ_A = PMWA_GQ_AMAX;
constexpr int GQ_TERMS = 256;
constexpr uint32_t RNG_GQ = 10;

struct GqDev {
    int32_t d, na;
    double qn;                        // max column sum of Q
    double q[GQ_A][GQ_D][GQ_D];       // <out|Q_alpha|in>
    double Q[GQ_D][GQ_D];             // sum over alpha, alpha ascending
};

struct GqArgs {
    const GqDev* g;
    double lam;
    int64_t n_int;
    const int32_t* p;
    const int32_t* q;
    const int64_t* ell;
    uint32_t key0, key1, stream, sweep, unit0;
    int32_t cap;
    double* ws;
    int32_t* n_out;
    int32_t* slots;
    uint8_t* alpha;
    uint8_t* after;
    uint8_t* dirs;
};

// v <- (x / j) * Q v on the first d components (rows ascending, the sum over
// columns ascending from 0).  Q is read from LDS row by row rather than held
// in registers.
PMWA_DEV void gq_step(const double (&Q)[GQ_D][GQ_D], int d, double x, int j, double (&v)[GQ_D])
{
    const double c = x / (double)j;
    double w[GQ_D];
#pragma unroll
    for (int a = 0; a < GQ_D; a++) w[a] = 0.0;
#pragma unroll 1
    for (int a = 0; a < d; a++) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < GQ_D; b++)
            if (b < d) s = s + Q[a][b] * v[b];
        const double r = c * s;
#pragma unroll
        for (int aa = 0; aa < GQ_D; aa++)
            if (aa == a) w[aa] = r;
    }
#pragma unroll
    for (int a = 0; a < GQ_D; a++) v[a] = w[a];
}

PMWA_DEV double pick(const double (&v)[GQ_D], int i)
{
    double r = 0.0;
#pragma unroll
    for (int a = 0; a < GQ_D; a++)
        if (a == i) r = v[a];
    return r;
}

__global__ __launch_bounds__(256) void k_worms_general(GqArgs A)
{
    __shared__ GqDev G;
    {
        const int nw = (int)(sizeof(GqDev) / sizeof(double));
        static_assert(sizeof(GqDev) % sizeof(double) == 0, "GqDev is whole doubles");
        const double* src = reinterpret_cast<const double*>(A.g);
        double* dst = reinterpret_cast<double*>(&G);
        for (int i = threadIdx.x; i < nw; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    const int d = G.d, na = G.na, cap = A.cap;
    const int64_t lanes = (int64_t)gridDim.x * blockDim.x;
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = A.n_int;

    for (int64_t i = lane; i < N; i += lanes) {
        const int p = A.p[i], q = A.q[i];
        const int64_t ell = A.ell[i];
        if (p < 0 || p >= d || q < 0 || q >= d || ell < 0) { A.n_out[i] = PMWA_EINVAL; continue; }
        if (ell == 0) { A.n_out[i] = p == q ? 0 : PMWA_ESTATE; continue; }
        const double x = A.lam * (double)ell;
        const double y = x * G.qn;
        auto ws = [&](int j, int a) -> double& { return A.ws[((int64_t)j * d + a) * lanes + lane]; };

        // 1. the series of f_qp
        double u[GQ_D];
#pragma unroll
        for (int a = 0; a < GQ_D; a++) u[a] = a == p ? 1.0 : 0.0;
        double S = 0.0;
        int J = -1;
        for (int j = 0; j < GQ_TERMS; j++) {
            if (j > 0) gq_step(G.Q, d, x, j, u);
            S = S + pick(u, q);
            if (j <= cap) {
#pragma unroll
                for (int a = 0; a < GQ_D; a++)
                    if (a < d) ws(j, a) = u[a];
            }
            double norm = 0.0;
#pragma unroll
            for (int a = 0; a < GQ_D; a++)
                if (a < d) norm = norm + u[a];
            if ((double)(j + 2) >= 2.0 * y &&
                (norm == 0.0 || (S > 0.0 && 2.0 * y * norm / (double)(j + 1) <= 0x1p-60 * S))) {
                J = j;
                break;
            }
        }
        if (J < 0) { A.n_out[i] = PMWA_EINVAL; continue; }
        if (!(S > 0.0)) { A.n_out[i] = PMWA_ESTATE; continue; }
        const double f = S;

        Stream s;
        s.init_keys(A.key0, A.key1, A.stream, A.sweep, RNG_GQ, A.unit0 + (uint32_t)i);

        // count: the partial sums again, from the stored vectors up to cap and
        // by the same recursion beyond
        int n = -1;
        for (int tries = 0; tries < 1000 && n < 0; tries++) {
            const double U = u53(s.next()) * f;
            double cum = 0.0;
            double v[GQ_D];
            for (int j = 0; j <= J; j++) {
                double t;
                if (j <= cap) {
                    t = ws(j, q);
                } else {
                    if (j == cap + 1) {
#pragma unroll
                        for (int a = 0; a < GQ_D; a++) v[a] = a < d ? ws(cap, a) : 0.0;
                    }
                    gq_step(G.Q, d, x, j, v);
                    t = pick(v, q);
                }
                cum = cum + t;
                if (U < cum) {
                    if ((int64_t)j <= ell) n = j;
                    break;
                }
            }
        }
        if (n < 0) { A.n_out[i] = PMWA_ESTATE; continue; }
        if (n > cap) { A.n_out[i] = PMWA_EOVERFLOW; continue; }

        // 2. slots: distinct, then sorted in place
        int32_t* sl = A.slots + i;
        bool bad = false;
        for (int k = 0; k < n && !bad; k++) {
            int32_t r = 0;
            bool again = true;
            for (int guard = 0; again && guard < 100000; guard++) {
                r = (int32_t)below(s.next(), (uint64_t)ell);
                again = false;
                for (int m = 0; m < k; m++)
                    if (sl[(int64_t)m * N] == r) { again = true; break; }
            }
            if (again) bad = true;
            sl[(int64_t)k * N] = r;
        }
        if (bad) { A.n_out[i] = PMWA_ESTATE; continue; }
        for (int a = 1; a < n; a++) {
            const int32_t v = sl[(int64_t)a * N];
            int b = a - 1;
            while (b >= 0 && sl[(int64_t)b * N] > v) { sl[(int64_t)(b + 1) * N] = sl[(int64_t)b * N]; b--; }
            sl[(int64_t)(b + 1) * N] = v;
        }

        // 3. the sequence, last worm first
        int st = q;
        for (int k = n; k >= 1 && !bad; k--) {
            double uu[GQ_D];
#pragma unroll
            for (int b = 0; b < GQ_D; b++) uu[b] = b < d ? ws(k - 1, b) : 0.0;
            double T = 0.0;
#pragma unroll 1
            for (int al = 0; al < na; al++) {
#pragma unroll
                for (int b = 0; b < GQ_D; b++)
                    if (b < d) T = T + G.q[al][st][b] * uu[b];
            }
            if (!(T > 0.0)) { bad = true; break; }
            const double U = u53(s.next()) * T;
            double cum = 0.0;
            int ca = -1, cb = -1, la = -1, lb = -1;
#pragma unroll 1
            for (int al = 0; al < na && ca < 0; al++) {
#pragma unroll
                for (int b = 0; b < GQ_D; b++) {
                    if (b < d && ca < 0) {
                        const double w = G.q[al][st][b] * uu[b];
                        if (w > 0.0) { la = al; lb = b; }
                        cum = cum + w;
                        if (U < cum) { ca = al; cb = b; }
                    }
                }
            }
            if (ca < 0) { ca = la; cb = lb; }
            A.alpha[(int64_t)(k - 1) * N + i] = (uint8_t)ca;
            A.after[(int64_t)(k - 1) * N + i] = (uint8_t)st;
            st = cb;
        }
        if (bad || st != p) { A.n_out[i] = PMWA_ESTATE; continue; }

        // 4. directions
        for (int k = 0; k < n; k++) A.dirs[(int64_t)k * N + i] = (uint8_t)(s.next() >> 63);
        A.n_out[i] = n;
    }
}

}  // namespace pmwa

using namespace pmwa;

namespace {
// Workspace of the vectors u_j, one per device, grown on demand and kept for
// the process.  A call waits (on its stream) for the previous call's kernel
// before reusing it, so calls on different streams do not overlap on it.
constexpr int WS_MAX_DEVICES = 64;
constexpr size_t WS_BUDGET = size_t(512) << 20;
struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool used = false;
};
std::mutex g_ws_mu;
Workspace g_ws[WS_MAX_DEVICES];
}  // namespace

extern "C" int pmwa_worms_general(const pmwa_localq* g, double lam, int64_t n_int, const int32_t* p,
                                  const int32_t* q, const int64_t* ell, uint64_t seed, uint32_t stream,
                                  uint32_t sweep, uint32_t unit0, int32_t cap, int32_t* n_out,
                                  int32_t* slots, uint8_t* alpha, uint8_t* after, uint8_t* dirs,
                                  void* hip_stream)
{
    if (!g || g->d < 2 || g->d > PMWA_GQ_DMAX || g->nalpha < 1 || g->nalpha > PMWA_GQ_AMAX) return PMWA_EINVAL;
    if (!(lam >= 0.0) || !std::isfinite(lam) || n_int < 0 || cap < 0 || cap > PMWA_GQ_CAPMAX) return PMWA_EINVAL;
    if (stream >= (1u << 24) || (uint64_t)unit0 + (uint64_t)n_int > (uint64_t(1) << 32)) return PMWA_EINVAL;
    if (n_int == 0) return PMWA_OK;
    if (!p || !q || !ell || !n_out) return PMWA_EINVAL;
    if (cap > 0 && (!slots || !alpha || !after || !dirs)) return PMWA_EINVAL;

    GqDev h{};
    h.d = g->d;
    h.na = g->nalpha;
    for (int al = 0; al < g->nalpha; al++)
        for (int a = 0; a < g->d; a++)
            for (int b = 0; b < g->d; b++) {
                const double v = g->q[al][a][b];
                if (!(v >= 0.0) || !std::isfinite(v)) return PMWA_EINVAL;
                h.q[al][a][b] = v;
            }
    for (int a = 0; a < g->d; a++)
        for (int b = 0; b < g->d; b++) {
            double s = 0.0;
            for (int al = 0; al < g->nalpha; al++) s = s + h.q[al][a][b];
            h.Q[a][b] = s;
        }
    h.qn = 0.0;
    for (int b = 0; b < g->d; b++) {
        double s = 0.0;
        for (int a = 0; a < g->d; a++) s = s + h.Q[a][b];
        if (s > h.qn) h.qn = s;
    }

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= WS_MAX_DEVICES) return PMWA_EDEVICE;
    hipStream_t st = (hipStream_t)hip_stream;

    // lanes: enough blocks to fill the chip, fewer when the workspace per lane
    // is large (grid-stride over the intervals)
    const size_t per_lane = (size_t)(cap + 1) * (size_t)g->d * sizeof(double);
    int64_t blocks = (n_int + 255) / 256;
    const int64_t max_blocks = std::max<int64_t>(1, (int64_t)(WS_BUDGET / per_lane) / 256);
    blocks = std::min<int64_t>(blocks, std::min<int64_t>(max_blocks, 8192));
    const size_t lanes = (size_t)blocks * 256;
    const size_t need = sizeof(GqDev) + lanes * per_lane + 256;

    std::lock_guard<std::mutex> lock(g_ws_mu);
    Workspace& W = g_ws[dev];
    if (!W.done && hipEventCreateWithFlags(&W.done, hipEventDisableTiming) != hipSuccess) {
        W.done = nullptr;
        return PMWA_EDEVICE;
    }
    if (W.bytes < need) {
        if (W.used && hipEventSynchronize(W.done) != hipSuccess) return PMWA_EDEVICE;
        if (W.ptr) (void)hipFree(W.ptr);
        W.ptr = nullptr;
        W.bytes = 0;
        W.used = false;
        if (hipMalloc(&W.ptr, need) != hipSuccess) { W.ptr = nullptr; return PMWA_ENOMEM; }
        W.bytes = need;
    } else if (W.used && hipStreamWaitEvent(st, W.done, 0) != hipSuccess) {
        return PMWA_EDEVICE;
    }
    GqDev* gdev = (GqDev*)W.ptr;
    double* ws = (double*)((char*)W.ptr + ((sizeof(GqDev) + 255) & ~size_t(255)));
    if (hipMemcpyAsync(gdev, &h, sizeof(GqDev), hipMemcpyHostToDevice, st) != hipSuccess) return PMWA_EDEVICE;

    GqArgs A{};
    A.g = gdev; A.lam = lam; A.n_int = n_int; A.p = p; A.q = q; A.ell = ell;
    A.key0 = (uint32_t)seed; A.key1 = (uint32_t)(seed >> 32); A.stream = stream; A.sweep = sweep;
    A.unit0 = unit0; A.cap = cap; A.ws = ws; A.n_out = n_out; A.slots = slots; A.alpha = alpha;
    A.after = after; A.dirs = dirs;
    hipLaunchKernelGGL(k_worms_general, dim3((unsigned)blocks), dim3(256), 0, st, A);
    if (hipGetLastError() != hipSuccess) return PMWA_EDEVICE;
    if (hipEventRecord(W.done, st) != hipSuccess) return PMWA_EDEVICE;
    W.used = true;
    return PMWA_OK;
}
