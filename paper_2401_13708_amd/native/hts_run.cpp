// hts_run.cpp -- hyperbolic t-SNE iterations through the C ABI of
// include/hts.h with no Python in the process: input affinities (Sec. 2-A,
// eq. (1)) from X, then iterations of the Sec. 5 schedule (early
// exaggeration 12 with momentum 0.5 for the first 250 iterations, then 1 and
// 0.8; learning rate n / 12000; gains with floor 0.01), each one polar
// quadtree build, one Barnes-Hut gradient (eqs. (15), (19)) and one
// Riemannian step (eqs. (16)-(18)) on one stream with no host
// synchronisation.  Prints one JSON line with the timing of the timed
// iterations (HIP events on that stream).  With --copy-mib M it finally runs a
// plain device copy of M MiB, a kernel of known traffic for reading hardware
// byte counters against.
//
// usage: hts_run --peaks     (attainable copy bandwidth and vector FMA rates)
//        hts_run <input.bin> [--warmup W] [--steps K] [--theta T]
//                [--item-list L] [--copy-mib M] [--out Y.bin] [--progress P]
//                [--reload]
//   input.bin: int64 n, int32 d, int32 it0, float X[n*d] (row-major),
//              float Y0[2n] (the embedding in the Poincare disk at iteration
//              it0 of the schedule, where the run starts), optionally float
//              update[2n] and gains[2n] of the optimiser at it0 (else update
//              0 and gains 1)
//   Y.bin:     float Y[2n] after the warm-up and timed iterations
//   --progress P: a line on stderr every P iterations as they are issued
//                 (for runs under a profiler that serialises launches)
//   --reload:     the warm-up runs the counting kernels (same results), then
//                 the state of the input file is loaded again, so the timed
//                 steps are iterations it0 .. it0 + K - 1 from that state and
//                 the plain kernels run in them only (a window of bench.py)
// Exit status 0 on success; otherwise the failing call is printed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hts.h"

static void die(const char *what) {
    std::fprintf(stderr, "hts_run: %s: %s\n", what, hts_last_error());
    std::exit(1);
}

#define HIPCHK(call)                                                                           \
    do {                                                                                       \
        hipError_t e__ = (call);                                                               \
        if (e__ != hipSuccess) {                                                               \
            std::fprintf(stderr, "hts_run: %s: %s\n", #call, hipGetErrorString(e__));        \
            std::exit(1);                                                                      \
        }                                                                                      \
    } while (0)

#define HTSCHK(call)                 \
    do {                             \
        if ((call) != HTS_OK) die(#call); \
    } while (0)

// 16-byte elements, grid-stride: reads and writes count * 16 bytes once each
__global__ void copy_u4(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        dst[i] = src[i];
}

// kFmaChains independent multiply-add chains per thread, kFmaSteps steps each:
// 2 * kFmaChains * kFmaSteps flops per thread at the vector unit's rate
constexpr int kFmaChains = 8, kFmaSteps = 2048;
template <typename F>
__global__ void fma_chains(F b, F c, F *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    F a[kFmaChains];
#pragma unroll
    for (int j = 0; j < kFmaChains; ++j) a[j] = (F)(i & 7) + (F)j;
    for (int s = 0; s < kFmaSteps; ++s)
#pragma unroll
        for (int j = 0; j < kFmaChains; ++j) a[j] = a[j] * b + c;
    F r = 0;
#pragma unroll
    for (int j = 0; j < kFmaChains; ++j) r += a[j];
    out[i] = r;
}

// Attainable rates of this device: a 1 GiB device copy (HBM bytes read +
// written per second) and the FP32 / FP64 vector multiply-add rate (no
// packed FP32); the best of five timed runs of each, one JSON line.
static int run_peaks() {
    hipStream_t st;
    HIPCHK(hipStreamCreate(&st));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto best_ms = [&](auto launch) {
        float best = 1e30f;
        launch();  // warm-up
        for (int r = 0; r < 5; ++r) {
            HIPCHK(hipEventRecord(e0, st));
            launch();
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) best = ms;
        }
        return (double)best;
    };
    const int64_t count = ((int64_t)1 << 30) / 16;
    uint4 *a, *b;
    HIPCHK(hipMalloc(&a, (size_t)count * 16));
    HIPCHK(hipMalloc(&b, (size_t)count * 16));
    HIPCHK(hipMemsetAsync(a, 0, (size_t)count * 16, st));
    const double copy_ms = best_ms([&]() {
        hipLaunchKernelGGL(copy_u4, dim3(8192), dim3(256), 0, st, a, b, count);
    });
    HIPCHK(hipGetLastError());
    const int blocks = 8192, threads = 256;
    float *of;
    double *od;
    HIPCHK(hipMalloc(&of, sizeof(float) * blocks * threads));
    HIPCHK(hipMalloc(&od, sizeof(double) * blocks * threads));
    const double f32_ms = best_ms([&]() {
        hipLaunchKernelGGL(fma_chains<float>, dim3(blocks), dim3(threads), 0, st, 0.999f, 0.001f, of);
    });
    const double f64_ms = best_ms([&]() {
        hipLaunchKernelGGL(fma_chains<double>, dim3(blocks), dim3(threads), 0, st, 0.999, 0.001, od);
    });
    HIPCHK(hipGetLastError());
    const double flops = 2.0 * kFmaChains * kFmaSteps * (double)blocks * threads;
    std::printf("{\"copy_GBps\": %.1f, \"fp32_fma_TFLOPs\": %.2f, \"fp64_fma_TFLOPs\": %.2f, "
                "\"copy_bytes\": %lld, \"copy_ms\": %.4f, \"fma_flops\": %.0f, \"fp32_ms\": %.4f, "
                "\"fp64_ms\": %.4f}\n",
                2.0 * count * 16 / (copy_ms * 1e6), flops / (f32_ms * 1e9), flops / (f64_ms * 1e9),
                (long long)(2 * count * 16), copy_ms, flops, f32_ms, f64_ms);
    for (void *p : {(void *)a, (void *)b, (void *)of, (void *)od}) HIPCHK(hipFree(p));
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
    HIPCHK(hipStreamDestroy(st));
    return 0;
}

template <typename V>
static void read_all(std::FILE *f, V *p, size_t count) {
    if (std::fread(p, sizeof(V), count, f) != count) {
        std::fprintf(stderr, "hts_run: short input file\n");
        std::exit(1);
    }
}

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int main(int argc, char **argv) {
    if (argc == 2 && !std::strcmp(argv[1], "--peaks")) return run_peaks();
    if (argc < 2) {
        std::fprintf(stderr, "usage: hts_run <input.bin> [--warmup W] [--steps K] [--theta T] "
                             "[--item-list L] [--copy-mib M] [--out Y.bin] [--progress P]\n");
        return 2;
    }
    int warmup = 10, steps = 100, item_list = -1, progress = 0;
    double theta = 0.5;
    int64_t copy_mib = 0;
    const char *out_path = nullptr;
    bool reload = false;
    for (int a = 2; a < argc; ++a) {
        if (!std::strcmp(argv[a], "--reload")) {
            reload = true;
            continue;
        }
        if (a + 1 >= argc) {
            std::fprintf(stderr, "hts_run: %s needs a value\n", argv[a]);
            return 2;
        }
        const char *v = argv[a + 1];
        if (!std::strcmp(argv[a], "--warmup")) warmup = std::atoi(v);
        else if (!std::strcmp(argv[a], "--steps")) steps = std::atoi(v);
        else if (!std::strcmp(argv[a], "--theta")) theta = std::atof(v);
        else if (!std::strcmp(argv[a], "--item-list")) item_list = std::atoi(v);
        else if (!std::strcmp(argv[a], "--copy-mib")) copy_mib = std::atoll(v);
        else if (!std::strcmp(argv[a], "--out")) out_path = v;
        else if (!std::strcmp(argv[a], "--progress")) progress = std::atoi(v);
        else {
            std::fprintf(stderr, "hts_run: unknown option %s\n", argv[a]);
            return 2;
        }
        ++a;
    }
    if (warmup < 0 || steps < 1 || copy_mib < 0) {
        std::fprintf(stderr, "hts_run: need warmup >= 0, steps >= 1, copy-mib >= 0\n");
        return 2;
    }

    std::FILE *in = std::fopen(argv[1], "rb");
    if (!in) {
        std::fprintf(stderr, "hts_run: cannot open %s\n", argv[1]);
        return 1;
    }
    int64_t n = 0;
    int32_t d = 0, it0 = 0;
    read_all(in, &n, 1);
    read_all(in, &d, 1);
    read_all(in, &it0, 1);
    const int k = 90;
    if (n <= k || d < 1 || it0 < 0) {
        std::fprintf(stderr, "hts_run: bad header (n %lld, d %d)\n", (long long)n, d);
        return 1;
    }
    std::vector<float> X((size_t)n * d), Y0(2 * (size_t)n);
    std::vector<float> U0(2 * (size_t)n, 0.0f), G0(2 * (size_t)n, 1.0f);
    read_all(in, X.data(), X.size());
    read_all(in, Y0.data(), Y0.size());
    // the optimiser state, when the file carries it
    if (std::fread(U0.data(), sizeof(float), U0.size(), in) == U0.size())
        read_all(in, G0.data(), G0.size());
    else
        std::fill(U0.begin(), U0.end(), 0.0f);
    std::fclose(in);

    hipStream_t st;
    HIPCHK(hipStreamCreate(&st));
    hts_ctx ctx = nullptr;
    HTSCHK(hts_create(0, &ctx));
    if (item_list >= 0) HTSCHK(hts_set_item_list(ctx, item_list));

    // input affinities on the device
    const int64_t cap = 2 * n * (int64_t)k;
    float *dX, *dval;
    int64_t *drp;
    int32_t *dcol;
    HIPCHK(hipMalloc(&dX, sizeof(float) * X.size()));
    HIPCHK(hipMalloc(&drp, sizeof(int64_t) * (n + 1)));
    HIPCHK(hipMalloc(&dcol, sizeof(int32_t) * cap));
    HIPCHK(hipMalloc(&dval, sizeof(float) * cap));
    HIPCHK(hipMemcpy(dX, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice));
    int64_t nnz = 0;
    double t0 = now_s();
    HTSCHK(hts_build_affinities(ctx, st, dX, n, d, HTS_F32, 30.0, k, nullptr, drp, dcol, dval,
                                HTS_F32, cap, &nnz));
    const double aff_s = now_s() - t0;
    HIPCHK(hipFree(dX));
    std::fprintf(stderr, "hts_run: affinities nnz=%lld in %.2fs\n", (long long)nnz, aff_s);

    // state: Y, update, gains, gradient, Z
    float *dY, *dU, *dGain, *dG;
    double *dz;
    HIPCHK(hipMalloc(&dY, sizeof(float) * 2 * n));
    HIPCHK(hipMalloc(&dU, sizeof(float) * 2 * n));
    HIPCHK(hipMalloc(&dGain, sizeof(float) * 2 * n));
    HIPCHK(hipMalloc(&dG, sizeof(float) * 2 * n));
    HIPCHK(hipMalloc(&dz, sizeof(double)));
    auto upload_state = [&]() {
        HIPCHK(hipMemcpy(dY, Y0.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(dU, U0.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(dGain, G0.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice));
    };
    upload_state();
    hts_tree tree = nullptr;
    HTSCHK(hts_tree_create(ctx, n, 20, &tree));

    const double eta = (double)n / 12000.0;
    uint64_t *dstats = nullptr;  // counters of the counting kernels (not read)
    HIPCHK(hipMalloc(&dstats, 64 * sizeof(uint64_t)));
    HIPCHK(hipMemset(dstats, 0, 64 * sizeof(uint64_t)));
    int it = it0;
    auto iterate = [&](bool counting) {
        const bool early = it < 250;
        const double ex = early ? 12.0 : 1.0, mu = early ? 0.5 : 0.8;
        if (counting) {
            // the counting kernels (same results) through the separate calls
            HTSCHK(hts_build_polar_tree(ctx, st, dY, n, HTS_F32, tree));
            HTSCHK(hts_gradient_bh(ctx, st, dY, n, HTS_F32, drp, dcol, dval, ex, tree, theta, dG,
                                   dz, dstats));
            HTSCHK(hts_step(ctx, st, dY, dU, dGain, dG, n, HTS_F32, eta, mu, 0.01, 1e-5, 2));
        } else {
            HTSCHK(hts_iteration_bh(ctx, st, dY, dU, dGain, n, HTS_F32, drp, dcol, dval, ex, tree,
                                    theta, dG, dz, eta, mu, 0.01, 1e-5, 2));
        }
        ++it;
        if (progress > 0 && it % progress == 0) std::fprintf(stderr, "hts_run: iteration %d issued\n", it);
    };
    uint32_t bits = 0;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int w = 0; w < warmup; ++w) iterate(reload);
    HTSCHK(hts_check(ctx, st, &bits));
    if (reload) {
        upload_state();
        it = it0;
    }
    std::fprintf(stderr, "hts_run: %d warm-up iterations done%s\n", warmup,
                 reload ? " (counting kernels; state loaded again)" : "");
    t0 = now_s();
    HIPCHK(hipEventRecord(e0, st));
    for (int s = 0; s < steps; ++s) iterate(false);
    HIPCHK(hipEventRecord(e1, st));
    HTSCHK(hts_check(ctx, st, &bits));
    const double wall = now_s() - t0;
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    std::printf("{\"n\": %lld, \"nnz\": %lld, \"theta\": %.3f, \"start_iteration\": %d, "
                "\"warmup\": %d, \"steps\": %d, \"ms_per_step\": %.5f, \"iters_per_s\": %.2f, "
                "\"wall_s\": %.3f, \"affinities_s\": %.3f}\n",
                (long long)n, (long long)nnz, theta, it0, warmup, steps, ms / steps,
                1000.0 * steps / ms, wall, aff_s);
    std::fflush(stdout);
    if (out_path) {
        std::vector<float> Y(2 * n);
        HIPCHK(hipMemcpy(Y.data(), dY, sizeof(float) * 2 * n, hipMemcpyDeviceToHost));
        std::FILE *out = std::fopen(out_path, "wb");
        if (!out || std::fwrite(Y.data(), sizeof(float), Y.size(), out) != Y.size()) {
            std::fprintf(stderr, "hts_run: cannot write %s\n", out_path);
            return 1;
        }
        std::fclose(out);
    }

    if (copy_mib > 0) {
        const int64_t count = copy_mib * (1 << 20) / 16;
        uint4 *a, *b;
        HIPCHK(hipMalloc(&a, (size_t)count * 16));
        HIPCHK(hipMalloc(&b, (size_t)count * 16));
        HIPCHK(hipMemsetAsync(a, 0, (size_t)count * 16, st));
        hipLaunchKernelGGL(copy_u4, dim3(4096), dim3(256), 0, st, a, b, count);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        std::fprintf(stderr, "hts_run: copied %lld MiB\n", (long long)copy_mib);
        HIPCHK(hipFree(a));
        HIPCHK(hipFree(b));
    }

    HTSCHK(hts_tree_destroy(tree));
    HTSCHK(hts_destroy(ctx));
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
    HIPCHK(hipStreamDestroy(st));
    for (void *p : {(void *)drp, (void *)dcol, (void *)dval, (void *)dY, (void *)dU, (void *)dGain,
                    (void *)dG, (void *)dz, (void *)dstats})
        HIPCHK(hipFree(p));
    return 0;
}
