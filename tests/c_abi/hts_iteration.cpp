// hts_iteration.cpp -- one Barnes-Hut iteration of hyperbolic t-SNE through
// the C ABI of include/hts.h alone (no Python): build the polar quadtree of Y,
// take the gradient (eq. (15) with the Barnes-Hut repulsion of eq. (19)),
// then one Riemannian step (eqs. (16)-(18)).  HIP is used only to allocate
// device memory and copy.
//
// usage: hts_iteration <in.bin> <out.bin>
//   in.bin : int64 n, int64 nnz, double theta, double exaggeration,
//            double eta, double momentum, float Y[2n], int64 row_ptr[n+1],
//            int32 col[nnz], float val[nnz]
//   out.bin: float grad[2n], double Z, float Y_after_step[2n]
// Exit status 0 on success; otherwise the library's message is printed.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hts.h"

static void die(const char *what) {
    std::fprintf(stderr, "hts_iteration: %s: %s\n", what, hts_last_error());
    std::exit(1);
}

#define HIPCHK(call)                                                                  \
    do {                                                                              \
        hipError_t e__ = (call);                                                      \
        if (e__ != hipSuccess) {                                                      \
            std::fprintf(stderr, "hts_iteration: %s: %s\n", #call, hipGetErrorString(e__)); \
            std::exit(1);                                                             \
        }                                                                             \
    } while (0)

template <typename V>
static void read_all(std::FILE *f, V *p, size_t count) {
    if (std::fread(p, sizeof(V), count, f) != count) {
        std::fprintf(stderr, "hts_iteration: short input file\n");
        std::exit(1);
    }
}

int main(int argc, char **argv) {
    if (argc != 3) {
        std::fprintf(stderr, "usage: hts_iteration <in.bin> <out.bin>\n");
        return 2;
    }
    std::FILE *in = std::fopen(argv[1], "rb");
    if (!in) {
        std::fprintf(stderr, "hts_iteration: cannot open %s\n", argv[1]);
        return 1;
    }
    int64_t n = 0, nnz = 0;
    double theta = 0.0, ex = 0.0, eta = 0.0, mu = 0.0;
    read_all(in, &n, 1);
    read_all(in, &nnz, 1);
    read_all(in, &theta, 1);
    read_all(in, &ex, 1);
    read_all(in, &eta, 1);
    read_all(in, &mu, 1);
    if (n < 2 || nnz < 0) {
        std::fprintf(stderr, "hts_iteration: bad sizes\n");
        return 1;
    }
    std::vector<float> Y(2 * n), val(nnz);
    std::vector<int64_t> rp(n + 1);
    std::vector<int32_t> col(nnz);
    read_all(in, Y.data(), Y.size());
    read_all(in, rp.data(), rp.size());
    read_all(in, col.data(), col.size());
    read_all(in, val.data(), val.size());
    std::fclose(in);

    float *dY, *dG, *dU, *dGain, *dval;
    int64_t *drp;
    int32_t *dcol;
    double *dz;
    HIPCHK(hipMalloc(&dY, sizeof(float) * 2 * n));
    HIPCHK(hipMalloc(&dG, sizeof(float) * 2 * n));
    HIPCHK(hipMalloc(&dU, sizeof(float) * 2 * n));
    HIPCHK(hipMalloc(&dGain, sizeof(float) * 2 * n));
    HIPCHK(hipMalloc(&drp, sizeof(int64_t) * (n + 1)));
    HIPCHK(hipMalloc(&dcol, sizeof(int32_t) * (nnz > 0 ? nnz : 1)));
    HIPCHK(hipMalloc(&dval, sizeof(float) * (nnz > 0 ? nnz : 1)));
    HIPCHK(hipMalloc(&dz, sizeof(double)));
    HIPCHK(hipMemcpy(dY, Y.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(drp, rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dcol, col.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dval, val.data(), sizeof(float) * nnz, hipMemcpyHostToDevice));
    std::vector<float> zeros(2 * n, 0.0f), ones(2 * n, 1.0f);
    HIPCHK(hipMemcpy(dU, zeros.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dGain, ones.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice));

    hts_ctx ctx = nullptr;
    hts_tree tree = nullptr;
    hipStream_t st;
    HIPCHK(hipStreamCreate(&st));
    if (hts_create(0, &ctx) != HTS_OK) die("hts_create");
    if (hts_tree_create(ctx, n, 20, &tree) != HTS_OK) die("hts_tree_create");
    if (hts_build_polar_tree(ctx, st, dY, n, HTS_F32, tree) != HTS_OK) die("hts_build_polar_tree");
    if (hts_gradient_bh(ctx, st, dY, n, HTS_F32, drp, dcol, dval, ex, tree, theta, dG, dz, nullptr) !=
        HTS_OK)
        die("hts_gradient_bh");
    std::vector<float> grad(2 * n), Y1(2 * n);
    double z = 0.0;
    HIPCHK(hipMemcpyAsync(grad.data(), dG, sizeof(float) * 2 * n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&z, dz, sizeof(double), hipMemcpyDeviceToHost, st));
    if (hts_step(ctx, st, dY, dU, dGain, dG, n, HTS_F32, eta, mu, 0.01, 1e-5, 2) != HTS_OK)
        die("hts_step");
    HIPCHK(hipMemcpyAsync(Y1.data(), dY, sizeof(float) * 2 * n, hipMemcpyDeviceToHost, st));
    uint32_t bits = 0;
    if (hts_check(ctx, st, &bits) != HTS_OK) die("hts_check");  // waits for the stream

    std::FILE *out = std::fopen(argv[2], "wb");
    if (!out) {
        std::fprintf(stderr, "hts_iteration: cannot write %s\n", argv[2]);
        return 1;
    }
    std::fwrite(grad.data(), sizeof(float), grad.size(), out);
    std::fwrite(&z, sizeof(double), 1, out);
    std::fwrite(Y1.data(), sizeof(float), Y1.size(), out);
    std::fclose(out);

    hts_tree_destroy(tree);
    hts_destroy(ctx);
    HIPCHK(hipStreamDestroy(st));
    for (void *p : {(void *)dY, (void *)dG, (void *)dU, (void *)dGain, (void *)drp, (void *)dcol,
                    (void *)dval, (void *)dz})
        HIPCHK(hipFree(p));
    return 0;
}
