// capi_check.cpp -- drives libsat.so through its C ABI alone (no Python, no torch): device
// memory from the HIP runtime, every call from include/sat.h, results written to a file that the
// GPU test compares with the oracle.
//
//   capi_check H W out_path
//
// The image is 8-bit, pixel (y, x) = (y * 131 + x * 71 + (x * y) % 17) % 256, rows on a pitch of
// W + 3 elements (so not aligned).  The program builds the table and the squared table, the sums
// of 7 x 5 windows at stride 2 (window_sum, uint32), the fused sums of 3 x 3 and 9 x 9 windows at
// stride 1 (window_sum_multi, uint32), and the mean and std of 4 x 6 windows at stride 3
// (window_mean_std), and writes, in order: the two tables (H x W uint64 each), the window sums,
// the two fused outputs, the sums, means and standard deviations, all dense.  Then it builds the
// table again in two bands of rows, [0, H/2) and [H/2, H) (sat_build_band): the lower band's carry
// comes from sat_column_totals of the upper rows and is advanced in place by the lower band's
// build.  It appends the table so assembled (H x W), the upper band's own totals output, the
// column totals of the upper rows and the final totals (W uint64 each).
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "sat.h"

namespace {

int die(const char *what) {
    std::fprintf(stderr, "capi_check: %s: %s\n", what, sat_last_error());
    return 1;
}

int hip_die(const char *what, hipError_t e) {
    std::fprintf(stderr, "capi_check: %s: %s\n", what, hipGetErrorString(e));
    return 1;
}

template <typename T>
bool append(std::FILE *f, const std::vector<T> &v) {
    return std::fwrite(v.data(), sizeof(T), v.size(), f) == v.size();
}

}  // namespace

int main(int argc, char **argv) {
    if (argc != 4) {
        std::fprintf(stderr, "usage: capi_check H W out_path\n");
        return 2;
    }
    const int64_t H = std::atoll(argv[1]), W = std::atoll(argv[2]);
    if (H < 9 || W < 9) {
        std::fprintf(stderr, "capi_check: H and W must be at least 9\n");
        return 2;
    }
    const int64_t ip = W + 3, sp = W;
    std::vector<uint8_t> img(static_cast<size_t>(H * ip), 0);
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) img[y * ip + x] = static_cast<uint8_t>((y * 131 + x * 71 + (x * y) % 17) % 256);

    hipError_t e;
    void *d_img = nullptr, *d_ws = nullptr;
    uint64_t *d_S = nullptr, *d_Q = nullptr;
    if ((e = hipMalloc(&d_img, img.size()))) return hip_die("hipMalloc image", e);
    if ((e = hipMalloc(reinterpret_cast<void **>(&d_S), H * sp * 8))) return hip_die("hipMalloc table", e);
    if ((e = hipMalloc(reinterpret_cast<void **>(&d_Q), H * sp * 8))) return hip_die("hipMalloc squared table", e);
    if ((e = hipMemcpy(d_img, img.data(), img.size(), hipMemcpyHostToDevice))) return hip_die("copy image", e);
    const size_t wsb = sat_build_workspace_bytes(H, W, SAT_U8, 1);
    if (wsb == 0) return die("sat_build_workspace_bytes");
    if ((e = hipMalloc(&d_ws, wsb))) return hip_die("hipMalloc workspace", e);
    if (sat_build(d_img, SAT_U8, H, W, ip, d_S, d_Q, sp, d_ws, wsb, nullptr)) return die("sat_build");
    if (sat_workspace_check(d_ws, nullptr)) return die("sat_workspace_check");

    // window_sum: 7 x 5 at stride 2
    int64_t oh = 0, ow = 0;
    if (window_out_shape(H, W, 7, 5, 2, &oh, &ow)) return die("window_out_shape");
    uint32_t *d_sum = nullptr;
    if ((e = hipMalloc(reinterpret_cast<void **>(&d_sum), oh * ow * 4))) return hip_die("hipMalloc sums", e);
    if (window_sum(d_S, SAT_U8, H, W, sp, 7, 5, 2, d_sum, SAT_U32, ow, nullptr)) return die("window_sum");

    // window_sum_multi: 3 x 3 and 9 x 9 at stride 1
    const int64_t mh[2] = {3, 9}, mw[2] = {3, 9};
    int64_t moh[2], mow[2];
    void *d_multi[2];
    int64_t mpitch[2];
    for (int i = 0; i < 2; ++i) {
        if (window_out_shape(H, W, mh[i], mw[i], 1, &moh[i], &mow[i])) return die("window_out_shape");
        if ((e = hipMalloc(&d_multi[i], moh[i] * mow[i] * 4))) return hip_die("hipMalloc multi", e);
        mpitch[i] = mow[i];
    }
    if (window_sum_multi(d_S, SAT_U8, H, W, sp, 2, mh, mw, 1, d_multi, SAT_U32, mpitch, nullptr))
        return die("window_sum_multi");

    // window_mean_std: 4 x 6 at stride 3
    int64_t soh = 0, sow = 0;
    if (window_out_shape(H, W, 4, 6, 3, &soh, &sow)) return die("window_out_shape");
    uint64_t *d_s1 = nullptr;
    double *d_mean = nullptr, *d_std = nullptr;
    if ((e = hipMalloc(reinterpret_cast<void **>(&d_s1), soh * sow * 8))) return hip_die("hipMalloc s1", e);
    if ((e = hipMalloc(reinterpret_cast<void **>(&d_mean), soh * sow * 8))) return hip_die("hipMalloc mean", e);
    if ((e = hipMalloc(reinterpret_cast<void **>(&d_std), soh * sow * 8))) return hip_die("hipMalloc std", e);
    if (window_mean_std(d_S, d_Q, H, W, sp, 4, 6, 3, d_s1, d_mean, d_std, sow, nullptr)) return die("window_mean_std");
    if ((e = hipDeviceSynchronize())) return hip_die("synchronize", e);

    std::vector<uint64_t> S(H * sp), Q(H * sp), s1(soh * sow);
    std::vector<uint32_t> sums(oh * ow), m0(moh[0] * mow[0]), m1(moh[1] * mow[1]);
    std::vector<double> mean(soh * sow), stdv(soh * sow);
    if ((e = hipMemcpy(S.data(), d_S, S.size() * 8, hipMemcpyDeviceToHost))) return hip_die("copy table", e);
    if ((e = hipMemcpy(Q.data(), d_Q, Q.size() * 8, hipMemcpyDeviceToHost))) return hip_die("copy table", e);
    if ((e = hipMemcpy(sums.data(), d_sum, sums.size() * 4, hipMemcpyDeviceToHost))) return hip_die("copy sums", e);
    if ((e = hipMemcpy(m0.data(), d_multi[0], m0.size() * 4, hipMemcpyDeviceToHost))) return hip_die("copy multi", e);
    if ((e = hipMemcpy(m1.data(), d_multi[1], m1.size() * 4, hipMemcpyDeviceToHost))) return hip_die("copy multi", e);
    if ((e = hipMemcpy(s1.data(), d_s1, s1.size() * 8, hipMemcpyDeviceToHost))) return hip_die("copy s1", e);
    if ((e = hipMemcpy(mean.data(), d_mean, mean.size() * 8, hipMemcpyDeviceToHost))) return hip_die("copy mean", e);
    if ((e = hipMemcpy(stdv.data(), d_std, stdv.size() * 8, hipMemcpyDeviceToHost))) return hip_die("copy std", e);

    // the same table in two bands
    const int64_t h1 = H / 2;
    uint64_t *d_B = nullptr, *d_top = nullptr, *d_carry = nullptr;
    if ((e = hipMalloc(reinterpret_cast<void **>(&d_B), H * sp * 8))) return hip_die("hipMalloc band table", e);
    if ((e = hipMalloc(reinterpret_cast<void **>(&d_top), W * 8))) return hip_die("hipMalloc totals", e);
    if ((e = hipMalloc(reinterpret_cast<void **>(&d_carry), W * 8))) return hip_die("hipMalloc carry", e);
    const uint8_t *d_lower = static_cast<const uint8_t *>(d_img) + h1 * ip;
    size_t bwsb = sat_build_workspace_bytes(h1, W, SAT_U8, 0);
    const size_t lower_wsb = sat_build_workspace_bytes(H - h1, W, SAT_U8, 0);
    if (bwsb == 0 || lower_wsb == 0) return die("sat_build_workspace_bytes");
    if (lower_wsb > bwsb) bwsb = lower_wsb;
    void *d_bws = nullptr;
    if ((e = hipMalloc(&d_bws, bwsb))) return hip_die("hipMalloc band workspace", e);
    if (sat_build_band(d_img, SAT_U8, h1, W, ip, nullptr, nullptr, 0, d_B, nullptr, sp, d_top, nullptr, d_bws, bwsb,
                       nullptr))
        return die("sat_build_band (upper)");
    if (sat_column_totals(d_img, SAT_U8, h1, W, ip, nullptr, nullptr, d_carry, nullptr, nullptr))
        return die("sat_column_totals");
    if (sat_build_band(d_lower, SAT_U8, H - h1, W, ip, d_carry, nullptr, h1, d_B + h1 * sp, nullptr, sp, d_carry,
                       nullptr, d_bws, bwsb, nullptr))
        return die("sat_build_band (lower)");
    if (sat_workspace_check(d_bws, nullptr)) return die("sat_workspace_check");
    std::vector<uint64_t> B(H * sp), top(W), upper(W), fin(W);
    if ((e = hipMemcpy(B.data(), d_B, B.size() * 8, hipMemcpyDeviceToHost))) return hip_die("copy band table", e);
    if ((e = hipMemcpy(top.data(), d_top, W * 8, hipMemcpyDeviceToHost))) return hip_die("copy totals", e);
    if ((e = hipMemcpy(fin.data(), d_carry, W * 8, hipMemcpyDeviceToHost))) return hip_die("copy totals", e);
    // the upper rows' totals once more, from sat_column_totals alone
    if (sat_column_totals(d_img, SAT_U8, h1, W, ip, nullptr, nullptr, d_carry, nullptr, nullptr))
        return die("sat_column_totals");
    if ((e = hipMemcpy(upper.data(), d_carry, W * 8, hipMemcpyDeviceToHost))) return hip_die("copy totals", e);

    std::FILE *f = std::fopen(argv[3], "wb");
    if (!f) {
        std::fprintf(stderr, "capi_check: cannot open %s\n", argv[3]);
        return 1;
    }
    const bool ok = append(f, S) && append(f, Q) && append(f, sums) && append(f, m0) && append(f, m1) &&
                    append(f, s1) && append(f, mean) && append(f, stdv) && append(f, B) && append(f, top) &&
                    append(f, upper) && append(f, fin);
    std::fclose(f);
    if (!ok) {
        std::fprintf(stderr, "capi_check: short write\n");
        return 1;
    }
    for (void *p : {d_img, d_ws, static_cast<void *>(d_S), static_cast<void *>(d_Q), static_cast<void *>(d_sum),
                    d_multi[0], d_multi[1], static_cast<void *>(d_s1), static_cast<void *>(d_mean),
                    static_cast<void *>(d_std), static_cast<void *>(d_B), static_cast<void *>(d_top),
                    static_cast<void *>(d_carry), d_bws})
        (void)hipFree(p);
    std::printf("capi_check ok: %lld x %lld\n", static_cast<long long>(H), static_cast<long long>(W));
    return 0;
}
