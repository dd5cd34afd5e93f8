// Host build of the 2-D/3-D reassignment scan (nearest4 and its centre
// tables, prep_centres) from the library's own device header, for the
// certificate fuzz test.  lloyd_device_host.h is that header with its one
// inline-assembly bitfield insert replaced by the same bit operation in C
// (written by the test at build time).
#include "lloyd_device_host.h"

thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;

extern "C" int scan_points_host(const float* X, int64_t N, int64_t ld, int d,
                                const float* mu32, int K, uint32_t xmax_bits,
                                int32_t* arg, int32_t* ok) {
    using namespace km;
    if (K < 1 || K > KMAX || (d != 2 && d != 3)) return -1;
    float4 m32[KMAX];
    for (int k = 0; k < K; ++k)
        m32[k] = make_float4(mu32[4 * k], mu32[4 * k + 1], mu32[4 * k + 2], 0.0f);
    float4 cand[KPAD];
    float4 bnd;
    float sc[KPAD], sa[3 * KPAD];
    // one block's threads in reverse order: every table entry is written
    // before thread 0 forms the bound from them
    for (int t = BLOCK - 1; t >= 0; --t) {
        threadIdx.x = (unsigned)t;
        prep_centres(m32, K, KPAD, cand, &bnd, sc, sa, xmax_bits);
    }
    const float ninf = -INFINITY;
    for (int64_t g = 0; g * 4 < N; ++g) {
        float x[3][4];
        for (int j = 0; j < 3; ++j)
            for (int p = 0; p < 4; ++p)
                x[j][p] = (j < d && g * 4 + p < N) ? X[j * ld + g * 4 + p] : 0.0f;
        float best[4];
        int a[4];
        bool o[4];
        if (d == 3) {
            nearest4<3>(cand, m32, K, bnd, ninf, reinterpret_cast<const float(&)[3][4]>(x), best, a, o);
        } else {
            nearest4<2>(cand, m32, K, bnd, ninf, reinterpret_cast<const float(&)[2][4]>(x), best, a, o);
        }
        for (int p = 0; p < 4 && g * 4 + p < N; ++p) {
            arg[g * 4 + p] = a[p];
            ok[g * 4 + p] = o[p] ? 1 : 0;
        }
    }
    return 0;
}
