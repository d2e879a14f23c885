// Library GEMMs for the surrogate's training products (plain BF16 x BF16 ->
// FP32 matrix products with no fused epilogue): hipBLASLt, column-major.
//
// A GemmArgs product C[M][N] (row-major, ldc) = sum_k A(i, k) B(k, j) is the
// column-major product D (N x M, ld ldc) = X (N x K) Y (K x M) with
// X(j, k) = B(k, j) and Y(k, i) = A(i, k); a unit stride along k or along the
// other index of an operand gives its stored column-major matrix and whether
// it enters transposed.  Descriptors and the heuristic's algorithm are cached
// per shape; the workspace is the context's.
#include <hipblaslt/hipblaslt.h>

#include <map>
#include <tuple>

#include "engine.h"

namespace lidar {

namespace {

struct Plan {
    hipblasLtMatmulDesc_t desc = nullptr;
    hipblasLtMatrixLayout_t a = nullptr, b = nullptr, d = nullptr;
    hipblasLtMatmulAlgo_t algo{};
    size_t ws = 0;
};

using Key = std::tuple<int, int, int, int, int, long, long, long>;

}  // namespace

struct BlasCtx {
    hipblasLtHandle_t handle = nullptr;
    std::map<Key, Plan> plans;
    DevBuf<char> ws;
};

constexpr size_t kBlasMaxWorkspace = 32u << 20;

BlasCtx* blas_create()
{
    BlasCtx* c = new (std::nothrow) BlasCtx();
    if (!c) return nullptr;
    if (hipblasLtCreate(&c->handle) != HIPBLAS_STATUS_SUCCESS) {
        delete c;
        return nullptr;
    }
    return c;
}

void blas_destroy(BlasCtx* c)
{
    if (!c) return;
    for (auto& kv : c->plans) {
        Plan& p = kv.second;
        if (p.a) hipblasLtMatrixLayoutDestroy(p.a);
        if (p.b) hipblasLtMatrixLayoutDestroy(p.b);
        if (p.d) hipblasLtMatrixLayoutDestroy(p.d);
        if (p.desc) hipblasLtMatmulDescDestroy(p.desc);
    }
    if (c->handle) hipblasLtDestroy(c->handle);
    delete c;
}

hipError_t blas_gemm(BlasCtx* c, hipStream_t s, const GemmArgs& g)
{
    if (!c || g.M <= 0 || g.N <= 0) return g.M <= 0 || g.N <= 0 ? hipSuccess : hipErrorNotSupported;
    // X (N x K): from B; Y (K x M): from A
    hipblasOperation_t opx, opy;
    long ldx, ldy;
    if (g.sbn == 1) {
        opx = HIPBLAS_OP_N;                       // stored N x K, column k at k * sbk
        ldx = g.sbk;
    } else if (g.sbk == 1) {
        opx = HIPBLAS_OP_T;                       // stored K x N, column j at j * sbn
        ldx = g.sbn;
    } else {
        return hipErrorNotSupported;
    }
    if (g.sak == 1) {
        opy = HIPBLAS_OP_N;                       // stored K x M, column i at i * sam
        ldy = g.sam;
    } else if (g.sam == 1) {
        opy = HIPBLAS_OP_T;                       // stored M x K, column k at k * sak
        ldy = g.sak;
    } else {
        return hipErrorNotSupported;
    }
    const Key key{g.M, g.N, g.K, (int)opx, (int)opy, ldx, ldy, g.ldc};
    auto it = c->plans.find(key);
    if (it == c->plans.end()) {
        Plan p;
        bool ok = hipblasLtMatmulDescCreate(&p.desc, HIPBLAS_COMPUTE_32F, HIP_R_32F) == HIPBLAS_STATUS_SUCCESS;
        const int32_t ta = opx, tb = opy;
        ok = ok && hipblasLtMatmulDescSetAttribute(p.desc, HIPBLASLT_MATMUL_DESC_TRANSA, &ta, sizeof(ta)) ==
                       HIPBLAS_STATUS_SUCCESS;
        ok = ok && hipblasLtMatmulDescSetAttribute(p.desc, HIPBLASLT_MATMUL_DESC_TRANSB, &tb, sizeof(tb)) ==
                       HIPBLAS_STATUS_SUCCESS;
        // stored shapes: X is N x K (or K x N), Y is K x M (or M x K), D is N x M
        ok = ok && hipblasLtMatrixLayoutCreate(&p.a, HIP_R_16BF, opx == HIPBLAS_OP_N ? g.N : g.K,
                                               opx == HIPBLAS_OP_N ? g.K : g.N, ldx) == HIPBLAS_STATUS_SUCCESS;
        ok = ok && hipblasLtMatrixLayoutCreate(&p.b, HIP_R_16BF, opy == HIPBLAS_OP_N ? g.K : g.M,
                                               opy == HIPBLAS_OP_N ? g.M : g.K, ldy) == HIPBLAS_STATUS_SUCCESS;
        ok = ok && hipblasLtMatrixLayoutCreate(&p.d, HIP_R_32F, g.N, g.M, g.ldc) == HIPBLAS_STATUS_SUCCESS;
        hipblasLtMatmulPreference_t pref = nullptr;
        ok = ok && hipblasLtMatmulPreferenceCreate(&pref) == HIPBLAS_STATUS_SUCCESS;
        const uint64_t wmax = kBlasMaxWorkspace;
        ok = ok && hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &wmax,
                                                         sizeof(wmax)) == HIPBLAS_STATUS_SUCCESS;
        hipblasLtMatmulHeuristicResult_t res{};
        int n = 0;
        ok = ok && hipblasLtMatmulAlgoGetHeuristic(c->handle, p.desc, p.a, p.b, p.d, p.d, pref, 1, &res, &n) ==
                       HIPBLAS_STATUS_SUCCESS && n > 0;
        if (pref) hipblasLtMatmulPreferenceDestroy(pref);
        if (!ok) {
            if (p.a) hipblasLtMatrixLayoutDestroy(p.a);
            if (p.b) hipblasLtMatrixLayoutDestroy(p.b);
            if (p.d) hipblasLtMatrixLayoutDestroy(p.d);
            if (p.desc) hipblasLtMatmulDescDestroy(p.desc);
            return hipErrorNotSupported;
        }
        p.algo = res.algo;
        p.ws = res.workspaceSize;
        it = c->plans.emplace(key, p).first;
    }
    const Plan& p = it->second;
    if (p.ws > 0) {
        const hipError_t e = c->ws.ensure(p.ws);
        if (e != hipSuccess) return e;
    }
    const float one = 1.0f, zero = 0.0f;
    const hipblasStatus_t st = hipblasLtMatmul(c->handle, p.desc, &one, g.B, p.a, g.A, p.b, &zero, g.C, p.d,
                                               g.C, p.d, &p.algo, p.ws ? c->ws.p : nullptr, p.ws, s);
    return st == HIPBLAS_STATUS_SUCCESS ? hipSuccess : hipErrorLaunchFailure;
}

}  // namespace lidar
