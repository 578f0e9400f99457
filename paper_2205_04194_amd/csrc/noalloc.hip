// The fast product for callers that cannot allocate device memory (code
// under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
// imq_matvec_noalloc.  The same kernels as imq_matvec, with every per-product
// workspace of the tree (gathered weights, multipole and local expansions,
// X-list partial expansions, W-list partial sums, the FP64 result
// accumulator) carved from one file-scope device array instead of the
// tree's own workspace buffers, which are allocated on first use.  All
// stages run in order on the caller's stream (the overlapped schedule needs
// streams and events the tree creates on first use).
#include "device.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

namespace imq {

template <typename T, typename Tio>
imq_status matvec_typed(imq_tree_s *t, int nrhs, const Tio *u, int64_t ldu, Tio *b, int64_t ldb,
                        hipStream_t s);
void set_serial_product(bool on);

namespace {

// The workspace of every call on a device.  In host code `scratch` names a
// host-side stand-in, not device memory: the device address comes from
// hipGetSymbolAddress (per device) and only that address is used.
constexpr size_t SCRATCH_BYTES = size_t(128) << 20;
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// The device address of this device's copy of `scratch`, looked up once per
// device with that device current.
imq_status scratch_address(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("device ordinal beyond the devices the workspace table holds");
        return IMQ_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return IMQ_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[dev]);
    return IMQ_OK;
}

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// The workspace buffers of one product in arithmetic T with nrhs columns,
// and their offsets in the scratch array.
struct Layout {
    size_t us, M, L, Lx, bs, Pw, total;
};

template <typename T>
Layout layout(const imq_tree_s *t, int nrhs)
{
    const size_t nbox = t->h.level.size(), N = size_t(t->h.N), r = size_t(nrhs);
    Layout l;
    size_t o = 0;
    l.us = o; o += align256(sizeof(T) * N * r);
    l.M = o;  o += align256(sizeof(T) * nbox * r * coef_stride(t->h.K));
    l.L = o;  o += align256(sizeof(T) * nbox * r * coef_stride(t->h.K));
    l.Lx = o; o += align256(sizeof(T) * size_t(t->nxpairs) * r * t->h.K);
    l.bs = o; o += align256(sizeof(double) * N * r);
    l.Pw = o; o += align256(sizeof(double) * size_t(t->nwscr) * r);
    l.total = o;
    return l;
}

// Puts views of the scratch array in place of the tree's workspace buffers
// for one call and restores the tree's own buffers (untouched, still owned
// by the tree) when the call returns, on every path.
template <typename T>
struct WorkspaceSwap {
    imq_tree_s *t;
    PrecData &pd;
    DevBuf us, M, L, Lx, bs, Pw;
    size_t ws_nrhs, lx_nrhs, bs_nrhs;
    WorkspaceSwap(imq_tree_s *tree, unsigned char *base, const Layout &l, int nrhs)
        : t(tree), pd(prec_data<T>(tree)), us(pd.us), M(pd.M), L(pd.L), Lx(pd.Lx), bs(tree->bs),
          Pw(tree->Pw), ws_nrhs(pd.ws_nrhs), lx_nrhs(pd.lx_nrhs), bs_nrhs(tree->bs_nrhs)
    {
        auto view = [&](size_t off, size_t end) { return DevBuf{base + off, end - off, nullptr}; };
        pd.us = view(l.us, l.M);
        pd.M = view(l.M, l.L);
        pd.L = view(l.L, l.Lx);
        pd.Lx = view(l.Lx, l.bs);
        t->bs = view(l.bs, l.Pw);
        t->Pw = view(l.Pw, l.total);
        pd.ws_nrhs = pd.lx_nrhs = t->bs_nrhs = size_t(nrhs);   // large enough: nothing is allocated
    }
    ~WorkspaceSwap()
    {
        pd.us = us; pd.M = M; pd.L = L; pd.Lx = Lx;
        t->bs = bs; t->Pw = Pw;
        pd.ws_nrhs = ws_nrhs; pd.lx_nrhs = lx_nrhs; t->bs_nrhs = bs_nrhs;
    }
};

struct SerialProduct {
    SerialProduct() { set_serial_product(true); }
    ~SerialProduct() { set_serial_product(false); }
};

template <typename T, typename Tio>
imq_status matvec_noalloc_typed(imq_tree_s *t, unsigned char *base, int nrhs, const Tio *u, int64_t ldu, Tio *b,
                                int64_t ldb, hipStream_t s)
{
    const Layout l = layout<T>(t, nrhs);
    if (l.total > SCRATCH_BYTES) {
        set_error("imq_matvec_noalloc: the product needs " + std::to_string(l.total) +
                  " bytes of workspace, more than the fixed " + std::to_string(SCRATCH_BYTES));
        return IMQ_EINVAL;
    }
    WorkspaceSwap<T> swap(t, base, l, nrhs);
    SerialProduct serial;
    return matvec_typed<T, Tio>(t, nrhs, u, ldu, b, ldb, s);
}

}  // namespace

imq_status matvec_noalloc(imq_tree_s *t, int nrhs, imq_dtype dtype, const void *u, int64_t ldu, void *b,
                          int64_t ldb, imq_prec prec, hipStream_t s)
{
    unsigned char *base = nullptr;
    imq_status st = scratch_address(t->device, &base);
    if (st != IMQ_OK) return st;
    if (dtype == IMQ_F64 && prec == IMQ_PREC_FP64)
        return matvec_noalloc_typed<double, double>(t, base, nrhs, (const double *)u, ldu, (double *)b, ldb, s);
    if (dtype == IMQ_F32 && prec == IMQ_PREC_FP64)
        return matvec_noalloc_typed<double, float>(t, base, nrhs, (const float *)u, ldu, (float *)b, ldb, s);
    if (dtype == IMQ_F64 && prec == IMQ_PREC_FP32)
        return matvec_noalloc_typed<float, double>(t, base, nrhs, (const double *)u, ldu, (double *)b, ldb, s);
    if (dtype == IMQ_F32 && prec == IMQ_PREC_FP32)
        return matvec_noalloc_typed<float, float>(t, base, nrhs, (const float *)u, ldu, (float *)b, ldb, s);
    set_error("unknown dtype or precision");
    return IMQ_EINVAL;
}

size_t noalloc_scratch_bytes() { return SCRATCH_BYTES; }

}  // namespace imq
