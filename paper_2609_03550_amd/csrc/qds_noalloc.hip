// Loss evaluation that allocates nothing (qds_loss_eval_noalloc in
// include/qds.h), for callers that cannot call hipMalloc: code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation.
//
// qds_loss_eval without a gradient buffer takes a temporary state-sized
// allocation for the gradient its seed kernel writes.  This variant computes
// the loss alone: each workgroup reduces a 64-column x 4-row tile of the loss
// window and stores its partial sum in the file-scope device array
// ``scratch``; one more workgroup then adds the partials in a fixed order and
// adds the total to the caller's device double.  Every call on a GPU shares
// that GPU's array (it is overwritten, never read before being written), so
// calls that overlap on one GPU race; calls on one stream are ordered.
#include <mutex>

#include "qds_ctx.hpp"

using namespace qdsi;

namespace {

// 65536 partial sums (512 KiB per GPU, held until the process ends): the
// loss window may span at most this many 64 x 4 tiles.
constexpr int kScratchDoubles = 65536;
__device__ __align__(256) double scratch[kScratchDoubles];

// Device address of ``scratch`` per device, looked up once per device with
// that device current.  The array's name in host code is a host-side stand-in,
// never a device address.
constexpr int kMaxDevices = 64;
double* g_scratch_dev[kMaxDevices];
std::mutex g_scratch_mu;

hipError_t scratch_ptr(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// Same loss as the seed kernel of qds_loss_eval (energy of one mode of one
// set over columns [x0, x1); transverse fields with weight 1/4, E_x and B_x
// with 1/2; area r dr with the axis row at dr/8; mode weight 2 pi or pi).
// Block (bx, by) covers columns x0 + 64 bx .. +63 and rows 4 by .. +3 and
// writes its partial to part[by * gridDim.x + bx].
template <typename T>
__global__ void __launch_bounds__(256) k_loss_partial(qds::SetPtr<T> u, qds::Geo g, int md, int x0, int x1,
                                                     double* part) {
    const int i = x0 + blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    double acc = 0.0;
    if (i < x1 && j <= g.nr) {
        const double pi = 3.141592653589793;
        const double w = (md == 0 ? 2.0 * pi : pi) * g.h * g.dr;
        const double rk = (j + 0.5) * g.dr;
        const double rj = j == 0 ? g.dr / 8.0 : j * g.dr;
        auto one = [&](const qds::cx<T>* p, double c) {
            const qds::cx<T> v = qds::ld(p + g.at(md, j, i));
            acc += c * (double(v.re) * v.re + double(v.im) * v.im);
        };
        if (j < g.nr) {
            one(u.trp, 0.25 * w * rk);
            one(u.trm, 0.25 * w * rk);
            one(u.bx, 0.5 * w * rk);
        }
        one(u.ttp, 0.25 * w * rj);
        one(u.ttm, 0.25 * w * rj);
        one(u.ex, 0.5 * w * rj);
    }
    __shared__ double red[256];
    const int t = threadIdx.y * 64 + threadIdx.x;
    red[t] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// Sum of n partials in a fixed order (thread t takes t, t + 256, ...; then a
// tree), added to *out.
__global__ void __launch_bounds__(256) k_loss_finish(const double* part, int n, double* out) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int q = t; q < n; q += 256) acc += part[q];
    red[t] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    if (t == 0) atomicAdd(out, red[0]);
}

template <typename T>
hipError_t launch(const qds_ctx* h, const void* buf, const qds_loss* L, double* out, double* part, dim3 grd,
                  hipStream_t s) {
    qds::cx<T>* U[QDS_NPLANES];
    plane_table<T>(h, const_cast<void*>(buf), U);
    const int b = 9 * L->set;
    qds::SetPtr<T> u{U[b + 0], U[b + 1], U[b + 2], U[b + 3], U[b + 4], U[b + 5], U[b + 6], U[b + 7], U[b + 8]};
    hipLaunchKernelGGL(k_loss_partial<T>, grd, dim3(64, 4), 0, s, u, geo(h), L->mode, L->x_begin, L->x_end, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, s, static_cast<const double*>(part),
                       int(grd.x * grd.y), out);
    return hipGetLastError();
}

}  // namespace

extern "C" qds_status qds_loss_eval_noalloc(qds_handle h, const void* buf, const qds_loss* loss, double* out_dev,
                                            void* stream) {
    if (!h || !buf || !loss || !out_dev) return fail(h, QDS_EINVAL, "null argument%s");
    if (loss->set < 0 || loss->set > 1 || (loss->set == 1 && !has(h, QDS_P_SET1)))
        return fail(h, QDS_EINVAL, "loss set not in the state%s");
    if (loss->mode < 0 || loss->mode >= h->M) return fail(h, QDS_EINVAL, "loss mode out of range%s");
    if (loss->x_begin < 0 || loss->x_end > h->g.nx || loss->x_begin >= loss->x_end)
        return fail(h, QDS_EINVAL, "loss column range must satisfy 0 <= x_begin < x_end <= nx%s");
    const dim3 grd((loss->x_end - loss->x_begin + 63) / 64, (h->g.nr + 1 + 3) / 4);
    if (size_t(grd.x) * size_t(grd.y) > size_t(kScratchDoubles))
        return fail(h, QDS_EINVAL,
                    "loss window too large for the static scratch: ceil(columns/64) * ceil((nr+1)/4) must be <= "
                    "65536%s");
    double* part = nullptr;
    hipError_t e = scratch_ptr(&part);
    if (e != hipSuccess) return fail(h, QDS_EHIP, "looking up the static scratch failed: %s", hipGetErrorString(e));
    e = h->g.dtype == QDS_F64 ? launch<double>(h, buf, loss, out_dev, part, grd, hipStream_t(stream))
                              : launch<float>(h, buf, loss, out_dev, part, grd, hipStream_t(stream));
    if (e != hipSuccess) return fail(h, QDS_EHIP, "launch failed: %s", hipGetErrorString(e));
    return QDS_OK;
}
