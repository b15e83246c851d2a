// xfer.hip — conversions between the boundary particle layout (linear cell index) and the
// packed cell code used inside the library.
#include "pic_internal.h"

namespace pic {

__global__ __launch_bounds__(kBlock) void lin_to_packed_kernel(const int32_t* lin, int32_t* packed,
                                                               int64_t n, int nx, int ny, int nz,
                                                               CellCode cc, uint32_t* err)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t c = lin[i];
    if (c < 0 || (int64_t)c >= (int64_t)nx * ny * nz) {
        packed[i] = cc.encode(0, 0, 0);
        atomicOr(err, 8u);
        return;
    }
    const int x = c % nx;
    const int r = c / nx;
    packed[i] = cc.encode(x, r % ny, r / ny);
}

__global__ __launch_bounds__(kBlock) void packed_to_lin_kernel(const int32_t* packed, int32_t* lin,
                                                               int64_t n, int nx, int ny,
                                                               CellCode cc)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t c = packed[i];
    if (c < 0) {
        lin[i] = -1;
        return;
    }
    int x, y, z;
    cc.decode(c, x, y, z);
    lin[i] = x + nx * (y + ny * z);
}

__global__ __launch_bounds__(kBlock) void iota_kernel(uint32_t* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = (uint32_t)i;
}

// Plain streaming copy in 16-byte words (the reference kernel of known traffic used to scale
// hardware memory counters).
__global__ __launch_bounds__(kBlock) void copy_kernel(uint4* __restrict__ dst,
                                                      const uint4* __restrict__ src, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ void set_i32_kernel(int32_t* p, int32_t v) { *p = v; }

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t cells_linear_to_packed(const int32_t* lin, int32_t* packed, int64_t n, const int nn[3],
                                  CellCode cc, uint32_t* err, hipStream_t st)
{
    if (n > 0)
        lin_to_packed_kernel<<<nblk(n), kBlock, 0, st>>>(lin, packed, n, nn[0], nn[1], nn[2], cc, err);
    return hipGetLastError();
}

hipError_t cells_packed_to_linear(const int32_t* packed, int32_t* lin, int64_t n, const int nn[3],
                                  CellCode cc, hipStream_t st)
{
    if (n > 0) packed_to_lin_kernel<<<nblk(n), kBlock, 0, st>>>(packed, lin, n, nn[0], nn[1], cc);
    return hipGetLastError();
}

hipError_t device_copy16(void* dst, const void* src, int64_t nwords, hipStream_t st)
{
    if (nwords > 0) {
        const int64_t want = (nwords + kBlock - 1) / kBlock;
        const unsigned grid = (unsigned)(want < 256 * 64 ? want : 256 * 64);
        copy_kernel<<<grid, kBlock, 0, st>>>(static_cast<uint4*>(dst), static_cast<const uint4*>(src),
                                             nwords);
    }
    return hipGetLastError();
}

hipError_t set_i32(int32_t* p, int32_t v, hipStream_t st)
{
    set_i32_kernel<<<1, 1, 0, st>>>(p, v);
    return hipGetLastError();
}

hipError_t iota_u32(uint32_t* p, int64_t n, hipStream_t st)
{
    if (n > 0) iota_kernel<<<nblk(n), kBlock, 0, st>>>(p, n);
    return hipGetLastError();
}

}  // namespace pic
