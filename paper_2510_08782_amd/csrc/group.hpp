// Kernel launches that can be merged across the size classes of a group
// handle (independent batches of different grid sizes run as one handle).
//
// Every kernel of the library is written as a body,
//     struct XBody { static constexpr int kBlock; struct-or-alias Args;
//                    __device__ static void run(const Args&, const Blk&); }
// that reads its workgroup coordinates from a Blk instead of blockIdx /
// gridDim.  A launch goes through submit<Body, GBody>():
//   * outside a group handle it is an ordinary launch of single_kernel<Body>;
//   * inside one (a class running under the cooperative scheduler of
//     runtime.hip) the launch is handed to the scheduler, which waits until
//     every class has reached its next launch or synchronisation point and
//     then issues the launches of one family (same GBody) as ONE launch of
//     grouped_kernel<GBody>: the workgroups of class c occupy the flat range
//     [begin[c], begin[c+1]) of the grid and see their own coordinates.
// GBody has the same Args as Body and may dispatch at run time on them (the
// transform length, the tile variant), so that classes whose Body differs
// only in such compile-time constants still merge.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <type_traits>

namespace gan {

// Workgroup coordinates of a body (x, y) within its own grid (gx, gy).
struct Blk {
    unsigned x, y, gx, gy;
};

constexpr int kMaxGroup = 4;        // classes per merged launch
constexpr int kMaxArgBytes = 1024;  // arguments of one class's launch
constexpr unsigned kGroupAlign = 8; // class ranges start at multiples of the XCD count

struct LaunchDesc;
struct LaunchFamily {
    hipError_t (*launch_group)(const LaunchDesc* const* d, int n, hipStream_t st);
};
struct LaunchDesc {
    const LaunchFamily* fam;
    hipError_t (*launch_single)(const LaunchDesc& d, hipStream_t st);
    unsigned gx, gy;
    size_t lds;
    alignas(16) unsigned char args[kMaxArgBytes];
};

// The cooperative scheduler (runtime.hip): the task of the class running on
// this thread, or nullptr outside a group handle; handing over a launch
// returns once the scheduler has issued it (throws what the launch failed
// with).
struct CoopTask;
CoopTask* coop_current();
void coop_launch(CoopTask* t, const LaunchDesc& d);

template <class Body>
__global__ void __launch_bounds__(Body::kBlock) single_kernel(typename Body::Args a) {
    Body::run(a, Blk{blockIdx.x, blockIdx.y, gridDim.x, gridDim.y});
}

template <class Args>
struct GroupArgs {
    int n;
    unsigned begin[kMaxGroup + 1];
    unsigned gx[kMaxGroup], gy[kMaxGroup];
    Args a[kMaxGroup];
};

template <class Body>
__global__ void __launch_bounds__(Body::kBlock) grouped_kernel(GroupArgs<typename Body::Args> g) {
    int c = 0;
    while (c + 1 < g.n && blockIdx.x >= g.begin[c + 1]) ++c;
    const unsigned local = blockIdx.x - g.begin[c];
    if (local >= g.gx[c] * g.gy[c]) return;
    Body::run(g.a[c], Blk{local % g.gx[c], local / g.gx[c], g.gx[c], g.gy[c]});
}

template <class GBody>
hipError_t launch_group_impl(const LaunchDesc* const* d, int n, hipStream_t st) {
    using Args = typename GBody::Args;
    static_assert(sizeof(GroupArgs<Args>) <= 4096, "merged launch arguments too large");
    GroupArgs<Args> g;
    std::memset(static_cast<void*>(&g), 0, sizeof g);
    g.n = n;
    unsigned off = 0;
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
        g.begin[i] = off;
        g.gx[i] = d[i]->gx;
        g.gy[i] = d[i]->gy;
        std::memcpy(static_cast<void*>(&g.a[i]), d[i]->args, sizeof(Args));
        off += (d[i]->gx * d[i]->gy + kGroupAlign - 1) / kGroupAlign * kGroupAlign;
        lds = d[i]->lds > lds ? d[i]->lds : lds;
    }
    g.begin[n] = off;
    grouped_kernel<GBody><<<off, GBody::kBlock, lds, st>>>(g);
    return hipGetLastError();
}

template <class GBody>
const LaunchFamily* launch_family() {
    static const LaunchFamily f{&launch_group_impl<GBody>};
    return &f;
}

template <class Body>
hipError_t launch_single_impl(const LaunchDesc& d, hipStream_t st) {
    typename Body::Args a;
    std::memcpy(static_cast<void*>(&a), d.args, sizeof a);
    single_kernel<Body><<<dim3(d.gx, d.gy), Body::kBlock, d.lds, st>>>(a);
    return hipGetLastError();
}

// Launch Body over grid (x, y) with lds bytes of dynamic LDS; inside a group
// handle the launch may be merged with the other classes' launches of GBody.
template <class Body, class GBody = Body>
void submit(dim3 grid, size_t lds, hipStream_t st, const typename Body::Args& a) {
    static_assert(std::is_same<typename Body::Args, typename GBody::Args>::value,
                  "a merged family shares its arguments");
    static_assert(sizeof(typename Body::Args) <= kMaxArgBytes, "launch arguments too large");
    static_assert(Body::kBlock == GBody::kBlock, "a merged family shares its workgroup size");
    CoopTask* t = coop_current();
    if (!t) {
        single_kernel<Body><<<grid, Body::kBlock, lds, st>>>(a);
        return;
    }
    LaunchDesc d;
    d.fam = launch_family<GBody>();
    d.launch_single = &launch_single_impl<Body>;
    d.gx = grid.x;
    d.gy = grid.y;
    d.lds = lds;
    std::memcpy(d.args, static_cast<const void*>(&a), sizeof a);
    coop_launch(t, d);
}

// An ordinary launch of Body, never merged (arguments too large to merge).
template <class Body>
void launch_now(dim3 grid, size_t lds, hipStream_t st, const typename Body::Args& a) {
    single_kernel<Body><<<grid, Body::kBlock, lds, st>>>(a);
}

}  // namespace gan
