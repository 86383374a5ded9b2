// Block conjugate gradients over the s right-hand sides of one grid: dispatch on s and the
// precision, and the Gram kernels (one workgroup per group).  The method and the per-pixel
// kernels are described and defined in sylv_block_impl.h.

#include "sylv_block_impl.h"

namespace sylv {
namespace {

template <int S>
struct STag {
    static constexpr int value = S;
};

template <typename F>
hipError_t dispatch_s(int s, F &&fn) {
    switch (s) {
        case 2: return fn(STag<2>{});
        case 4: return fn(STag<4>{});
        case 8: return fn(STag<8>{});
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int block_rhs_supported(int s) { return s == 2 || s == 4 || s == 8; }

hipError_t launch_bpinit(const GroupSet &g, int k, int mixed, hipStream_t st) {
    return dispatch_s(g.s, [&](auto stag) {
        constexpr int S = decltype(stag)::value;
        return mixed ? BlockLaunch<S, float>::pinit(g, k, st)
                     : BlockLaunch<S, double>::pinit(g, k, st);
    });
}

hipError_t launch_bgram(const GroupSet &g, int phase, int mixed, double inner_tol, double safety,
                        int max_iter, hipStream_t st) {
    return dispatch_s(g.s, [&](auto stag) {
        constexpr int S = decltype(stag)::value;
        hipLaunchKernelGGL((k_bgram_fold<S>), dim3(g.ngroup, gram_n<S>() + S), dim3(kBlock), 0,
                           st, g.groups, phase, mixed);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_bgram<S>), dim3(g.ngroup), dim3(kBlock), 0, st, g.table, g.groups,
                           phase, mixed, inner_tol, safety, max_iter);
        return hipGetLastError();
    });
}

hipError_t launch_bdir(const GroupSet &g, int k, int mixed, int it, hipStream_t st) {
    return dispatch_s(g.s, [&](auto stag) {
        constexpr int S = decltype(stag)::value;
        return mixed ? BlockLaunch<S, float>::dir(g, k, it, st)
                     : BlockLaunch<S, double>::dir(g, k, it, st);
    });
}

hipError_t launch_bapply(const GroupSet &g, int k, int mixed, int it, hipStream_t st) {
    return dispatch_s(g.s, [&](auto stag) {
        constexpr int S = decltype(stag)::value;
        return mixed ? BlockLaunch<S, float>::apply(g, k, it, st)
                     : BlockLaunch<S, double>::apply(g, k, it, st);
    });
}

hipError_t launch_bupdate(const GroupSet &g, int k, int mixed, int it, hipStream_t st) {
    return dispatch_s(g.s, [&](auto stag) {
        constexpr int S = decltype(stag)::value;
        return mixed ? BlockLaunch<S, float>::update(g, k, it, st)
                     : BlockLaunch<S, double>::update(g, k, it, st);
    });
}

}  // namespace sylv
