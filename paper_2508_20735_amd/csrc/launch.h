// Kernel launches that go either to a stream or, while a graph is being
// built on the calling thread, into that graph as kernel nodes.
//
// Round graphs are built node by node instead of being captured from a
// stream: a stream capture can be invalidated by a call that another thread
// makes meanwhile, and a capture left invalidated blocks its stream; a graph
// built through the graph API depends on no stream state.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <tuple>
#include <utility>

namespace dfamin {

// A graph under construction.  Each launch appends a kernel node that
// depends on the previous one: the order the stream would have kept.
struct GraphRecorder {
    hipGraph_t graph = nullptr;
    hipGraphNode_t last = nullptr;
    hipError_t error = hipSuccess;
};

// The calling thread's recorder (nullptr: launches go to their stream).
GraphRecorder *&graph_recorder();

template <typename... P, typename... A>
void launch_kernel(void (*kernel)(P...), dim3 grid, dim3 block, uint32_t shmem, hipStream_t s,
                   A &&...args) {
    static_assert(sizeof...(P) == sizeof...(A), "argument count");
    GraphRecorder *rec = graph_recorder();
    if (!rec) {
        hipLaunchKernelGGL(kernel, grid, block, shmem, s, std::forward<A>(args)...);
        return;
    }
    if (rec->error != hipSuccess) return;
    // the node copies the argument values when it is added
    std::tuple<P...> values(std::forward<A>(args)...);
    void *ptrs[sizeof...(P) + 1] = {};
    std::apply(
        [&ptrs](auto &...v) {
            size_t i = 0;
            ((ptrs[i++] = static_cast<void *>(&v)), ...);
        },
        values);
    hipKernelNodeParams np{};
    np.func = reinterpret_cast<void *>(kernel);
    np.gridDim = grid;
    np.blockDim = block;
    np.sharedMemBytes = shmem;
    np.kernelParams = ptrs;
    np.extra = nullptr;
    hipGraphNode_t node = nullptr;
    rec->error = hipGraphAddKernelNode(&node, rec->graph, rec->last ? &rec->last : nullptr,
                                       rec->last ? 1 : 0, &np);
    if (rec->error == hipSuccess) rec->last = node;
}

}  // namespace dfamin
