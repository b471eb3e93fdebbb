// Kernel launches that either run now or become nodes of a graph being built.
//
// Graphs are built node by node (hipGraphAddKernelNode), not by stream
// capture: building one then never puts a stream into capture mode, so work
// that other host threads enqueue meanwhile (including on the legacy default
// stream) is unaffected, and nothing they enqueue can enter the graph.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <tuple>
#include <type_traits>
#include <utility>

namespace kfbi {

// The graph this host thread is recording, or null (launches then run on their stream).
struct GraphRec {
    hipGraph_t graph = nullptr;
    hipGraphNode_t last = nullptr;   // nodes form one chain, in launch order
};
GraphRec*& graph_rec();

// Events that the next direct launch from this host thread records from its
// own dispatch packet: the kernel's start and end, without the gap between
// a stream marker and the dispatch.  klaunch clears them after that launch.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents& launch_events();

template <class... KArgs, class... Args>
hipError_t klaunch(void (*kern)(KArgs...), dim3 grid, dim3 block, size_t lds, hipStream_t s, Args&&... args) {
    static_assert(sizeof...(KArgs) == sizeof...(Args), "kernel argument count");
    std::tuple<std::decay_t<KArgs>...> vals(std::forward<Args>(args)...);
    void* params[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1] = {nullptr};
    std::apply([&](auto&... v) {
        int i = 0;
        ((params[i++] = static_cast<void*>(&v)), ...);
    }, vals);
    GraphRec* r = graph_rec();
    if (!r) {
        LaunchEvents& le = launch_events();
        if (le.start || le.stop) {
            const LaunchEvents use = le;
            le = LaunchEvents{};
            return hipExtLaunchKernel(reinterpret_cast<const void*>(kern), grid, block, params, lds, s, use.start,
                                      use.stop, 0);
        }
        return hipLaunchKernel(reinterpret_cast<const void*>(kern), grid, block, params, lds, s);
    }
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(kern);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = static_cast<unsigned>(lds);
    kp.kernelParams = params;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    const hipError_t e = hipGraphAddKernelNode(&node, r->graph, r->last ? &r->last : nullptr, r->last ? 1 : 0, &kp);
    if (e == hipSuccess) r->last = node;
    return e;
}

}  // namespace kfbi
