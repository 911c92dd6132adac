// Host-only stand-in for the HIP runtime header, used to build the library's
// plan, graph and event bookkeeping (flame_api.hip) with the host sanitizers
// (tests/native/plan_bookkeeping_check.cpp). It declares the types and calls
// that file uses; hip_stub.cpp implements them as a checked model of the
// runtime's asynchronous object lifetimes. No device code is built with it.
#pragma once

#include <cstddef>
#include <cstdint>
#include <cmath>

#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define __align__(n) __attribute__((aligned(n)))

struct float2 {
  float x, y;
};
inline float2 make_float2(float x, float y) { return float2{x, y}; }

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
extern dim3 threadIdx, blockIdx, blockDim, gridDim;

enum hipError_t { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorInvalidResourceHandle = 400 };
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3 };
enum hipDeviceAttribute_t {
  hipDeviceAttributeMaxSharedMemoryPerBlock = 74,
  hipDeviceAttributeMultiprocessorCount = 75,
  hipDeviceAttributeWallClockRate = 76,
  hipDeviceAttributeCooperativeLaunch = 77
};

typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef struct ihipGraph* hipGraph_t;
typedef struct hipGraphExec* hipGraphExec_t;
typedef struct hipGraphNode* hipGraphNode_t;

#define hipEventDisableTiming 0x2
#define hipStreamNonBlocking 0x1

struct hipKernelNodeParams {
  dim3 blockDim;
  void** extra;
  void* func;
  dim3 gridDim;
  void** kernelParams;
  unsigned int sharedMemBytes;
};

hipError_t hipGetDevice(int* dev);
hipError_t hipSetDevice(int dev);
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int dev);
hipError_t hipGetLastError(void);
const char* hipGetErrorString(hipError_t e);
hipError_t hipGetSymbolAddress(void** p, const void* symbol);
#define HIP_SYMBOL(X) ((const void*)&(X))
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind k, hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGraphCreate(hipGraph_t* g, unsigned flags);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphAddKernelNode(hipGraphNode_t* node, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps,
                                 const hipKernelNodeParams* p);
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t* err_node, char* log, size_t n);
enum hipKernelNodeAttrID { hipKernelNodeAttributeCooperative = 2 };
union hipKernelNodeAttrValue {
  char pad[64];
  int cooperative;
};
hipError_t hipGraphKernelNodeSetAttribute(hipGraphNode_t node, hipKernelNodeAttrID attr,
                                          const hipKernelNodeAttrValue* value);
hipError_t hipGraphExecDestroy(hipGraphExec_t x);
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s);

// kernel launches record their stream only (nothing runs)
void hip_stub_launch(const void* kernel, hipStream_t s);
#define hipLaunchKernelGGL(kernel, grid, block, lds, stream, ...) hip_stub_launch((const void*)&(kernel), (stream))
