// Host-only stand-in for the part of the HIP runtime API that the serving
// front end calls, so that its scheduling can be exercised on the CPU.
// "Device" memory is host memory; copies run at once; an event reports
// completion only after a number of queries chosen by the test, so work
// appears to stay in flight for a while.
#ifndef MOCK_HIP_RUNTIME_API_H
#define MOCK_HIP_RUNTIME_API_H

#include <stddef.h>
#include <stdlib.h>
#include <string.h>

typedef enum {
  hipSuccess = 0,
  hipErrorOutOfMemory = 2,
  hipErrorLaunchFailure = 719,
  hipErrorNotReady = 600,
} hipError_t;

typedef enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 } hipMemcpyKind;

#define hipStreamNonBlocking 1u
#define hipEventDisableTiming 2u
#define hipHostMallocDefault 0u

struct MockStream {
  int id;
};
struct MockEvent {
  int pending;  // queries left before it reports completion
  bool recorded;
};
typedef MockStream* hipStream_t;
typedef MockEvent* hipEvent_t;

// queries an event takes to complete after each record (set by the test)
extern int (*mock_event_latency)(void);
extern int mock_live_streams, mock_live_events, mock_live_pinned;

inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  static int next = 0;
  *s = new MockStream{next++};
  mock_live_streams++;
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  mock_live_streams--;
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new MockEvent{0, false};
  mock_live_events++;
  return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  mock_live_events--;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  e->pending = mock_event_latency ? mock_event_latency() : 0;
  e->recorded = true;
  return hipSuccess;
}
inline hipError_t hipEventQuery(hipEvent_t e) {
  if (!e->recorded) return hipErrorLaunchFailure;  // the server queries only recorded events
  if (e->pending > 0) {
    e->pending--;
    return hipErrorNotReady;
  }
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  memmove(dst, src, n);
  return hipSuccess;
}
inline hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
                                   size_t height, hipMemcpyKind, hipStream_t) {
  for (size_t r = 0; r < height; r++)
    memmove(static_cast<char*>(dst) + r * dpitch, static_cast<const char*>(src) + r * spitch, width);
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
  *p = malloc(n);
  if (!*p) return hipErrorOutOfMemory;
  mock_live_pinned++;
  return hipSuccess;
}
inline hipError_t hipHostFree(void* p) {
  free(p);
  mock_live_pinned--;
  return hipSuccess;
}

#endif
