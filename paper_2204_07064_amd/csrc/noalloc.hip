// stream_process_noalloc: stream_process for callers that cannot allocate
// device memory while processing (graph capture, tight serving loops).
//
// The step's workspace (every layer's activation buffer and operand copy)
// and its descriptor live in one fixed device array, `scratch`, instead of
// the model's growable workspace and descriptor ring.  Each device holds its
// own copy of the array from library load until the process ends; its
// device address is resolved once per device when the first model is
// created there (scratch_setup) and only that address is ever handed to
// kernels.  All calls on one device share the array: calls whose work
// overlaps on the device race and must be serialized by the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "model_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)SC_NOALLOC_SCRATCH_BYTES;
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;
constexpr int kMaxBuffers = 64;   // workspace buffers + operand copies of one plan

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` per device

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Writes a one-stream step descriptor: header, the entry, and the granule
// table (every granule belongs to entry 0).
__global__ void write_desc_kernel(sc::Entry e, int32_t frames, int32_t n_gran, unsigned char* desc) {
  int32_t* hdr = reinterpret_cast<int32_t*>(desc);
  sc::Entry* ents = reinterpret_cast<sc::Entry*>(desc + sc::kDescHeaderBytes);
  int32_t* fent = reinterpret_cast<int32_t*>(desc + sc::kDescHeaderBytes + sizeof(sc::Entry));
  const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i == 0) {
    hdr[0] = 1;
    hdr[1] = frames;
    ents[0] = e;
  }
  for (int32_t g = i; g < n_gran; g += (int32_t)(gridDim.x * blockDim.x)) fent[g] = 0;
}

}  // namespace

hipError_t sc::scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = p;
  return hipSuccess;
}

extern "C" sc_status stream_process_noalloc(sc_stream* s, const float* d_in, int32_t n_frames, float* d_out,
                                            void* hip_stream) {
  if (!s) return sc::fail_status(SC_EINVAL, "null stream");
  sc_model* m = s->m;
  std::lock_guard<std::mutex> g(m->mu);
  if (m->prof_on || m->amax_on)
    return sc::fail_status(SC_EINVAL, "stream_process_noalloc does not run with profiling or calibration on");
  int64_t total = 0;
  sc_status st = sc::validate_step(m, 1, &s, &d_in, &n_frames, &d_out, &total);
  if (st != SC_OK) return st;
  const sc::Plan& pl = m->plan;
  if (pl.buf_floats.size() > (size_t)kMaxBuffers || pl.twin_elems.size() > (size_t)kMaxBuffers)
    return sc::fail_status(SC_EINVAL, "model has more workspace buffers than the no-alloc path supports");
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> gs(g_mu);
    if (m->device >= 0 && m->device < kMaxDevices) base = static_cast<unsigned char*>(g_scratch[m->device]);
  }
  if (!base) return sc::fail_status(SC_ESTATE, "scratch array of this device was not set up");

  // layout: descriptor, then each activation buffer, then each operand copy,
  // every region 256-byte aligned and sized as the model's own workspace
  // would be for a step of `total` input frames
  const int64_t gr = pl.input_multiple;
  size_t off = round_up(sc::desc_bytes(1, total, gr));
  float* ws[kMaxBuffers];
  void* tw[kMaxBuffers];
  for (size_t b = 0; b < pl.buf_floats.size(); ++b) {
    ws[b] = reinterpret_cast<float*>(base + off);
    off += round_up((size_t)(pl.buf_floats[b].of(total) + 1) * sizeof(float));
  }
  for (size_t t = 0; t < pl.twin_elems.size(); ++t) {
    tw[t] = base + off;
    off += round_up((size_t)(pl.twin_elems[t].of(total) * pl.twin_esize[t] + 64));
  }
  if (off > kScratchBytes)
    return sc::fail_status(SC_ELENGTH, ("buffer needs " + std::to_string(off) + " bytes of scratch; the no-alloc path "
                                        "holds " + std::to_string(kScratchBytes) + " (use fewer frames per call)").c_str());

  hipError_t e = hipSetDevice(m->device);
  if (e != hipSuccess) return sc::fail_status(SC_EDEVICE, "hipSetDevice failed");
  const hipStream_t hs = static_cast<hipStream_t>(hip_stream);
  sc::Entry en;
  std::memset(&en, 0, sizeof(en));
  en.in = d_in;
  en.out = d_out;
  en.state = s->d_state;
  en.T = n_frames;
  en.off = 0;
  en.parity = s->parity;
  en.flags = (int32_t)s->flags;
  en.pos = s->pos;
  en.end = s->end;
  const int32_t n_gran = (int32_t)((total + gr - 1) / gr);
  const unsigned threads = 256, blocks = (unsigned)std::min<int32_t>(std::max<int32_t>((n_gran + 255) / 256, 1), 64);
  write_desc_kernel<<<blocks, threads, 0, hs>>>(en, (int32_t)total, n_gran, base);
  e = hipGetLastError();
  const sc::WsView w{ws, tw};
  if (e == hipSuccess) e = sc::enqueue_kernels_ws(m, base, 1, total, hs, 0, w);
  if (e != hipSuccess) {
    s->bad = true;
    return sc::fail_status(SC_EDEVICE, (std::string("kernel launch: ") + hipGetErrorString(e)).c_str());
  }
  sc::commit_step(1, &s, &n_frames);
  return SC_OK;
}
