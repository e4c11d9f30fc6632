// Seeded synthetic inputs generated in device memory.
//
// Same definition as workload/philox.py: Philox4x32-10 (Salmon et al., SC'11)
// on the counter (index_lo, index_hi, stream, field) with key (seed_lo,
// salt ^ seed_hi); an Irwin-Hall(4) unit normal
//   z = (double(u0 + u1 + u2 + u3 - 2^33) * 2^-32) * sqrt(3)
// times the segment scale.  Floating-point contraction is off so every value
// is bit-identical to the host generator.  Holds no arithmetic of the method.
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace {

struct Seg {          // matches workload.problem.SEG_DTYPE (48 bytes)
  int64_t off;
  int64_t stream;
  int32_t field, mode, layers, rows, cols, pad;
  double scale;
};

constexpr uint32_t kSalt = 0x5EED0DF1u;

__device__ __forceinline__ void philox(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                       uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    if (r < 9) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
  }
}

__device__ __forceinline__ double normal(uint64_t idx, uint64_t stream, uint32_t field, uint64_t seed) {
  uint32_t c0 = (uint32_t)idx, c1 = (uint32_t)(idx >> 32), c2 = (uint32_t)stream, c3 = field;
  philox(c0, c1, c2, c3, (uint32_t)seed, kSalt ^ (uint32_t)(seed >> 32));
  const int64_t s = (int64_t)((uint64_t)c0 + c1 + c2 + c3) - (int64_t(1) << 33);
  const double x = (double)s * 0x1p-32;
  return x * 0x1.bb67ae8584caap+0;   // sqrt(3) rounded to double
}

__device__ __forceinline__ double uniform(uint64_t idx, uint64_t stream, uint32_t field, uint64_t seed) {
  uint32_t c0 = (uint32_t)idx, c1 = (uint32_t)(idx >> 32), c2 = (uint32_t)stream, c3 = field;
  philox(c0, c1, c2, c3, (uint32_t)seed, kSalt ^ (uint32_t)(seed >> 32));
  return (double)c0 * 0x1p-32;
}

__global__ __launch_bounds__(256) void gen_kernel(const Seg* segs, int64_t nseg, uint64_t seed, double* out) {
  for (int64_t si = blockIdx.x; si < nseg; si += gridDim.x) {
    const Seg sg = segs[si];
    const int64_t per = (int64_t)sg.rows * sg.cols;
    const int64_t total = per * sg.layers;
    for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
      const int64_t L = e / per;
      const int rem = (int)(e - L * per);
      const int x = rem / sg.cols, y = rem - x * sg.cols;
      const uint64_t lay = (uint64_t)L * 4096u;
      double v;
      switch (sg.mode) {
        case 0: v = normal(lay + (uint64_t)x * 64u + y, sg.stream, sg.field, seed) * sg.scale; break;
        case 3: v = normal(lay + (uint64_t)y * 64u + x, sg.stream, sg.field, seed) * sg.scale; break;
        case 4: v = x == y ? 1.0 : 0.0; break;   // identity block
        case 5: {   // staircase decay 2^-floor((x + y) / pad)
          const double z = normal(lay + (uint64_t)x * 64u + y, sg.stream, sg.field, seed);
          v = z * ldexp(1.0, -((x + y) / sg.pad)) * sg.scale;
          break;
        }
        case 7:
        case 8: {   // overlap of SOMO-augmented PNO sets: identity on the last pad rows/columns
          const int xs = x - (sg.rows - sg.pad), ys = y - (sg.cols - sg.pad);
          if (xs < 0 && ys < 0) {
            const uint64_t idx = sg.mode == 7 ? lay + (uint64_t)x * 64u + y : lay + (uint64_t)y * 64u + x;
            v = normal(idx, sg.stream, sg.field, seed) * sg.scale;
          } else {
            v = (xs >= 0 && xs == ys) ? 1.0 : 0.0;
          }
          break;
        }
        case 6: {   // symmetric Fock-like block: 0.2 + 2.8 u on the diagonal
          const int lo = x < y ? x : y, hi = x < y ? y : x;
          const uint64_t idx = lay + (uint64_t)lo * 64u + hi;
          v = x == y ? 0.2 + 2.8 * uniform(idx, sg.stream, sg.field, seed)
                     : normal(idx, sg.stream, sg.field, seed) * sg.scale;
          break;
        }
        case 1: {
          const int lo = x < y ? x : y, hi = x < y ? y : x;
          v = normal(lay + (uint64_t)lo * 64u + hi, sg.stream, sg.field, seed) * sg.scale;
          break;
        }
        default: {
          const double z1 = normal(lay + (uint64_t)x * 64u + y, sg.stream, sg.field, seed);
          const double z2 = normal(lay + (uint64_t)y * 64u + x, sg.stream, sg.field, seed);
          v = (z1 - z2) * sg.scale;
          break;
        }
      }
      out[sg.off + e] = v;
    }
  }
}

}  // namespace

// Fill `out` (device, float64) with the given segments (device array of nseg
// descriptors).  Returns a hipError_t code.
extern "C" int dlpno_gen_segments(const void* segs_dev, int64_t nseg, uint64_t seed, double* out, void* stream) {
  if (nseg <= 0) return 0;
  const int64_t grid = nseg < 65536 ? nseg : 65536;
  hipLaunchKernelGGL(gen_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                     (const Seg*)segs_dev, nseg, seed, out);
  return (int)hipGetLastError();
}
