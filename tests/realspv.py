"""Real SPIR-V modules for the tests: HIP kernels compiled here by hipcc for
the generic SPIR-V target (--offload-arch=amdgcnspirv); the SPIR-V image is
taken out of the offload bundle with clang-offload-bundler.  Built once per
process into a temporary directory; available() says whether the tools are
there."""
import functools
import os
import subprocess
import tempfile

import numpy as np

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
BUNDLER = "/opt/rocm/lib/llvm/bin/clang-offload-bundler"

SOURCES = {
    "add": r"""
#include <hip/hip_runtime.h>
__global__ void add(int* a, const int* b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] += b[i];
}
""",
    "mix": r"""
#include <hip/hip_runtime.h>
struct P { float x, y; int k; };
__device__ float f(float v, int k) { for (int j = 0; j < k; ++j) v = v * 1.5f + (float)j; return v; }
__global__ void mix(P* p, float* out, int* hist, int n, int m) {
  __shared__ float s[256];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  float acc = 0.f;
  for (int j = i; j < n; j += gridDim.x * blockDim.x) {
    P q = p[j];
    acc += f(q.x, q.k & 7) - q.y;
    atomicAdd(&hist[(q.k % m + m) % m], 1);
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int d = blockDim.x / 2; d > 0; d >>= 1) {
    if (threadIdx.x < d) s[threadIdx.x] += s[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}
__global__ void scale(double* v, double a, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = v[i] * a + (double)(i % 3);
}
""",
}


def available() -> bool:
    return os.path.exists(HIPCC) and os.path.exists(BUNDLER)


@functools.lru_cache(maxsize=None)
def module(name: str) -> np.ndarray:
    """uint32 words of the SPIR-V module built from SOURCES[name]."""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, name + ".hip")
        bundle = os.path.join(d, name + ".o")
        spv = os.path.join(d, name + ".spv")
        with open(src, "w") as f:
            f.write(SOURCES[name])
        subprocess.run([HIPCC, "--offload-arch=amdgcnspirv", "-c", "--offload-device-only", src, "-o", bundle],
                       check=True, capture_output=True, timeout=300)
        targets = subprocess.run([BUNDLER, "--list", "--type=o", "--input=" + bundle], check=True,
                                 capture_output=True, text=True, timeout=60).stdout.split()
        target = next(t for t in targets if "spirv" in t)
        subprocess.run([BUNDLER, "--unbundle", "--type=o", "--targets=" + target, "--input=" + bundle,
                        "--output=" + spv], check=True, capture_output=True, timeout=60)
        return np.fromfile(spv, dtype=np.uint32)
