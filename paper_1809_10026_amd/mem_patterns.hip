// Memory-pattern reference: the global-memory access patterns of the hot
// kernels of the space-time solve, without their arithmetic, at the shape of
// the d = 3, p = 4, 48-elements-per-direction workload (n1 = n2 = n3 = 50
// unknowns in space, nt = 51 in time).  Each pattern moves the bytes of its
// kernel in that kernel's order and is timed with HIP events, median of ten
// launches, in two states of the memory-side cache:
//   warm: the same buffers as the previous launch (they fit in the cache),
//   cold: after a 2 GiB write to another buffer (the cache then holds dirty
//         lines of that buffer that must be written back first).
// The figures bound what the kernels can reach with their access order.
//
//   python paper_1809_10026_amd/build.py && ./paper_1809_10026_amd/mem_patterns
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                                  \
  do {                                                                                            \
    hipError_t e_ = (x);                                                                          \
    if (e_ != hipSuccess) {                                                                       \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);         \
      std::exit(1);                                                                               \
    }                                                                                             \
  } while (0)

// read x, write A, B, C in one grid-stride sweep (the matvec inner stage's
// bytes in the ideal order)
__global__ __launch_bounds__(256) void contig_1to3(const double* __restrict__ x, double* __restrict__ A,
                                                   double* __restrict__ B, double* __restrict__ C, long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const double v = x[i];
    A[i] = v;
    B[i] = v + 1.0;
    C[i] = v + 2.0;
  }
}

// the same bytes, one whole (i3, t) slab of n1 n2 values per workgroup (the
// inner stage's order)
__global__ __launch_bounds__(512) void slab_1to3(const double* __restrict__ x, double* __restrict__ A,
                                                 double* __restrict__ B, double* __restrict__ C, int ns, int nslab) {
  for (int s = blockIdx.x; s < nslab; s += gridDim.x) {
    const size_t b = (size_t)s * ns;
    for (int e = threadIdx.x; e < ns; e += 512) {
      const double v = x[b + e];
      A[b + e] = v;
      B[b + e] = v + 1.0;
      C[b + e] = v + 2.0;
    }
  }
}

// read A, B, C, P, write y: each thread one (row, l) of a tile of LB
// consecutive l times 256 / LB rows, walking the time slices (the outer
// stage's order; LB = 16 is its tile width, LB * 8 bytes its row segment)
template <int LB>
__global__ __launch_bounds__(256) void outer_4to1(const double* __restrict__ A, const double* __restrict__ B,
                                                  const double* __restrict__ C, const double* __restrict__ P,
                                                  double* __restrict__ y, int L, int nd, int nt) {
  constexpr int RW = 256 / LB;
  const int ntd = (nd + RW - 1) / RW;
  const int lb = blockIdx.x / ntd, td = blockIdx.x % ntd;
  const int l = lb * LB + (int)(threadIdx.x % LB), row = td * RW + (int)(threadIdx.x / LB);
  if (l >= L || row >= nd) return;
  const size_t plane = (size_t)L * nd;
  for (int t = 0; t < nt; ++t) {
    const size_t g = (size_t)t * plane + (size_t)row * L + l;
    y[g] = A[g] + B[g] + C[g] + P[g];
  }
}

__global__ __launch_bounds__(256) void contig_4to1(const double* __restrict__ A, const double* __restrict__ B,
                                                   const double* __restrict__ C, const double* __restrict__ P,
                                                   double* __restrict__ y, long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) y[i] = A[i] + B[i] + C[i] + P[i];
}

// FP32 copy in the order of the strided FD passes: a wave takes 16
// consecutive columns c of the (L, n, R) view and walks the n rows (64-byte
// segments at stride L), the 8 waves of a workgroup take adjacent units
__global__ __launch_bounds__(512) void strided_copy(const float* __restrict__ X, float* __restrict__ Y, int L, int n,
                                                    int ncols) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nunits = (ncols + 15) / 16;
  for (int u = blockIdx.x * 8 + wave; u < nunits; u += gridDim.x * 8) {
    const int c = u * 16 + (lane & 15);
    if (c >= ncols) continue;
    const size_t base = (size_t)(c % L) + (size_t)(c / L) * L * n;
    for (int k = lane >> 4; k < n; k += 4) Y[base + (size_t)k * L] = X[base + (size_t)k * L];
  }
}

__global__ __launch_bounds__(256) void contig_copy_f32(const float* __restrict__ X, float* __restrict__ Y, long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) Y[i] = X[i];
}

int main() {
  const int n1 = 50, n2 = 50, n3 = 50, nt = 51;
  const int ns = n1 * n2, nslab = n3 * nt;
  const long N = (long)ns * nslab;
  const long NF = 1L << 28;  // 2 GiB of doubles
  double *x, *A, *B, *C, *P, *y, *flush;
  CHECK(hipMalloc(&x, N * 8));
  CHECK(hipMalloc(&A, N * 8));
  CHECK(hipMalloc(&B, N * 8));
  CHECK(hipMalloc(&C, N * 8));
  CHECK(hipMalloc(&P, N * 8));
  CHECK(hipMalloc(&y, N * 8));
  CHECK(hipMalloc(&flush, NF * 8));
  for (double* b : {x, A, B, C, P, y}) CHECK(hipMemset(b, 0, N * 8));
  float* xf = reinterpret_cast<float*>(x);
  float* yf = reinterpret_cast<float*>(y);
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  std::printf("%-52s %-5s %9s %9s\n", "pattern (bytes of the kernel it stands for)", "state", "us", "TB/s");
  auto run = [&](const char* name, double bytes, bool cold, auto launch) {
    std::vector<float> ts;
    for (int rep = 0; rep < 12; ++rep) {
      if (cold) CHECK(hipMemsetAsync(flush, rep & 1, NF * 8, 0));
      CHECK(hipEventRecord(e0, 0));
      launch();
      CHECK(hipGetLastError());
      CHECK(hipEventRecord(e1, 0));
      CHECK(hipEventSynchronize(e1));
      float ms;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (rep >= 2) ts.push_back(ms);
    }
    std::sort(ts.begin(), ts.end());
    const float ms = ts[ts.size() / 2];
    std::printf("%-52s %-5s %9.1f %9.2f\n", name, cold ? "cold" : "warm", ms * 1e3, bytes / (ms * 1e-3) / 1e12);
    std::fflush(stdout);
  };
  const double b4 = 4.0 * N * 8, b5 = 5.0 * N * 8, bf = 2.0 * N * 4;
  const int ntd16 = (n3 + 15) / 16, ntd64 = (n3 + 3) / 4, ntd256 = n3;
  for (int cold = 0; cold < 2; ++cold) {
    run("contiguous, read 1 write 3 (inner stage)", b4, cold,
        [&] { hipLaunchKernelGGL(contig_1to3, dim3(8192), dim3(256), 0, 0, x, A, B, C, N); });
    run("one slab per workgroup, read 1 write 3", b4, cold,
        [&] { hipLaunchKernelGGL(slab_1to3, dim3(512), dim3(512), 0, 0, x, A, B, C, ns, nslab); });
    run("contiguous, read 4 write 1 (outer stage)", b5, cold,
        [&] { hipLaunchKernelGGL(contig_4to1, dim3(8192), dim3(256), 0, 0, A, B, C, P, y, N); });
    run("16-wide l tiles over t, read 4 write 1 (128 B rows)", b5, cold, [&] {
      hipLaunchKernelGGL(outer_4to1<16>, dim3(((ns + 15) / 16) * ntd16), dim3(256), 0, 0, A, B, C, P, y, ns, n3, nt);
    });
    run("64-wide l tiles over t, read 4 write 1 (512 B rows)", b5, cold, [&] {
      hipLaunchKernelGGL(outer_4to1<64>, dim3(((ns + 63) / 64) * ntd64), dim3(256), 0, 0, A, B, C, P, y, ns, n3, nt);
    });
    run("256-wide l tiles over t, read 4 write 1 (2 KB rows)", b5, cold, [&] {
      hipLaunchKernelGGL(outer_4to1<256>, dim3(((ns + 255) / 256) * ntd256), dim3(256), 0, 0, A, B, C, P, y, ns, n3,
                         nt);
    });
    run("FP32 copy, contiguous (one FD pass's bytes)", bf, cold,
        [&] { hipLaunchKernelGGL(contig_copy_f32, dim3(8192), dim3(256), 0, 0, xf, yf, N); });
    run("FP32 copy, 16-column units along mode 3 (64 B rows)", bf, cold, [&] {
      hipLaunchKernelGGL(strided_copy, dim3(2048), dim3(512), 0, 0, xf, yf, ns, n3, (int)(N / n3));
    });
    run("FP32 copy, 16-column units along time (64 B rows)", bf, cold, [&] {
      hipLaunchKernelGGL(strided_copy, dim3(2048), dim3(512), 0, 0, xf, yf, ns * n3, nt, (int)(N / nt));
    });
  }
  CHECK(hipDeviceSynchronize());
  std::printf("done\n");
  return 0;
}
