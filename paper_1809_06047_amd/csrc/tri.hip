// Loop (App. B) and sqrt(3) (App. A) level steps on gfx950. Both use the
// adjacency of the same level from the generic build: twin half-edges give
// G(i,j)/G(j,i) (the opposite vertices, Loop) and F(l,k) (the neighbouring
// face, sqrt(3)); edge ids come from the upper triangle of E.
//
// Loop:   edge point 3/8 (p_a + p_b) + 1/8 (p_c + p_d), boundary midpoint;
//         vertex (1 - n beta_n) p + beta_n sum p_j (eq:loop_smooth), boundary
//         3/4 p + 1/8 (p_prev + p_next); children 4r+j (j<3) =
//         (v_j, e(j,j+1), e(j-1,j)), 4r+3 = (e01, e12, e20).
// sqrt3:  face point mapped M^T P with (1,2,3) -> 1/3; vertex
//         (1 - alpha_n) p + alpha_n / n sum p_j (equ:sqrt2, equ:alpha), boundary
//         vertices fixed; child 3r+j = (v_j, face across edge j, face r) or
//         (v_j, v_j+1, face r) on a boundary edge (the face point of face i has
//         index |v| + i).
// beta_n and alpha_n are evaluated once on the host in FP64 and rounded to
// FP32 into constant memory: no device cosine decides a weight.
#include <cmath>
#include <mutex>

#include "subdiv_internal.h"

namespace subdiv {

__constant__ float c_loop_beta[SUBDIV_MAX_VALENCE + 1];
__constant__ float c_sqrt3_alpha[SUBDIV_MAX_VALENCE + 1];

hipError_t init_weight_tables() {
  static std::mutex mu;
  static int done_device = -1;
  std::lock_guard<std::mutex> lock(mu);
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  if (done_device == dev) return hipSuccess;
  static float beta[SUBDIV_MAX_VALENCE + 1], alpha[SUBDIV_MAX_VALENCE + 1];
  const double pi = 3.14159265358979323846;
  beta[0] = alpha[0] = 0.f;
  for (int n = 1; n <= SUBDIV_MAX_VALENCE; ++n) {
    const double c = 3.0 / 8.0 + 0.25 * std::cos(2.0 * pi / n);
    beta[n] = (float)((5.0 / 8.0 - c * c) / n);
    alpha[n] = (float)((4.0 - 2.0 * std::cos(2.0 * pi / n)) / 9.0);
  }
  if ((err = hipMemcpyToSymbol(HIP_SYMBOL(c_loop_beta), beta, sizeof(beta))) != hipSuccess) return err;
  if ((err = hipMemcpyToSymbol(HIP_SYMBOL(c_sqrt3_alpha), alpha, sizeof(alpha))) != hipSuccess) return err;
  done_device = dev;
  return hipSuccess;
}

// ring walk around v: sum of the neighbours, count of faces, boundary ends
struct Ring {
  f3 sum;
  int faces;
  int w0;  // end of the first half-edge (boundary neighbour if on the boundary)
  int ub;  // start of the last incoming boundary half-edge, -1 if interior
};

__device__ __forceinline__ Ring ring3(const Topo &t, const Adj &a, const float *P, int v) {
  const int h0 = a.vhe[v];
  Ring R{{0.f, 0.f, 0.f}, 0, t.fv[he_next<3>(t, h0)], -1};
  int h = h0;
  while (true) {
    R.sum = add3(R.sum, ld3(P, t.fv[he_next<3>(t, h)]));
    ++R.faces;
    const int hp = he_prev<3>(t, h);
    const int tw = a.twin[hp];
    if (tw < 0) {
      R.ub = t.fv[hp];
      R.sum = add3(R.sum, ld3(P, R.ub));
      break;
    }
    if (tw == h0 || R.faces >= SUBDIV_MAX_VALENCE) break;
    h = tw;
  }
  return R;
}

// ------------------------------------------------------------------ Loop
__global__ void __launch_bounds__(kBlock) k_loop_edge(TriStep c) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= c.a.E) return;
  const int h = c.a.e2h[e];
  const f3 pab = add3(ld3(c.P, c.t.fv[h]), ld3(c.P, c.t.fv[he_next<3>(c.t, h)]));
  const int t = c.a.twin[h];
  f3 ep;
  if (t < 0) ep = mul3(0.5f, pab);
  else {
    const f3 pcd = add3(ld3(c.P, c.t.fv[he_prev<3>(c.t, h)]), ld3(c.P, c.t.fv[he_prev<3>(c.t, t)]));
    ep = fma3(0.375f, pab, mul3(0.125f, pcd));
  }
  st3(c.P1, c.t.V + e, ep);
}

__global__ void __launch_bounds__(kBlock) k_loop_vertex(TriStep c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.t.V) return;
  const f3 p = ld3(c.P, v);
  const Ring R = ring3(c.t, c.a, c.P, v);
  f3 S;
  if (R.ub >= 0) {
    S = fma3(0.75f, p, mul3(0.125f, add3(ld3(c.P, R.w0), ld3(c.P, R.ub))));
  } else {
    const int n = R.faces;
    const float beta = c_loop_beta[n];
    S = fma3(1.0f - (float)n * beta, p, mul3(beta, R.sum));
  }
  st3(c.P1, v, S);
}

__global__ void __launch_bounds__(kBlock) k_loop_face(TriStep c) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= c.t.F) return;
  const int V = c.t.V;
  const int v0 = c.t.fv[3 * r], v1 = c.t.fv[3 * r + 1], v2 = c.t.fv[3 * r + 2];
  const int e0 = V + c.a.eid[3 * r], e1 = V + c.a.eid[3 * r + 1], e2 = V + c.a.eid[3 * r + 2];
  int4 *o = reinterpret_cast<int4 *>(c.fv1 + 12ll * r);
  o[0] = make_int4(v0, e0, e2, v1);
  o[1] = make_int4(e1, e0, v2, e2);
  o[2] = make_int4(e1, e0, e1, e2);
}

// ------------------------------------------------------------------ sqrt(3)
__global__ void __launch_bounds__(kBlock) k_sqrt3_face(TriStep c) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= c.t.F) return;
  const int V = c.t.V;
  int v[3], tw[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    v[j] = c.t.fv[3 * r + j];
    tw[j] = c.a.twin[3 * r + j];
  }
  const f3 sum = add3(add3(ld3(c.P, v[0]), ld3(c.P, v[1])), ld3(c.P, v[2]));
  st3(c.P1, V + r, mul3(1.0f / 3.0f, sum));
  int *o = c.fv1 + 9ll * r;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    o[3 * j + 0] = v[j];
    o[3 * j + 1] = tw[j] < 0 ? v[(j + 1) % 3] : V + tw[j] / 3;
    o[3 * j + 2] = V + r;
  }
}

__global__ void __launch_bounds__(kBlock) k_sqrt3_vertex(TriStep c) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.t.V) return;
  const f3 p = ld3(c.P, v);
  const Ring R = ring3(c.t, c.a, c.P, v);
  f3 S;
  if (R.ub >= 0) {
    S = p;
  } else {
    const int n = R.faces;
    const float alpha = c_sqrt3_alpha[n];
    S = fma3(1.0f - alpha, p, mul3(alpha / (float)n, R.sum));
  }
  st3(c.P1, v, S);
}

hipError_t tri_launch(int which, const TriStep &c, hipStream_t s) {
  switch (which) {
    case LOOP_EDGE:
      hipLaunchKernelGGL(k_loop_edge, dim3(grid_for(c.a.E)), dim3(kBlock), 0, s, c);
      break;
    case LOOP_VERTEX:
      hipLaunchKernelGGL(k_loop_vertex, dim3(grid_for(c.t.V)), dim3(kBlock), 0, s, c);
      break;
    case LOOP_FACE:
      hipLaunchKernelGGL(k_loop_face, dim3(grid_for(c.t.F)), dim3(kBlock), 0, s, c);
      break;
    case SQRT3_FACE:
      hipLaunchKernelGGL(k_sqrt3_face, dim3(grid_for(c.t.F)), dim3(kBlock), 0, s, c);
      break;
    default:
      hipLaunchKernelGGL(k_sqrt3_vertex, dim3(grid_for(c.t.V)), dim3(kBlock), 0, s, c);
      break;
  }
  return hipGetLastError();
}

}  // namespace subdiv
