// cones.hip - texture-coordinate gradients of a hit from its ray cone.
//
// Sec. 3.1: a ray cone meets the surface in an ellipse; its two axes carried
// into texture space are the gradients g1 and g2 from which Eq. 1 takes the
// virtual mip level (after Akenine-Moller et al. 2021, ray cones).  Per hit:
// the cone of radius r around the ray meets the triangle's plane in an
// ellipse with semi-axes r / |cos| along the ray's projection onto the plane
// and r across it (|cos| clamped below at 1/1024); a ray within 1e-4 rad of
// the normal takes the tangent frame of Duff et al. 2017 instead of the
// undefined projection.  An in-plane offset a moves the barycentric
// coordinates by ((a x e2).n, (e1 x a).n) / (n.n), n = e1 x e2, hence the UV by
// that combination of the triangle's UV edges.  Degenerate or non-finite
// inputs give NaN gradients (the hit then bypasses the cache).
//
// One thread per hit, a grid-stride loop; 56 bytes in, 16 out per hit.
#include "context.h"

namespace pmc {
namespace {

struct ConeArgs {
  const float* dir;
  const float* radius;
  const float2* edge;        // [n][3] float2 = e1.xyz, e2.xyz
  const float4* uv_edge;     // [n] = t1.xy, t2.xy
  float4* duv;               // [n] = g1.xy, g2.xy
  uint64_t n;
};

constexpr float kMinCos = 1.0f / 1024.0f;
constexpr float kHeadOn = 1e-4f;

struct V3 {
  float x, y, z;
};

__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 mul(V3 a, float s) { return v3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ V3 divs(V3 a, float s) { return v3(a.x / s, a.y / s, a.z / s); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// UV change of the in-plane world offset a on the triangle (e1, e2; n = e1 x e2).
__device__ __forceinline__ float2 uv_of_offset(V3 a, V3 e1, V3 e2, V3 n, float nn, float4 t) {
  const float du = dot(cross(a, e2), n) / nn;
  const float dv = dot(cross(e1, a), n) / nn;
  return make_float2(du * t.x + dv * t.z, du * t.y + dv * t.w);
}

__global__ __launch_bounds__(256) void k_ray_cone(ConeArgs a) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    const V3 d = v3(a.dir[3 * i], a.dir[3 * i + 1], a.dir[3 * i + 2]);
    const float r = a.radius[i];
    const float2 p0 = a.edge[3 * i], p1 = a.edge[3 * i + 1], p2 = a.edge[3 * i + 2];
    const V3 e1 = v3(p0.x, p0.y, p1.x), e2 = v3(p1.y, p2.x, p2.y);
    const float4 t = a.uv_edge[i];
    // the normal in binary64: the products of binary32 edges are exact there, so
    // an exactly degenerate triangle gives exactly n = 0 (in binary32 a fused
    // multiply-add leaves a rounding residue)
    const double nx = (double)e1.y * e2.z - (double)e1.z * e2.y;
    const double ny = (double)e1.z * e2.x - (double)e1.x * e2.z;
    const double nz = (double)e1.x * e2.y - (double)e1.y * e2.x;
    const double nnd = nx * nx + ny * ny + nz * nz;
    const V3 n = v3((float)nx, (float)ny, (float)nz);
    const float nn = (float)nnd;
    const float dl = sqrtf(dot(d, d));
    const float nl = sqrtf(nn);
    const V3 m = divs(n, nl);
    const V3 dh = divs(d, dl);
    const float c = dot(dh, m);
    const V3 h = sub(dh, mul(m, c));
    const float hl = sqrtf(dot(h, h));
    const bool head_on = hl < kHeadOn;
    V3 a1, a2;
    if (head_on) {
      // tangent frame of m (Duff et al. 2017), sign = +1 when m.z >= 0
      const float sg = m.z >= 0.0f ? 1.0f : -1.0f;
      const float q = -1.0f / (sg + m.z);
      const float b = m.x * m.y * q;
      a1 = mul(v3(1.0f + sg * m.x * m.x * q, sg * b, -sg * m.x), r);
      a2 = mul(v3(b, sg + m.y * m.y * q, -m.y), r);
    } else {
      const V3 t1 = divs(h, hl);
      const float ac = fmaxf(fabsf(c), kMinCos);
      a1 = mul(t1, r / ac);
      a2 = mul(cross(m, t1), r);
    }
    const float2 g1 = uv_of_offset(a1, e1, e2, n, nn, t);
    const float2 g2 = uv_of_offset(a2, e1, e2, n, nn, t);
    const bool ok = nnd > 0.0 && nn > 0.0f && dl > 0.0f && isfinite(nn) && isfinite(dl) &&
                    isfinite(r) &&
                    isfinite(g1.x) && isfinite(g1.y) && isfinite(g2.x) && isfinite(g2.y) &&
                    isfinite(t.x) && isfinite(t.y) && isfinite(t.z) && isfinite(t.w);
    const float nan = __int_as_float(0x7FC00000);
    a.duv[i] = ok ? make_float4(g1.x, g1.y, g2.x, g2.y) : make_float4(nan, nan, nan, nan);
  }
}

}  // namespace
}  // namespace pmc

using namespace pmc;

extern "C" pmc_status pmc_ray_cone_gradients(pmc_ctx* ctx, const pmc_cone_hits* hits, float* duv,
                                             void* stream) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = need_device(ctx)) return st;
  if (!hits) return ctx->fail(PMC_ERR_INVALID, "null cone hits");
  if (hits->n == 0) return PMC_OK;
  if (!hits->dir || !hits->radius || !hits->edge || !hits->uv_edge || !duv)
    return ctx->fail(PMC_ERR_INVALID, "null cone array");
  if (((uintptr_t)hits->edge & 7u) || ((uintptr_t)hits->uv_edge & 15u) || ((uintptr_t)duv & 15u))
    return ctx->fail(PMC_ERR_INVALID, "edge must be 8-byte, uv_edge and duv 16-byte aligned");
  if (hits->n >= (1ull << 40)) return ctx->fail(PMC_ERR_INVALID, "too many cone hits");
  ConeArgs a;
  a.dir = hits->dir;
  a.radius = hits->radius;
  a.edge = reinterpret_cast<const float2*>(hits->edge);
  a.uv_edge = reinterpret_cast<const float4*>(hits->uv_edge);
  a.duv = reinterpret_cast<float4*>(duv);
  a.n = hits->n;
  const uint64_t blocks = (hits->n + 255) / 256;
  const uint32_t grid = (uint32_t)(blocks < (uint64_t)ctx->num_cus * 16 ? blocks
                                                                         : (uint64_t)ctx->num_cus * 16);
  hipLaunchKernelGGL(k_ray_cone, dim3(grid), dim3(256), 0, (hipStream_t)stream, a);
  HIP_TRY(ctx, hipGetLastError());
  return PMC_OK;
}
