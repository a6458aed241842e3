// Device-side building blocks of the gfx950 GPSS path tracer: scene record, counter-based
// random numbers, GP statistics at a point, the macrofacet medium (density, projected
// area, generalized NDF, phase function and its mixture proposal) and majorant-grid
// traversal.  Single precision; every function is inlined into the kernels that use it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpss {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvSqrt2 = 0.70710678118654752440f;
constexpr float kInvSqrt2Pi = 0.39894228040143267794f;     // 1 / sqrt(2 pi)
constexpr float kSqrt2Pi = 2.50662827463100050242f;
constexpr float kSqrtHalfPi = 1.25331413731550025121f;     // sqrt(pi / 2)
constexpr float kSqrt2OverPi = 0.79788456080286535588f;    // sqrt(2 / pi)
constexpr float kInvSqrtPi = 0.56418958354775628695f;
constexpr float kInv2PiPow1p5 = 0.06349363593424096978f;   // (2 pi)^(-3/2)
constexpr float kSqrt2 = 1.41421356237309504880f;

constexpr int kMaxPrims = 64;
constexpr int kMaxObs = 32;                 // observations of a conditioned GP (a multiple of 4)
// Stored lower triangle of L^-1: row i zero-padded to cond_row_blocks(i) blocks of four
// entries, each block one 64-byte scalar load against four k_j of one LDS read.
constexpr int cond_row_blocks(int i) { return (i >> 2) + 1; }
constexpr int cond_tri_entries(int n) {
    int t = 0;
    for (int i = 0; i < n; ++i) t += 4 * cond_row_blocks(i);
    return t;
}
constexpr int kCondTriEntries = cond_tri_entries(kMaxObs);
static_assert(kMaxObs % 4 == 0, "observations are processed four at a time");

// Scheduling policy of the persistent tracer for one scene: cell steps per walk operation and
// the lanes a scatter operation waits for.  Rough media (typical gradient spread
// s = sigma / l of at least sqrt(2), roughness alpha >= 2) scatter at most tentative
// collisions and run faster with short walks and fuller scatter operations (4, 24); smooth
// ones with longer walks (6, 16).  Measured on the sphere and mixed workloads; the choice
// reorders work across lanes only, never within a path, so images do not depend on it.
struct SchedPolicy {
    int walk_steps, scatter_min;
};
inline SchedPolicy sched_policy(float s_typical) {
    return s_typical >= 1.41421356f ? SchedPolicy{4, 24} : SchedPolicy{6, 16};
}
constexpr int kStepCap = 1 << 16;           // tentative collisions per segment
constexpr float kRRThreshold = 0.0625f;     // shadow-ray Russian roulette below this transmittance

enum : uint32_t { kStreamCam = 0, kStreamTrack = 1, kStreamPhase = 2, kStreamNee0 = 3 };

// ---------------------------------------------------------------------------
// Scene record, passed by value as a kernel argument.
// ---------------------------------------------------------------------------
struct SceneDev {
    int mean_kind;
    float mean_const;
    int n_prims;
    const float4* prims;          // 2 per primitive: (kind, cx, cy, cz), (a, b, c, albedo)
    const float* offset;          // nullable
    int off_res[3];
    float off_scale[3];           // (res - 1) / extent
    float variance;
    const float* var_grid;        // nullable
    int var_res[3];
    float var_scale[3];
    float lengthscale;
    float sigma0, s0;             // sqrt(variance) and sqrt(variance) / lengthscale (scalar variance)
    float inv_l;                  // 1 / lengthscale (gradient terms)
    int walk_steps, scatter_min;  // scheduling of the persistent tracer (sched_policy)
    float aniso_k;                // (l / l_n)^2 - 1 for lengthscale l_n along the mean gradient; 0: isotropic
    int ggx;                      // GGX height-field macrofacet instead of the generalized one
    float f_eta, f_k;             // conductor IOR eta + i k of the Fresnel term (eta = 0: F = albedo)
    int n_obs;                    // observations conditioning the GP (0: unconditioned)
    const float4* obs;            // per observation: position relative to obs_c, weight alpha
    const float4* obs_tri;        // lower triangle of L^-1 (L L^T = kappa(C,C) + noise I), row by row:
                                  // (L^-1_ij, L^-1_ij x_j) for j <= i, positions relative to obs_c,
                                  // each row zero-padded to 4 cond_row_blocks(i) entries
    float obs_c[3];               // origin of the observation positions
    float albedo;
    int albedo_per_prim;
    float lo[3], hi[3];
    float cw[3];                  // majorant cell size
    float inv_cw[3];
    double lo_d[3], hi_d[3], cw_d[3], inv_cw_d[3];  // the same box and cells in double
    double off_scale_d[3], var_scale_d[3];          // the grid scales in double
    int M[3];
    const uint16_t* maj16;        // majorant grid, x fastest, as the top 16 bits of each float: the
                                  // majorants have five significant bits, so this is exact
    const uint16_t* prim_cand;    // per majorant cell: the primitives that can be the union's minimum
                                  // there (count 1-3 in bits 0-1, 4-bit indices above in increasing
                                  // order; count 0: all); null: every cell takes all
    float R;
    float dl[4], pl[4], env;
    int cam_kind;
    double eye[3], fwd[3], right[3], upc[3];
    double tan_half, aspect, win[2];
    int W, H, max_depth;
    uint32_t key0, key1;
};

// Load from a scene array through the global address space.  The arrays are reached through
// pointers held in the scene record, whose address space the compiler cannot infer; plain
// loads would be flat loads, which also count on the LDS counter and so delay every LDS wait
// of the scheduled loop behind a memory access.
__device__ __forceinline__ float ld_global(const float* p) {
    return *(const __attribute__((address_space(1))) float*)p;
}
__device__ __forceinline__ uint32_t ld_global(const uint16_t* p) {
    return *(const __attribute__((address_space(1))) uint16_t*)p;
}
__device__ __forceinline__ float4 ld_global(const float4* p) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 v = *(const __attribute__((address_space(1))) v4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
// The same for arrays that no kernel writes while it reads them (primitives, observations):
// through the constant address space, a load whose address is the same for the whole wave
// becomes one scalar load.
__device__ __forceinline__ float4 ld_const(const float4* p) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 v = *(const __attribute__((address_space(4))) v4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

// ---------------------------------------------------------------------------
// float3 helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator-(float3 a) { return f3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ float3 operator*(float s, float3 a) { return f3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross(float3 a, float3 b) {
    return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float3 normalize(float3 a) { return (1.0f / sqrtf(dot(a, a))) * a; }
__device__ __forceinline__ float comp(float3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

// Ray geometry (origins, directions, distances, cell boundaries) is kept in double
// precision so that where a tentative collision falls relative to a majorant-cell
// boundary does not depend on single-precision rounding of the path's position.
struct D3 {
    double x, y, z;
};
__device__ __forceinline__ D3 d3(double x, double y, double z) { return D3{x, y, z}; }
__device__ __forceinline__ D3 d3(float3 a) { return D3{(double)a.x, (double)a.y, (double)a.z}; }
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return d3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ D3 operator-(D3 a) { return d3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ D3 operator*(double s, D3 a) { return d3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 normalize(D3 a) { return (1.0 / sqrt(dot(a, a))) * a; }
__device__ __forceinline__ float3 to_f3(D3 a) { return make_float3((float)a.x, (float)a.y, (float)a.z); }
__device__ __forceinline__ double comp(D3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

// Single roundings that the compiler may not fuse into neighbouring operations: the
// radiance and throughput accumulations use them so that the one-thread-per-path and the
// wavefront kernels (which store these values between kernels) round identically.
__device__ __forceinline__ float add_rn(float a, float b) {
#pragma clang fp contract(off)
    return a + b;
}
__device__ __forceinline__ float mul_rn(float a, float b) {
#pragma clang fp contract(off)
    return a * b;
}

// Running sum kept as an unevaluated pair hi + lo of floats: hi += v with the rounding error
// of that addition carried in lo (Knuth's two-sum), about 48 significant bits in all.
__device__ __forceinline__ void ff_add(float& hi, float& lo, float v) {
#pragma clang fp contract(off)
    const float s = hi + v;
    const float bb = s - hi;
    const float err = (hi - (s - bb)) + (v - bb);
    hi = s;
    lo += err;
}

// Orthonormal basis around unit n (Duff et al., JCGT 2017).
__device__ __forceinline__ void onb(float3 n, float3& t, float3& b) {
    const float sign = copysignf(1.0f, n.z);
    const float a = -1.0f / (sign + n.z);
    const float bb = n.x * n.y * a;
    t = f3(1.0f + sign * n.x * n.x * a, sign * bb, -sign * n.x);
    b = f3(bb, sign + n.y * n.y * a, -n.y);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds, each two 32x32 -> 64-bit products,
// key bumped by the Weyl constants between rounds.  Each product is one 64-bit multiply
// (both halves from one v_mad_u64_u32).
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k.x, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k.y,
                       (uint32_t)p0);
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

// Draws of one (pixel, sample, bounce, stream) address, consumed in order; counter word w
// numbers blocks of four draws.  Uniforms keep the top 24 bits (exact in float).
struct Rng {
    uint4 ctr;
    uint4 buf;
    uint2 key;
    int pos;            // next draw: buf[pos]; -1: `carry`, then buf[0]
    uint32_t carry;
    __device__ __forceinline__ void init(uint32_t k0, uint32_t k1, uint32_t pixel, uint32_t sample,
                                         uint32_t bounce, uint32_t stream) {
        key = make_uint2(k0, k1);
        ctr = make_uint4(pixel, sample, (bounce & 0xFFFFu) | (stream << 16), 0u);
        pos = 4;
    }
    __device__ __forceinline__ void refill() {
        buf = philox4x32_10(ctr, key);
        ctr.w += 1u;
    }
    // Make the next two draws available without generating a block between them: a block
    // that next() would generate later is generated here, the one unread draw of the current
    // block kept ahead of it.  The sequence of draws is unchanged; callers use this to
    // generate blocks at one place per operation.
    __device__ __forceinline__ void ensure2() {
        if (pos == 3) {
            carry = buf.w;
            refill();
            pos = -1;
        } else if (pos == 4) {
            refill();
            pos = 0;
        }
    }
    __device__ __forceinline__ uint32_t next() {
        if (pos < 0) {
            pos = 0;
            return carry;
        }
        if (pos == 4) {
            refill();
            pos = 0;
        }
        const uint32_t r = pos == 0 ? buf.x : (pos == 1 ? buf.y : (pos == 2 ? buf.z : buf.w));
        ++pos;
        return r;
    }
    __device__ __forceinline__ uint32_t next24() { return next() >> 8; }
    __device__ __forceinline__ float uniform() { return (float)next24() * 0x1p-24f; }
};

// ---------------------------------------------------------------------------
// Mean-function geometry and grids.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float sdf_prim(float4 a, float4 b, float3 x, float3& g) {
    const float3 v = f3(x.x - a.y, x.y - a.z, x.z - a.w);
    if (a.x < 0.5f) {  // sphere: one reciprocal square root gives the distance and the normal
        const float d2 = dot(v, v);
        const float ir = __builtin_amdgcn_rsqf(d2);
        g = d2 > 0.0f ? ir * v : f3(0.0f, 0.0f, 1.0f);
        return d2 * ir - b.x;
    }
    const float sx = v.x < 0.0f ? -1.0f : 1.0f, sy = v.y < 0.0f ? -1.0f : 1.0f,
                sz = v.z < 0.0f ? -1.0f : 1.0f;
    const float qx = fabsf(v.x) - b.x, qy = fabsf(v.y) - b.y, qz = fabsf(v.z) - b.z;
    const float qmax = fmaxf(qx, fmaxf(qy, qz));
    if (qmax > 0.0f) {
        const float px = fmaxf(qx, 0.0f), py = fmaxf(qy, 0.0f), pz = fmaxf(qz, 0.0f);
        const float n = sqrtf(px * px + py * py + pz * pz);
        const float in = 1.0f / n;
        g = f3(sx * px * in, sy * py * in, sz * pz * in);
        return n;
    }
    int ax = 0;
    if (qy > qx) ax = 1;
    if (qz > fmaxf(qx, qy)) ax = 2;
    g = f3(ax == 0 ? sx : 0.0f, ax == 1 ? sy : 0.0f, ax == 2 ? sz : 0.0f);
    return qmax;
}

// Candidate word of the majorant cell holding x (see SceneDev::prim_cand; the scene has a
// table), or 0 (every primitive) where x lies outside the grid.  The table's bounds hold on
// each cell widened by a margin far above the rounding of this cell index, so a point on a
// cell boundary may take either neighbour.
__device__ __forceinline__ uint32_t prim_candidates(const SceneDev& S, float3 x) {
    const int ix = (int)floorf((x.x - S.lo[0]) * S.inv_cw[0]);
    const int iy = (int)floorf((x.y - S.lo[1]) * S.inv_cw[1]);
    const int iz = (int)floorf((x.z - S.lo[2]) * S.inv_cw[2]);
    if ((unsigned)ix >= (unsigned)S.M[0] || (unsigned)iy >= (unsigned)S.M[1] || (unsigned)iz >= (unsigned)S.M[2])
        return 0u;
    return ld_global(S.prim_cand + (iz * S.M[1] + iy) * S.M[0] + ix);
}

// Union of the primitives' SDFs: the smallest distance, its primitive's gradient and index
// (the lower index on ties).  Only the cell's candidates can be that primitive (nor tie with
// it), so visiting them in increasing order gives the full loop's result exactly.
__device__ __forceinline__ void mean_geom(const SceneDev& S, float3 x, float& f, float3& g, int& which) {
    which = -1;
    if (S.mean_kind == 0) { f = x.z; g = f3(0.0f, 0.0f, 1.0f); return; }
    if (S.mean_kind == 2) { f = S.mean_const; g = f3(0.0f, 0.0f, 0.0f); return; }
    float best = INFINITY;
    float3 bg = f3(0.0f, 0.0f, 1.0f);
    const uint32_t cand = S.prim_cand ? prim_candidates(S, x) : 0u;
    if (cand != 0u) {
        for (int k = 0; k < (int)(cand & 3u); ++k) {
            const int i = (int)((cand >> (2 + 4 * k)) & 15u);
            float3 gi;
            const float fi = sdf_prim(ld_const(S.prims + 2 * i), ld_const(S.prims + 2 * i + 1), x, gi);
            if (fi < best) { best = fi; bg = gi; which = i; }
        }
    } else {
        for (int i = 0; i < S.n_prims; ++i) {
            float3 gi;
            const float fi = sdf_prim(ld_const(S.prims + 2 * i), ld_const(S.prims + 2 * i + 1), x, gi);
            if (fi < best) { best = fi; bg = gi; which = i; }
        }
    }
    f = best;
    g = bg;
}

// Trilinear cell lookup on a node-centred grid over the scene box.
struct TriCell {
    int base;        // flat index of the (i, j, k) corner
    float fx, fy, fz;
};

__device__ __forceinline__ TriCell tri_cell(const int res[3], const float scale[3], const float lo[3], float3 x) {
    TriCell c;
    float u[3] = {(x.x - lo[0]) * scale[0], (x.y - lo[1]) * scale[1], (x.z - lo[2]) * scale[2]};
    int i[3];
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float ua = fminf(fmaxf(u[a], 0.0f), (float)(res[a] - 1));
        int ia = (int)floorf(ua);
        ia = min(ia, res[a] - 2);
        i[a] = ia;
        f[a] = ua - (float)ia;
    }
    c.base = (i[2] * res[1] + i[1]) * res[0] + i[0];
    c.fx = f[0]; c.fy = f[1]; c.fz = f[2];
    return c;
}

// value and gradient (w.r.t. x) of the trilinear interpolant
__device__ __forceinline__ float tri_eval(const float* __restrict__ g, const int res[3], const float scale[3],
                                          const TriCell& c, float3* grad) {
    const int sx = 1, sy = res[0], sz = res[0] * res[1];
    const float v000 = ld_global(g + c.base), v100 = ld_global(g + c.base + sx), v010 = ld_global(g + c.base + sy),
                v110 = ld_global(g + c.base + sx + sy);
    const float v001 = ld_global(g + c.base + sz), v101 = ld_global(g + c.base + sx + sz),
                v011 = ld_global(g + c.base + sy + sz), v111 = ld_global(g + c.base + sx + sy + sz);
    const float fx = c.fx, fy = c.fy, fz = c.fz;
    const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
    const float x00 = gx * v000 + fx * v100, x10 = gx * v010 + fx * v110;
    const float x01 = gx * v001 + fx * v101, x11 = gx * v011 + fx * v111;
    const float y0 = gy * x00 + fy * x10, y1 = gy * x01 + fy * x11;
    if (grad) {
        const float dx = gy * gz * (v100 - v000) + fy * gz * (v110 - v010) + gy * fz * (v101 - v001) +
                         fy * fz * (v111 - v011);
        const float dy = gz * (x10 - x00) + fz * (x11 - x01);
        const float dz = y1 - y0;
        *grad = f3(dx * scale[0], dy * scale[1], dz * scale[2]);
    }
    return gz * y0 + fz * y1;
}

// GP statistics at x (Sec. 3.1, Eq. joint_fg): f ~ N(mu, sigma^2) and, independent at the
// same point, g ~ N(grad mu, Sigma) with Sigma = s^2 (I - n n^T) + s_n^2 n n^T about the
// local mean-gradient direction n (z where grad mu = 0), s = sigma / l, s_n = sigma / l_n;
// ak = (s_n / s)^2 - 1 (0 for the isotropic kernel, Sigma = s^2 I).
struct PointQ {
    float mu;
    float3 G;
    float sigma;
    float s;
    float ak;
    float albedo;
    int ggx;        // GGX height-field macrofacet (scene-wide)
    float feta, fk; // conductor Fresnel IOR (scene-wide; feta = 0: none)
    int cond;       // conditioned GP: G is the gradient mean given f = 0 and L the Cholesky factor
    float L[6];     // of its covariance (l00, l10, l11, l20, l21, l22)
};

__device__ __forceinline__ PointQ eval_point(const SceneDev& S, float3 x) {
    PointQ q;
    int which;
    mean_geom(S, x, q.mu, q.G, which);
    if (S.offset) {
        float3 go;
        const TriCell c = tri_cell(S.off_res, S.off_scale, S.lo, x);
        q.mu += tri_eval(S.offset, S.off_res, S.off_scale, c, &go);
        q.G = q.G + go;
    }
    if (S.var_grid) {
        const TriCell c = tri_cell(S.var_res, S.var_scale, S.lo, x);
        q.sigma = sqrtf(tri_eval(S.var_grid, S.var_res, S.var_scale, c, nullptr));
        q.s = q.sigma / S.lengthscale;
    } else {   // the same correctly rounded values, formed once per scene
        q.sigma = S.sigma0;
        q.s = S.s0;
    }
    q.ak = S.aniso_k;
    q.ggx = S.ggx;
    q.feta = S.f_eta;
    q.fk = S.f_k;
    q.albedo = (S.albedo_per_prim && which >= 0) ? ld_const(S.prims + 2 * which + 1).w : S.albedo;
    q.cond = 0;
    return q;
}

// GP conditioned on noisy point observations (Sec. 3.1, Eq. condition_gp), applied to the
// pair (f(x), grad f(x)) whose covariances with f(C) are k_j = kappa(x, x_j) and
// grad_x k_j = -k_j (x - x_j) / l^2, prior covariance diag(sigma^2, sigma^2 / l^2 I):
//   mu_C = mu + sum_j alpha_j k_j,   grad mu_C = grad mu - (1/l^2) sum_j alpha_j k_j (x - x_j),
//   with w = L^-1 k and W_a = L^-1 d k / dx_a (L L^T = kappa(C,C) + noise I):
//   var_C = sigma^2 - |w|^2,  c = cov(grad f, f) = -W^T w,  Sgg = sigma^2/l^2 I - W^T W.
// W_a is formed as -(1/l^2) (x_a w - P_a), P_a = sum_j (L^-1_ij x_ja) k_j, so that one pass
// over the lower triangle of L^-1 gives all four right-hand sides with four FMAs per entry,
// the entry's (L^-1_ij, L^-1_ij x_j) being one wave-uniform float4 (a scalar load), while only
// k_j is kept per lane, four to a float4 in that lane's column of an LDS array (no lane
// reads another's column: no barrier).  Rows are zero-padded to whole blocks of four
// entries; a padded entry adds 0 * k_j exactly, so the sums are those of the bare triangle.
// The gradient given f(x) = 0 (the surface) then has mean grad mu_C - c mu_C / var_C and
// covariance Sgg - c c^T / var_C, kept as its Cholesky factor; s (used only by the
// proposal) is the root of a third of its trace.
// Workgroups of at most kCondBlock threads.
constexpr int kCondBlock = 256;
__device__ __forceinline__ void condition_point(const SceneDev& S, float3 x, PointQ& q) {
    __shared__ float4 kl[kMaxObs / 4][kCondBlock];
    const int lt = threadIdx.x;
    const float il2 = 1.0f / (S.lengthscale * S.lengthscale);
    const float var = S.variance;
    const float3 xr = x - f3(S.obs_c[0], S.obs_c[1], S.obs_c[2]);
    const int n = S.n_obs;
    float am = 0.0f;
    float3 amx = f3(0.0f, 0.0f, 0.0f);
    for (int g = 0; g < (n + 3) >> 2; ++g) {
        float kv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * g + e;
            const float4 o = ld_const(S.obs + j);   // zeros beyond n (the array holds kMaxObs entries)
            const float3 d = xr - f3(o.x, o.y, o.z);
            const float kj = j < n ? var * expf(-0.5f * il2 * dot(d, d)) : 0.0f;
            kv[e] = kj;
            const float ak = o.w * kj;
            am += ak;
            amx = amx + ak * f3(o.x, o.y, o.z);
        }
        kl[g][lt] = make_float4(kv[0], kv[1], kv[2], kv[3]);
    }
    const float mu = q.mu + am;
    const float3 gm = q.G - il2 * (am * xr - amx);
    float ww = 0.0f;
    float3 c = f3(0.0f, 0.0f, 0.0f);
    float sxx = 0.0f, sxy = 0.0f, sxz = 0.0f, syy = 0.0f, syz = 0.0f, szz = 0.0f;
    const float4* row = S.obs_tri;
    for (int i = 0; i < n; ++i) {
        float w = 0.0f;
        float3 P = f3(0.0f, 0.0f, 0.0f);
        const int rb = cond_row_blocks(i);
        for (int g = 0; g < rb; ++g) {
            const float4 kv = kl[g][lt];
            const float4 b0 = ld_const(row + 4 * g), b1 = ld_const(row + 4 * g + 1),
                         b2 = ld_const(row + 4 * g + 2), b3 = ld_const(row + 4 * g + 3);
            // entries j = 4g .. 4g + 3 in order (padding adds 0 * k_j exactly)
            const float4 bs[4] = {b0, b1, b2, b3};
            const float ks[4] = {kv.x, kv.y, kv.z, kv.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                w = fmaf(bs[e].x, ks[e], w);
                P.x = fmaf(bs[e].y, ks[e], P.x);
                P.y = fmaf(bs[e].z, ks[e], P.y);
                P.z = fmaf(bs[e].w, ks[e], P.z);
            }
        }
        row += 4 * rb;
        const float3 W = (-il2) * (w * xr - P);
        ww += w * w;
        c = c + w * W;
        sxx += W.x * W.x; sxy += W.x * W.y; sxz += W.x * W.z;
        syy += W.y * W.y; syz += W.y * W.z; szz += W.z * W.z;
    }
    const float vc = fmaxf(var - ww, 1e-6f * var);   // positive whatever the rounding
    const float iv = 1.0f / vc;
    c = -c;
    const float sg = var * il2;
    const float Sxx = sg - sxx - c.x * c.x * iv, Sxy = -sxy - c.x * c.y * iv, Sxz = -sxz - c.x * c.z * iv;
    const float Syy = sg - syy - c.y * c.y * iv, Syz = -syz - c.y * c.z * iv, Szz = sg - szz - c.z * c.z * iv;
    const float l00 = sqrtf(Sxx);
    const float l10 = Sxy / l00, l20 = Sxz / l00;
    const float l11 = sqrtf(fmaxf(Syy - l10 * l10, 0.0f));
    const float l21 = (Syz - l20 * l10) / l11;
    const float l22 = sqrtf(fmaxf(Szz - l20 * l20 - l21 * l21, 0.0f));
    q.cond = 1;
    q.mu = mu;
    q.sigma = sqrtf(vc);
    q.G = gm - (mu * iv) * c;
    q.s = sqrtf((Sxx + Syy + Szz) * (1.0f / 3.0f));
    q.L[0] = l00; q.L[1] = l10; q.L[2] = l11; q.L[3] = l20; q.L[4] = l21; q.L[5] = l22;
}

// ---------------------------------------------------------------------------
// Macrofacet medium.
// ---------------------------------------------------------------------------
// Scaled complementary error function erfcx(y) = e^{y^2} erfc(y), branch-free: for y >= 0,
// t e^{P(2t - 1)} with t = 1 / (1 + y/2) and P the degree-12 least-squares fit of
// log(erfcx(y) / t) over t in (0, 1] (coefficients from fit_erfcx.py beside this file;
// relative error below 4e-7 in single precision for every y >= 0); for y < 0 through
// erfcx(y) = 2 e^{y^2} - erfcx(-y), which does not cancel (the first term is at least 2,
// the second at most 1).  Used by the density and the projected area, the per-collision
// work; the NDF keeps the library's erfcxf because its bracket cancels to O(k^-4) and
// amplifies any error of erfcx by about k^4.
__device__ __forceinline__ float erfcx_pos(float y) {
    const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, y, 1.0f));
    const float s = fmaf(2.0f, t, -1.0f);
    float p = 1.440079031e-05f;
    p = fmaf(p, s, -8.994532810e-05f);
    p = fmaf(p, s, -3.500219551e-05f);
    p = fmaf(p, s, 5.805670305e-04f);
    p = fmaf(p, s, -1.797636438e-04f);
    p = fmaf(p, s, -2.295030673e-03f);
    p = fmaf(p, s, 1.769224540e-03f);
    p = fmaf(p, s, 8.811324156e-03f);
    p = fmaf(p, s, -9.874227007e-03f);
    p = fmaf(p, s, -4.689404184e-02f);
    p = fmaf(p, s, 4.734339379e-02f);
    p = fmaf(p, s, 6.726431725e-01f);
    p = fmaf(p, s, -6.717940849e-01f);
    return t * __expf(p);
}
// q(y) = 1 - sqrt(pi) y erfcx(y), y >= 0, from its own fit (fit_mills.py): e^{P(2t - 1)} /
// (1 + 2 y + 2 y^2), t = 1 / (1 + y / 2), about 2.3e-7 relative error in float32.  It is the
// bracket of the projected area of a ray travelling up the mean gradient and of the density's
// log-derivative inside the medium; formed from erfcx as 1 - sqrt(pi) y erfcx(y) it cancels to
// about 1 / (2 y^2) and loses digits in proportion to y^2.
__device__ __forceinline__ float mills_q(float y) {
    const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, y, 1.0f));
    const float s = fmaf(2.0f, t, -1.0f);
    float p = -1.845568261e-04f;
    p = fmaf(p, s, -1.230521427e-03f);
    p = fmaf(p, s, -2.690260467e-03f);
    p = fmaf(p, s, 7.366559191e-04f);
    p = fmaf(p, s, 8.175576550e-03f);
    p = fmaf(p, s, 4.825736499e-03f);
    p = fmaf(p, s, 7.088512245e-03f);
    p = fmaf(p, s, 5.314682672e-02f);
    p = fmaf(p, s, 6.092653941e-02f);
    p = fmaf(p, s, -1.119519912e-01f);
    p = fmaf(p, s, -2.806525253e-01f);
    p = fmaf(p, s, 5.447329695e-02f);
    p = fmaf(p, s, 2.073366479e-01f);
    return __expf(p) * __builtin_amdgcn_rcpf(fmaf(2.0f * y, 1.0f + y, 1.0f));
}
// Ratio-tracking factor 1 - sigma_t / majorant with a single reciprocal instruction (about
// one ulp) instead of a correctly rounded division; every tracer form and the adjoint replay
// use this one function, so their transmittances and roulette decisions stay identical.
__device__ __forceinline__ float null_ratio(float sig, float maj) { return 1.0f - sig * __builtin_amdgcn_rcpf(maj); }

__device__ __forceinline__ float erfcx_any(float y) {
    const float r = erfcx_pos(fabsf(y));
    return y >= 0.0f ? r : 2.0f * expf(y * y) - r;
}

// Density rho = phi(mu; 0, sigma^2) / Phi(mu; 0, sigma^2) = sqrt(2/pi) / (sigma erfcx(-mu/(sigma sqrt2))).
__device__ __forceinline__ float rho_of(float mu, float sigma) {
    const float is = __builtin_amdgcn_rcpf(sigma);
    const float z = mu * is;
    return kSqrt2OverPi * is * __builtin_amdgcn_rcpf(erfcx_any(-z * kInvSqrt2));
}

// Cosine between a unit direction and the local mean-gradient direction (z where G = 0).
__device__ __forceinline__ float cos_to_normal(float3 G, float3 w) {
    const float g2 = dot(G, G);
    return g2 > 0.0f ? dot(w, G) * rsqrtf(g2) : w.z;
}

// Projected area sigma(d) = E[max(0, -d.g)], g ~ N(G, Sigma): -d.g is Gaussian with mean
// -m, m = d.G, and standard deviation s_d = s sqrt(1 + ak c^2), c = d.n; with z = m / s_d,
//   s_d phi(z) - m Phi(-z) = max(-m, 0) + s_d phi(z) (1 - |z| sqrt(pi/2) erfcx(|z|/sqrt2)),
// one scaled complementary error function for either sign of z (Phi of a non-positive
// argument written as sqrt(pi/2) phi erfcx).  Equals the paper's Lambda(w) cos(theta)
// (Eq. generalized_lambda, alpha_x = alpha_y = sqrt2 s, alpha_z = sqrt2 s_n) for G of unit
// length; scales with |G| otherwise.
__device__ __forceinline__ float sigma_proj(float3 G, float s, float ak, float3 d) {
    const float m = dot(d, G);
    float sd = s;
    if (ak != 0.0f) {
        const float c = cos_to_normal(G, d);
        sd = s * sqrtf(1.0f + ak * (c * c));
    }
    const float z = m * __builtin_amdgcn_rcpf(sd);
    const float az = fabsf(z);
    const float ph = kInvSqrt2Pi * expf(-0.5f * z * z);
    return fmaxf(-m, 0.0f) + sd * ph * mills_q(az * kInvSqrt2);
}

// Generalized NDF (Sec. 4.2.2) for g ~ N(G, Sigma): int_0^inf P(t wm) t^3 dt in closed form.
// With c = wm.n, r^2 = 1 + ak = (s_n / s)^2 and a = 1 - c^2 ak / (1 + ak) (wm^T Sigma^-1 wm
// = a / s^2), the exponent of P(t wm) is -(a/s^2)(t - t0)^2 / 2 - q / 2 with
//   k = G.wm / (s r^2 sqrt(a)),  q = |G|^2 (1 - c^2) / (s^2 r^2 a),  |G|^2/(s r)^2 = k^2 + q,
// so that (Eq. macro_ndf with alpha_x = alpha_y = sqrt2 s, alpha_z = sqrt2 s_n)
//   D = s / (r a^2) (2 pi)^(-3/2) [ (k^2 + 2) e^{-|G|^2/(2 s^2 r^2)} + sqrt(2 pi) k (k^2 + 3) e^{-q/2} Phi(k) ],
// and, with e^{-q/2} Phi(k) written through erfcx(|k|/sqrt2) for either sign of k,
//   D = s / (r a^2) (2 pi)^(-3/2) [ e^{-|G|^2/(2 s^2 r^2)} ((k^2+2) - sqrt(pi/2) |k| (k^2+3) erfcx(|k|/sqrt2))
//                                   + [k > 0] sqrt(2 pi) k (k^2+3) e^{-q/2} ].
// For the isotropic kernel (ak = 0): r = a = 1, k = G.wm / s, q = |G x wm|^2 / s^2.
__device__ __forceinline__ float ndf(float3 G, float s, float ak, float3 wm) {
    const float is = 1.0f / s;
    const float g2 = dot(G, G);
    float k, q, isr2, pre;
    if (ak != 0.0f) {
        const float r2 = 1.0f + ak;
        const float c = cos_to_normal(G, wm);
        const float a = 1.0f - (c * c) * (ak / r2);
        isr2 = is * is / r2;
        k = dot(G, wm) * is * rsqrtf(a) / r2;
        q = g2 * fmaxf(1.0f - c * c, 0.0f) * isr2 / a;
        pre = s * kInv2PiPow1p5 * rsqrtf(r2) / (a * a);
    } else {   // isotropic kernel: r = a = 1, q = |G x wm|^2 / s^2
        const float3 cr = cross(G, wm);
        isr2 = is * is;
        k = dot(G, wm) * is;
        q = dot(cr, cr) * isr2;
        pre = s * kInv2PiPow1p5;
    }
    const float eG = expf(-0.5f * g2 * isr2);
    const float k2 = k * k, akk = fabsf(k);
    const float b = (k2 + 2.0f) - kSqrtHalfPi * akk * (k2 + 3.0f) * erfcxf(akk * kInvSqrt2);
    const float up = k > 0.0f ? kSqrt2Pi * k * (k2 + 3.0f) * expf(-0.5f * q) : 0.0f;
    return pre * fmaxf(eG * b + up, 0.0f);
}

// GGX height-field macrofacet (any NDF may replace Beckmann under the Smith assumption, end
// of Sec. 4.1), about n = G/|G| with roughness alpha = sqrt(2) s / |G|, scaled by |G|:
//   sigma(d) = |G| (c + sqrt(c^2 + alpha^2 (1 - c^2))) / 2, c = -d.n of either sign
//            = (-m + sqrt(m^2 + 2 s^2 (1 - c^2))) / 2, m = d.G
// (cos (1 + Lambda) entering from above, |cos| Lambda from below, Lambda the GGX Smith
// function), and D(wm) = |G| alpha^2 / (pi ((n.wm)^2 (alpha^2 - 1) + 1)^2) for n.wm > 0.
__device__ __forceinline__ float sigma_proj_ggx(float3 G, float s, float3 d) {
    const float g2 = dot(G, G);
    if (!(g2 > 0.0f)) return 0.0f;
    const float m = dot(d, G);
    const float3 cr = cross(G, d);
    const float e = 2.0f * s * s * dot(cr, cr) / g2;   // 2 s^2 sin^2, sin from |G x d|
    const float r = sqrtf(m * m + e);
    // (-m + r) / 2, rationalized where it would cancel (rays leaving the surface, m > 0)
    return m > 0.0f ? 0.5f * e / (m + r) : 0.5f * (r - m);
}
__device__ __forceinline__ float ndf_ggx(float3 G, float s, float3 wm) {
    const float g2 = dot(G, G);
    if (!(g2 > 0.0f)) return 0.0f;
    const float ign = rsqrtf(g2);
    const float c = dot(wm, G) * ign;
    if (!(c > 0.0f)) return 0.0f;
    const float a2 = 2.0f * s * s / g2;
    const float den = c * c * (a2 - 1.0f) + 1.0f;
    return (1.0f / ign) * a2 / (kPi * den * den);
}

// Projected area and generalized NDF for g ~ N(G, L L^T) with a full covariance (the
// conditioned GP): -d.g has mean -d.G and standard deviation |L^T d|; with y = L^-1 wm and
// u = L^-1 G the NDF's exponent is -(A/2)(t - B/A)^2 - q/2 with A = |y|^2, B = y.u and
// q = |u x y|^2 / A, so the closed form above holds with k = B / sqrt(A), e^{-|u|^2/2} and the
// prefactor (2 pi)^(-3/2) / (l00 l11 l22 A^2).
__device__ __forceinline__ float sigma_proj_chol(float3 G, const float* L, float3 d) {
    const float3 u = f3(L[0] * d.x + L[1] * d.y + L[3] * d.z, L[2] * d.y + L[4] * d.z, L[5] * d.z);
    const float sd = sqrtf(dot(u, u));
    const float m = dot(d, G);
    const float z = m * __builtin_amdgcn_rcpf(sd);
    const float az = fabsf(z);
    const float ph = kInvSqrt2Pi * expf(-0.5f * z * z);
    return fmaxf(-m, 0.0f) + sd * ph * mills_q(az * kInvSqrt2);
}
__device__ __forceinline__ float3 chol_solve3(const float* L, float3 b) {
    const float y0 = b.x / L[0];
    const float y1 = (b.y - L[1] * y0) / L[2];
    return f3(y0, y1, (b.z - L[3] * y0 - L[4] * y1) / L[5]);
}
__device__ __forceinline__ float ndf_chol(float3 G, const float* L, float3 wm) {
    const float3 y = chol_solve3(L, wm), u = chol_solve3(L, G);
    const float A = dot(y, y);
    const float k = dot(y, u) * rsqrtf(A);
    const float3 cr = cross(u, y);
    const float q = dot(cr, cr) / A;
    const float pre = kInv2PiPow1p5 / (L[0] * L[2] * L[5] * A * A);
    const float eG = expf(-0.5f * dot(u, u));
    const float k2 = k * k, akk = fabsf(k);
    const float b = (k2 + 2.0f) - kSqrtHalfPi * akk * (k2 + 3.0f) * erfcxf(akk * kInvSqrt2);
    const float up = k > 0.0f ? kSqrt2Pi * k * (k2 + 3.0f) * expf(-0.5f * q) : 0.0f;
    return pre * fmaxf(eG * b + up, 0.0f);
}

// The medium's projected area and NDF at a point (generalized, GGX or conditioned macrofacet).
__device__ __forceinline__ float sigma_proj_at(const PointQ& q, float3 d) {
    if (q.cond) return sigma_proj_chol(q.G, q.L, d);
    return q.ggx ? sigma_proj_ggx(q.G, q.s, d) : sigma_proj(q.G, q.s, q.ak, d);
}
__device__ __forceinline__ float ndf_at(const PointQ& q, float3 wm) {
    if (q.cond) return ndf_chol(q.G, q.L, wm);
    return q.ggx ? ndf_ggx(q.G, q.s, wm) : ndf(q.G, q.s, q.ak, wm);
}

__device__ __forceinline__ float sigma_t_of(const PointQ& q, float3 d) {
    return rho_of(q.mu, q.sigma) * sigma_proj_at(q, d);
}

// Unpolarized Fresnel reflectance of a conductor with IOR eta + i k at incidence cosine c
// (real form of the Fresnel equations: a^2 + b^2 = |n^2 - sin^2|, a = Re sqrt(n^2 - sin^2)).
__device__ __forceinline__ float fresnel_conductor(float c, float eta, float k) {
    c = fminf(fmaxf(c, 0.0f), 1.0f);
    const float c2 = c * c, s2 = 1.0f - c2;
    const float t0 = eta * eta - k * k - s2;
    const float a2b2 = sqrtf(t0 * t0 + 4.0f * eta * eta * k * k);
    const float a = sqrtf(fmaxf(0.5f * (a2b2 + t0), 0.0f));
    const float t1 = a2b2 + c2, t2 = 2.0f * c * a;
    const float rs = (t1 - t2) / (t1 + t2);
    const float t3 = c2 * a2b2 + s2 * s2, t4 = t2 * s2;
    const float rp = rs * (t3 - t4) / (t3 + t4);
    return 0.5f * (rp + rs);
}

// F(-w_o, w_m) of Eq. phase at <v, w_m> = c: the albedo, times the conductor Fresnel
// reflectance when an index of refraction is given.
__device__ __forceinline__ float fresnel_F(const PointQ& q, float c) {
    return q.feta > 0.0f ? q.albedo * fresnel_conductor(c, q.feta, q.fk) : q.albedo;
}

// Conductor phase function for travel direction d, scattered direction wi.
__device__ __forceinline__ float phase_eval(const PointQ& q, float3 d, float3 wi) {
    float3 h = wi - d;
    const float hn = sqrtf(dot(h, h));
    if (hn < 1e-7f) return 0.0f;
    h = (1.0f / hn) * h;
    return fresnel_F(q, -dot(d, h)) * ndf_at(q, h) / (4.0f * sigma_proj_at(q, d));
}

// ---------------------------------------------------------------------------
// Mixture proposal over half vectors: Beckmann visible normals with probability R (while v
// is above the local horizon), uniform over the hemisphere about v otherwise.
// ---------------------------------------------------------------------------
struct Proposal {
    float3 N, T, B;
    float alpha, cosv, a;   // a = cot(theta_v) after stretching to unit roughness
    float Reff;
    bool beck;              // visible-normal component available (Beckmann, or GGX for a GGX macrofacet)
    bool ggx;
};

__device__ __forceinline__ float beckmann_lambda(float a) {
    if (isinf(a)) return 0.0f;
    return 0.5f * (expf(-a * a) * kInvSqrtPi / a - erfcf(a));
}

__device__ __forceinline__ float mixture_pdf(const Proposal& p, float3 v, float3 wm) {
    const float vm = dot(v, wm);
    if (vm <= 0.0f) return 0.0f;
    float pb = 0.0f;
    if (p.beck && p.ggx) {   // GGX visible normals: <v, wm> D(wm) / (cos_v (1 + Lambda(v)))
        const float cm = dot(wm, p.N);
        if (cm > 0.0f) {
            const float a2 = p.alpha * p.alpha;
            const float den = cm * cm * (a2 - 1.0f) + 1.0f;
            const float D = a2 / (kPi * den * den);
            const float lc = 0.5f * (p.cosv + sqrtf(p.cosv * p.cosv + a2 * (1.0f - p.cosv * p.cosv)));
            pb = vm * D / lc;
        }
    } else if (p.beck) {
        const float cm = dot(wm, p.N);
        if (cm > 0.0f) {
            const float3 cr = cross(wm, p.N);
            const float c2 = cm * cm, a2 = p.alpha * p.alpha;
            const float D = expf(-dot(cr, cr) / (c2 * a2)) / (kPi * a2 * c2 * c2);
            pb = vm * D / ((1.0f + beckmann_lambda(p.a)) * p.cosv);
        }
    }
    return p.Reff * pb + (1.0f - p.Reff) * (0.5f / kPi);
}

// Slope along the incidence plane at unit roughness: solve F(x) = u F(a) on [-8, a],
// F(x) = erfc(-x)/2 + exp(-x^2)/(2 a sqrt(pi)), by bracketed Newton iterations.  The start
// blends the two regimes of the visible-slope density (1 - x/a) e^{-x^2}: the Gaussian quantile
// erfinv(2u - 1) for large a (near normal incidence) and, for small a, the quantile
// -sqrt(-ln u) of the tail |x| e^{-x^2} that dominates there; weight min(a, 1).  The start only
// shortens the iteration; the bracket and the tolerance fix the root.  Kept out of line: inlined
// into every kernel, its code slowed the conditioned-GP specialization by a fifth.
__device__ __noinline__ float slope_start(float a, float u) {
    const float g = u > 0.0f ? erfinvf(2.0f * u - 1.0f) : 0.0f;
    const float t = -sqrtf(-logf(fmaxf(u, 1e-30f)));
    if (isinf(a)) return g;
    const float w = fminf(a, 1.0f);
    return fminf(w * g + (1.0f - w) * t, a);
}
__device__ __forceinline__ float sample_slope_x(float a, float u) {
    const bool fin = !isinf(a);
    const float c2 = fin ? 0.5f * kInvSqrtPi / a : 0.0f;
    const float ia = fin ? 1.0f / a : 0.0f;
    const float Fa = fin ? 0.5f * erfcf(-a) + expf(-a * a) * c2 : 1.0f;
    const float target = u * Fa;
    float lo = -8.0f, hi = fin ? fminf(a, 8.0f) : 8.0f;
    if (target <= 0.5f * erfcf(8.0f) + expf(-64.0f) * c2) return lo;
    float x = fminf(fmaxf(slope_start(a, u), lo), hi);
    for (int it = 0; it < 48; ++it) {
        const float e = expf(-x * x);
        const float fx = 0.5f * erfcf(-x) + e * c2 - target;
        if (fx == 0.0f) break;
        if (fx > 0.0f) hi = x; else lo = x;
        const float fp = e * kInvSqrtPi * (1.0f - x * ia);
        float xn = fp > 0.0f ? x - fx / fp : 0.5f * (lo + hi);
        if (!(xn > lo && xn < hi)) xn = 0.5f * (lo + hi);
        const float step = xn - x;
        x = xn;
        const float tol = 2e-7f * fmaxf(1.0f, fabsf(x));
        if (fabsf(step) <= tol || hi - lo <= tol) break;
    }
    return x;
}

// The random-variate part of the half-vector proposal, in single precision: which component
// (kind) and its coordinates c[0..2]: Beckmann visible slopes (x, y); GGX: (a1, a2, a3), the
// point on the unit hemisphere of the stretched configuration; uniform hemisphere: (cos theta,
// cos phi, sin phi).  combine_half_d maps them through the proposal's frame (in double).
enum { kHalfUniform = 0, kHalfBeckmann = 1, kHalfGgx = 2 };
struct HalfDraw {
    int kind;
    float c[3];
};
__device__ __forceinline__ HalfDraw draw_half(const Proposal& p, float usel, uint32_t ua24, uint32_t ub24) {
    const float ua = (float)ua24 * 0x1p-24f, ub = (float)ub24 * 0x1p-24f;
    HalfDraw h;
    if (usel < p.Reff && p.ggx) {
        // GGX visible normals (Heitz 2018): the projected hemisphere of the stretched view as a
        // disk whose far half is foreshortened; (a1, a2) on the disk, a3 lifts it (h.z of the
        // stretched view direction enters a2)
        const float hz = p.cosv / sqrtf(p.alpha * p.alpha * (1.0f - p.cosv * p.cosv) + p.cosv * p.cosv);
        const float r = sqrtf(ua);
        float sp, cp;
        sincosf(2.0f * kPi * ub, &sp, &cp);
        const float a1 = r * cp;
        const float sh = 0.5f * (1.0f + hz);
        const float a2 = (1.0f - sh) * sqrtf(fmaxf(0.0f, 1.0f - a1 * a1)) + sh * (r * sp);
        h.kind = kHalfGgx;
        h.c[0] = a1;
        h.c[1] = a2;
        h.c[2] = sqrtf(fmaxf(0.0f, 1.0f - a1 * a1 - a2 * a2));
    } else if (usel < p.Reff) {
        h.kind = kHalfBeckmann;
        h.c[0] = sample_slope_x(p.a, ua);
        // (2 k + 1) / 2^24 - 1, exact in float
        h.c[1] = erfinvf((float)((int)(2u * ub24 + 1u) - (1 << 24)) * 0x1p-24f);
        h.c[2] = 0.0f;
    } else {
        float sp, cp;
        sincosf(2.0f * kPi * ub, &sp, &cp);
        h.kind = kHalfUniform;
        h.c[0] = 1.0f - ua;
        h.c[1] = cp;
        h.c[2] = sp;
    }
    return h;
}

// ---------------------------------------------------------------------------
// The sampled half vector in double precision.
//
// A real collision's half vector sets the direction of the next segment. Formed in single
// precision (errors of about 1e-7 from the frame at the rounded position and from the final
// combination), that direction moves later cell crossings and collision points enough to
// change the discrete outcome of a later test (a short cell chord, a real/null choice) on a
// few paths in ten thousand; on deep scenes with many samples per pixel that reached more
// than a pixel in a thousand. The frame of the proposal (mean gradient and spread at the
// vertex) and the combination of the drawn coordinates with it therefore run in double; the
// inverse-CDF transforms stay in single precision (their relative error of about 1e-7 in the
// coordinates moved few decisions). It is once per real collision.
// ---------------------------------------------------------------------------
__device__ __forceinline__ D3 cross(D3 a, D3 b) {
    return d3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
// 1 / sqrt(x) and 1 / x for x > 0 in double: the hardware estimate refined by two Newton steps
// (to about one unit in the last place; the frame needs nothing closer, and these use far
// fewer registers than the correctly rounded sequences)
__device__ __forceinline__ double rsqrt_d(double x) {
    double r = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    r = r * (1.5 - hx * r * r);
    r = r * (1.5 - hx * r * r);
    return r;
}
__device__ __forceinline__ double rcp_d(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = r * (2.0 - x * r);
    r = r * (2.0 - x * r);
    return r;
}
__device__ __forceinline__ D3 unit_d(D3 a) { return rsqrt_d(dot(a, a)) * a; }
// Orthonormal basis around unit n (Duff et al., JCGT 2017), double precision.
__device__ __forceinline__ void onb(D3 n, D3& t, D3& b) {
    const double sign = copysign(1.0, n.z);
    const double a = -rcp_d(sign + n.z);
    const double bb = n.x * n.y * a;
    t = d3(1.0 + sign * n.x * n.x * a, sign * bb, -sign * n.x);
    b = d3(bb, sign + n.y * n.y * a, -n.y);
}

__device__ __forceinline__ double sdf_prim_dd(float4 a, float4 b, D3 x, D3& g) {
    const D3 v = d3(x.x - (double)a.y, x.y - (double)a.z, x.z - (double)a.w);
    if (a.x < 0.5f) {
        const double r2 = dot(v, v);
        const double ir = r2 > 0.0 ? rsqrt_d(r2) : 0.0;
        g = r2 > 0.0 ? ir * v : d3(0.0, 0.0, 1.0);
        return r2 * ir - (double)b.x;
    }
    const double sx = v.x < 0.0 ? -1.0 : 1.0, sy = v.y < 0.0 ? -1.0 : 1.0, sz = v.z < 0.0 ? -1.0 : 1.0;
    const double qx = fabs(v.x) - (double)b.x, qy = fabs(v.y) - (double)b.y, qz = fabs(v.z) - (double)b.z;
    const double qmax = fmax(qx, fmax(qy, qz));
    if (qmax > 0.0) {
        const double px = fmax(qx, 0.0), py = fmax(qy, 0.0), pz = fmax(qz, 0.0);
        const double n2 = px * px + py * py + pz * pz;
        const double in = rsqrt_d(n2);
        g = in * d3(sx * px, sy * py, sz * pz);
        return n2 * in;
    }
    int ax = 0;
    if (qy > qx) ax = 1;
    if (qz > fmax(qx, qy)) ax = 2;
    g = d3(ax == 0 ? sx : 0.0, ax == 1 ? sy : 0.0, ax == 2 ? sz : 0.0);
    return qmax;
}

// Trilinear value and gradient of a node-centred grid, double arithmetic on the float nodes.
__device__ __forceinline__ double tri_eval_d(const float* __restrict__ g, const int res[3], const double sc[3],
                                             const SceneDev& S, D3 x, D3* grad) {
    int i[3];
    double f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = fmin(fmax((comp(x, a) - S.lo_d[a]) * sc[a], 0.0), (double)(res[a] - 1));
        i[a] = min((int)floor(u), res[a] - 2);
        f[a] = u - (double)i[a];
    }
    const int base = (i[2] * res[1] + i[1]) * res[0] + i[0];
    const int sx = 1, sy = res[0], sz = res[0] * res[1];
    const double v000 = ld_global(g + base), v100 = ld_global(g + base + sx), v010 = ld_global(g + base + sy),
                 v110 = ld_global(g + base + sx + sy), v001 = ld_global(g + base + sz),
                 v101 = ld_global(g + base + sx + sz), v011 = ld_global(g + base + sy + sz),
                 v111 = ld_global(g + base + sx + sy + sz);
    const double fx = f[0], fy = f[1], fz = f[2], gx = 1.0 - fx, gy = 1.0 - fy, gz = 1.0 - fz;
    const double x00 = gx * v000 + fx * v100, x10 = gx * v010 + fx * v110;
    const double x01 = gx * v001 + fx * v101, x11 = gx * v011 + fx * v111;
    const double y0 = gy * x00 + fy * x10, y1 = gy * x01 + fy * x11;
    if (grad) {
        const double dx = gy * gz * (v100 - v000) + fy * gz * (v110 - v010) + gy * fz * (v101 - v001) +
                          fy * fz * (v111 - v011);
        *grad = d3(dx * sc[0], (gz * (x10 - x00) + fz * (x11 - x01)) * sc[1], (y1 - y0) * sc[2]);
    }
    return gz * y0 + fz * y1;
}

// Mean gradient and gradient spread s = sigma / l at x, in double (the frame of the proposal).
struct GeomD {
    D3 G;
    double s;
};
__device__ __forceinline__ GeomD eval_geom_d(const SceneDev& S, D3 x) {
    GeomD q;
    if (S.mean_kind == 0) {
        q.G = d3(0.0, 0.0, 1.0);
    } else if (S.mean_kind == 2) {
        q.G = d3(0.0, 0.0, 0.0);
    } else {
        double best = INFINITY;
        q.G = d3(0.0, 0.0, 1.0);
        // the cell's candidates (prim_candidates; the table's margin covers the rounding of x)
        const uint32_t cand = S.prim_cand ? prim_candidates(S, to_f3(x)) : 0u;
        if (cand != 0u) {
            for (int k = 0; k < (int)(cand & 3u); ++k) {
                const int i = (int)((cand >> (2 + 4 * k)) & 15u);
                D3 gi;
                const double fi = sdf_prim_dd(ld_const(S.prims + 2 * i), ld_const(S.prims + 2 * i + 1), x, gi);
                if (fi < best) { best = fi; q.G = gi; }
            }
        } else {
            for (int i = 0; i < S.n_prims; ++i) {
                D3 gi;
                const double fi = sdf_prim_dd(ld_const(S.prims + 2 * i), ld_const(S.prims + 2 * i + 1), x, gi);
                if (fi < best) { best = fi; q.G = gi; }
            }
        }
    }
    if (S.offset) {
        D3 go;
        tri_eval_d(S.offset, S.off_res, S.off_scale_d, S, x, &go);
        q.G = q.G + go;
    }
    const double var = S.var_grid ? tri_eval_d(S.var_grid, S.var_res, S.var_scale_d, S, x, nullptr)
                                  : (double)S.variance;
    q.s = var * rsqrt_d(var) * rcp_d((double)S.lengthscale);
    return q;
}

// The proposal's frame in double: normal N = G / |G| and, when v is above the local horizon,
// the incidence-plane tangent T and B = N x T, the roughness and cos(theta_v).
struct FrameD {
    D3 N, T, B;
    double alpha, cosv, a;   // a = cot(theta_v) after stretching to unit roughness
    bool beck;
};
__device__ __forceinline__ FrameD make_frame_d(const GeomD& q, D3 v) {
    FrameD f;
    f.beck = false;
    f.N = f.T = f.B = d3(0.0, 0.0, 0.0);
    f.alpha = f.cosv = f.a = 0.0;
    const double g2 = dot(q.G, q.G);
    if (g2 > 0.0) {
        const double ign = rsqrt_d(g2);
        f.N = ign * q.G;
        f.cosv = dot(v, f.N);
        if (f.cosv > 0.0) {
            f.beck = true;
            f.alpha = 1.41421356237309504880 * q.s * ign;
            const D3 vt = v - f.cosv * f.N;
            const double st2 = dot(vt, vt);
            if (st2 > 1e-14) {
                const double ist = rsqrt_d(st2);
                f.T = ist * vt;
                f.a = f.cosv * ist * rcp_d(f.alpha);
            } else {
                D3 b;
                onb(f.N, f.T, b);
                f.a = INFINITY;
            }
            f.B = cross(f.N, f.T);
        }
    }
    return f;
}

// The single-precision proposal of a double frame: the draws and the mixture pdf use it, so
// that the choice of component (v above the local horizon) is the double frame's.
__device__ __forceinline__ Proposal proposal_of(const FrameD& f, float R, int ggx) {
    Proposal p;
    p.N = to_f3(f.N);
    p.T = to_f3(f.T);
    p.B = to_f3(f.B);
    p.alpha = (float)f.alpha;
    p.cosv = (float)f.cosv;
    p.a = (float)f.a;
    p.beck = f.beck;
    p.Reff = f.beck ? R : 0.0f;
    p.ggx = ggx != 0;
    return p;
}

// The half vector from the drawn coordinates (draw_half with proposal_of(f)) and the frame f,
// in double: visible slopes or the stretched GGX hemisphere point mapped through the frame,
// or the uniform hemisphere about v.  Only N, alpha and cos(theta_v) of f are read (the
// tangents are formed again here, so that less of the frame stays live across the draws).
__device__ __forceinline__ D3 combine_half_d(const HalfDraw& h, FrameD f, D3 v) {
    if (h.kind != kHalfUniform) {
        const D3 vt = v - f.cosv * f.N;
        const double st2 = dot(vt, vt);
        if (st2 > 1e-14) {
            f.T = rsqrt_d(st2) * vt;
        } else {
            D3 b;
            onb(f.N, f.T, b);
        }
        f.B = cross(f.N, f.T);
    }
    if (h.kind == kHalfGgx) {
        // stretched configuration: local frame of the stretched view direction hs
        const double vx = dot(v, f.T), vy = dot(v, f.B);
        const D3 hs = unit_d(d3(f.alpha * vx, f.alpha * vy, f.cosv));
        const double l2 = hs.x * hs.x + hs.y * hs.y;
        D3 t1 = d3(1.0, 0.0, 0.0);
        if (l2 > 0.0) {
            const double il = rsqrt_d(l2);
            t1 = d3(-hs.y * il, hs.x * il, 0.0);
        }
        const D3 t2 = cross(hs, t1);
        const D3 m = (double)h.c[0] * t1 + (double)h.c[1] * t2 + (double)h.c[2] * hs;
        const D3 e = unit_d(d3(f.alpha * m.x, f.alpha * m.y, fmax(0.0, m.z)));
        return e.x * f.T + e.y * f.B + e.z * f.N;
    }
    if (h.kind == kHalfBeckmann) {
        const double x = f.alpha * (double)h.c[0], y = f.alpha * (double)h.c[1];
        return rsqrt_d(x * x + y * y + 1.0) * (f.N - x * f.T - y * f.B);
    }
    D3 t, b;
    onb(v, t, b);
    const double ct = (double)h.c[0];                  // 1 - u_a, exact
    const double st2 = (1.0 - ct) * (1.0 + ct);        // u_a (2 - u_a), exact
    const double st = st2 > 0.0 ? st2 * rsqrt_d(st2) : 0.0;
    return (st * (double)h.c[1]) * t + (st * (double)h.c[2]) * b + ct * v;
}

// ---------------------------------------------------------------------------
// Ray / box clipping and majorant-grid walking.
// ---------------------------------------------------------------------------
// Ray-box clip: [t0, t1] of o + t d inside the scene box (slab test with one reciprocal per
// axis, returned in inv for the cell walker of the same ray).
__device__ __forceinline__ bool clip_box(const SceneDev& S, D3 o, D3 d, double& t0, double& t1, D3& inv) {
    inv = d3(1.0 / d.x, 1.0 / d.y, 1.0 / d.z);
    t0 = 0.0;
    t1 = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double oa = comp(o, a), da = comp(d, a), ia = comp(inv, a);
        if (da == 0.0) {
            if (oa < S.lo_d[a] || oa > S.hi_d[a]) return false;
            continue;
        }
        double ta = (S.lo_d[a] - oa) * ia, tb = (S.hi_d[a] - oa) * ia;
        if (ta > tb) { const double tmp = ta; ta = tb; tb = tmp; }
        t0 = fmax(t0, ta);
        t1 = fmin(t1, tb);
    }
    return t0 < t1;
}
__device__ __forceinline__ bool clip_box(const SceneDev& S, D3 o, D3 d, double& t0, double& t1) {
    D3 inv;
    return clip_box(S, o, d, t0, t1, inv);
}

// Majorant-grid walker (3D DDA).  Boundary distances are computed once per segment with
// one reciprocal per axis and then advanced by the per-axis cell width in distance.
struct Walker {
    double tx, ty, tz;      // distance to the next boundary on each axis
    double dtx, dty, dtz;   // distance between successive boundaries on each axis
    int idx;                // flat index of the current cell (x fastest)
    int nx, ny, nz;         // cells left in the grid along each axis in the direction of travel
    int stx, sty, stz;      // flat-index step of a crossing along each axis
    // walker of ray o + t d from distance t; inv = per-axis reciprocals of d
    __device__ __forceinline__ void init(const SceneDev& S, D3 o, D3 d, D3 inv, double t) {
        const D3 p = o + t * d;
        const int ix = min(max((int)floor((p.x - S.lo_d[0]) * S.inv_cw_d[0]), 0), S.M[0] - 1);
        const int iy = min(max((int)floor((p.y - S.lo_d[1]) * S.inv_cw_d[1]), 0), S.M[1] - 1);
        const int iz = min(max((int)floor((p.z - S.lo_d[2]) * S.inv_cw_d[2]), 0), S.M[2] - 1);
        int sx, sy, sz;
        axis(S.lo_d[0], S.cw_d[0], o.x, d.x, inv.x, ix, tx, dtx, sx);
        axis(S.lo_d[1], S.cw_d[1], o.y, d.y, inv.y, iy, ty, dty, sy);
        axis(S.lo_d[2], S.cw_d[2], o.z, d.z, inv.z, iz, tz, dtz, sz);
        idx = (iz * S.M[1] + iy) * S.M[0] + ix;
        nx = sx > 0 ? S.M[0] - 1 - ix : (sx < 0 ? ix : 0);
        ny = sy > 0 ? S.M[1] - 1 - iy : (sy < 0 ? iy : 0);
        nz = sz > 0 ? S.M[2] - 1 - iz : (sz < 0 ? iz : 0);
        stx = sx;
        sty = sy * S.M[0];
        stz = sz * S.M[0] * S.M[1];
    }
    __device__ __forceinline__ static void axis(double lo, double cw, double o, double d, double inv, int i,
                                                double& tn, double& dt, int& s) {
        if (d > 0.0) {
            tn = (lo + (double)(i + 1) * cw - o) * inv;
            dt = cw * inv;
            s = 1;
        } else if (d < 0.0) {
            tn = (lo + (double)i * cw - o) * inv;
            dt = -cw * inv;
            s = -1;
        } else {
            tn = INFINITY;
            dt = 0.0;
            s = 0;
        }
    }
    // majorants as their top 16 bits (SceneDev::maj16); majorant_of turns them into floats
    __device__ __forceinline__ uint32_t majorant_bits(const SceneDev& S) const { return ld_global(S.maj16 + idx); }
    // bits of the majorant of the cell that step(ax) would enter (of the current cell if it
    // leaves the grid)
    __device__ __forceinline__ uint32_t next_majorant_bits(const SceneDev& S, int ax) const {
        const int m0 = -(int)(ax == 0), m1 = -(int)(ax == 1), m2 = -(int)(ax == 2);
        const int left = (nx & m0) | (ny & m1) | (nz & m2);
        const int n = left > 0 ? idx + ((stx & m0) | (sty & m1) | (stz & m2)) : idx;
        return ld_global(S.maj16 + n);
    }
    __device__ __forceinline__ static float majorant_of(uint32_t bits) { return __uint_as_float(bits << 16); }
    // distance along the ray to the exit of the current cell and the axis crossed (ties go
    // to the lower axis)
    __device__ __forceinline__ double exit(int& ax) const {
        const bool y = ty < tx;
        const double bxy = y ? ty : tx;
        const bool z = tz < bxy;
        ax = z ? 2 : (y ? 1 : 0);
        return z ? tz : bxy;
    }
    // cross into the next cell along ax; false if that leaves the grid (written with
    // lane masks rather than selects of members, so that the walker stays in registers)
    __device__ __forceinline__ bool step(int ax) {
        const int m0 = -(int)(ax == 0), m1 = -(int)(ax == 1), m2 = -(int)(ax == 2);
        const int left = (nx & m0) | (ny & m1) | (nz & m2);
        if (left <= 0) return false;
        nx += m0;
        ny += m1;
        nz += m2;
        idx += (stx & m0) | (sty & m1) | (stz & m2);
        tx += m0 ? dtx : 0.0;
        ty += m1 ? dty : 0.0;
        tz += m2 ? dtz : 0.0;
        return true;
    }
};

// Per-thread event counts (kept in registers, flushed once per path when requested).
struct PathStats {
    uint32_t track_steps, real, nee_steps, violations, capped, escaped, truncated, cells, phase, nee;
    uint32_t nonfinite, saturated;   // path radiances not finite or negative (added as 0) / at least 2^24
    __device__ __forceinline__ void clear() {
        track_steps = real = nee_steps = violations = capped = escaped = truncated = cells = phase = nee = 0;
        nonfinite = saturated = 0;
    }
};

}  // namespace gpss
