// arna_device.hpp -- device building blocks of the ARNA particle-filter step
// for gfx950 (wave64).  Everything here is __device__ code used by the kernels
// in arna.hip, including the debug entry points, so that those exercise the
// same instructions as pf_step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace arna {

constexpr int kWave = 64;

// Philox stream tags, counter word 3 bits 24..31.  Counter layout:
// (c0 = index, c1 = step, c2 = filter, c3 = tag << 24 | sub-call), key = seed.
constexpr uint32_t kTagInit = 1u, kTagRing = 2u, kTagExch = 3u, kTagProp = 4u,
                   kTagResample = 5u;

struct u4 {
    uint32_t x, y, z, w;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds; each
// multiplies words 0 and 2 by the round constants and mixes the high halves
// with words 1, 3 and the key; the key advances by the Weyl increments.
__device__ __forceinline__ u4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// floor(r * n / 2^32), an integer in [0, n).
__device__ __forceinline__ uint32_t mulshift(uint32_t r, uint32_t n) {
    return (uint32_t)(((uint64_t)r * n) >> 32);
}

// (2 (r >> 9) + 1) 2^-24: exact in float32, inside (0, 1).
__device__ __forceinline__ float unif24(uint32_t r) {
    return (float)(2u * (r >> 9) + 1u) * 0x1p-24f;
}
// (2 b + 1) 2^-19 for an 18-bit field b.
__device__ __forceinline__ float unif18(uint32_t b) {
    return (float)(2u * b + 1u) * 0x1p-19f;
}

// sin / cos of 2 pi t, t in revolutions (native v_sin_f32 / v_cos_f32).
__device__ __forceinline__ float sin_rev(float t) { return __builtin_amdgcn_sinf(t); }
__device__ __forceinline__ float cos_rev(float t) { return __builtin_amdgcn_cosf(t); }

// sqrt(-2 ln u) for u in (0, 1), through the native log2.
__device__ __forceinline__ float bm_radius(float u) {
    return __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u));
}

// Five standard normals from one Philox output: Box-Muller on the top 23 bits
// of (w0, w1) and (w2, w3), and on two 18-bit fields made of the low 9 bits of
// the four words (cosine branch).
__device__ __forceinline__ void five_normals(const u4 r, float e[5]) {
    const float ra = bm_radius(unif24(r.x));
    const float ta = unif24(r.y);
    const float rb = bm_radius(unif24(r.z));
    const float tb = unif24(r.w);
    const uint32_t b01 = (r.x & 511u) | ((r.y & 511u) << 9);
    const uint32_t b23 = (r.z & 511u) | ((r.w & 511u) << 9);
    const float rc = bm_radius(unif18(b01));
    e[0] = ra * cos_rev(ta);
    e[1] = ra * sin_rev(ta);
    e[2] = rb * cos_rev(tb);
    e[3] = rb * sin_rev(tb);
    e[4] = rc * cos_rev(unif18(b23));
}

struct Dyn {
    float a;        // sqrt(q / 3): position noise per unit normal
    float b;        // sqrt(q) sqrt(3) / 2: velocity noise from the same normal
    float c;        // sqrt(q) / 2: velocity noise from the second normal
    float sigma_I;  // intensity random walk
};

// (P): nearly-constant-velocity step, unit time, white-noise acceleration.
__device__ __forceinline__ void propagate(float s[5], const float e[5], const Dyn &d) {
    const float x = s[0] + s[2] + d.a * e[0];
    const float vx = s[2] + (d.b * e[0] + d.c * e[1]);
    const float y = s[1] + s[3] + d.a * e[2];
    const float vy = s[3] + (d.b * e[2] + d.c * e[3]);
    s[0] = x;
    s[1] = y;
    s[2] = vx;
    s[3] = vy;
    s[4] = s[4] + d.sigma_I * e[4];
}

struct Lik {
    const float *img;   // [H][W] (patch) or [F][2] (point)
    int W, H;
    float inv2s2;       // c = 1 / (2 psf_sigma^2)
    float k2;           // exp(-2 c), the step of the profile recurrence
    float bg;           // background level
    float inv_bg;       // 1 / background (Poisson mode)
    float inv_sn2;      // 1 / noise_sigma^2
};

// (U), patch mode: Gaussian log-likelihood ratio of the spot model against
// background only over the (2 HALF + 1)^2 patch centred on the nearest pixel,
//   l = (I sum g (z - B) - I^2 / 2 sum g^2) / sigma_n^2,
// with the separable profile g(u, v) = gx(u) gy(v).  Pixels outside the image
// are skipped (their weights are zero).  The patch position is decided first
// (patch_origin); the sums then read the pixels from the LDS tile or the frame.
template <int HALF>
__device__ __forceinline__ bool patch_origin(float x, float y, int W, int H, int &u0, int &v0) {
    const float cxf = floorf(x + 0.5f);
    const float cyf = floorf(y + 0.5f);
    if (!(cxf >= (float)-HALF && cxf <= (float)(W - 1 + HALF) && cyf >= (float)-HALF &&
          cyf <= (float)(H - 1 + HALF)))
        return false;
    u0 = (int)cxf - HALF;
    v0 = (int)cyf - HALF;
    return true;
}

enum PixelSource { kFromTile = 0, kFromImage = 1, kFromImageBorder = 2, kFromTileInside = 3 };

// The P profile values exp(-(u0 + j - x)^2 c), j = 0..2 HALF, by a recurrence
// outward from the centre pixel u0 + HALF (|d| <= 1/2): with d_j = u0 + j - x,
//   g_{j+1} = g_j r_j,  r_j = exp(-(2 d_j + 1) c),  r_{j+1} = r_j exp(-2 c),
// and symmetrically downward; every factor is <= 1, so values only shrink and
// underflow exactly where the profile itself does.  3 exponentials per axis.
template <int HALF>
__device__ __forceinline__ void profile(float d_centre, float c, float k2, float (&g)[2 * HALF + 1]) {
    g[HALF] = __expf(-d_centre * d_centre * c);
    float up = __expf(-(2.f * d_centre + 1.f) * c);
    float dn = __expf((2.f * d_centre - 1.f) * c);
#pragma unroll
    for (int j = 1; j <= HALF; ++j) {
        g[HALF + j] = g[HALF + j - 1] * up;
        g[HALF - j] = g[HALF - j + 1] * dn;
        up *= k2;
        dn *= k2;
    }
}

// SRC = kFromTile: `pix` points at (z - B) of the patch's first pixel in an
//   LDS tile of row pitch `pitch`, already zero outside the image;
// SRC = kFromTileInside: the same, for a tile that lies inside the image;
// SRC = kFromImage: `pix` points at the first pixel in the frame, the whole
//   patch lies inside the image (row pitch = W);
// SRC = kFromImageBorder: `pix` is the frame; every read is clamped and masked.
template <int HALF, int SRC>
__device__ __forceinline__ float patch_loglik(const float s[5], int u0, int v0, const float *pix,
                                              int pitch, const Lik &L) {
    constexpr int P = 2 * HALF + 1;
    float gx[P], gy[P];
    profile<HALF>((float)(u0 + HALF) - s[0], L.inv2s2, L.k2, gx);
    profile<HALF>((float)(v0 + HALF) - s[1], L.inv2s2, L.k2, gy);
    // pixels outside the image carry no weight (only patches at the border)
    constexpr bool inside = SRC == kFromImage || SRC == kFromTileInside;
    if (!inside && (u0 < 0 || v0 < 0 || u0 + P > L.W || v0 + P > L.H)) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            if ((unsigned)(u0 + j) >= (unsigned)L.W) gx[j] = 0.f;
            if ((unsigned)(v0 + j) >= (unsigned)L.H) gy[j] = 0.f;
        }
    }
    float sx2 = 0.f, sy2 = 0.f;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        sx2 += gx[j] * gx[j];
        sy2 += gy[j] * gy[j];
    }
    float acc = 0.f;
    if (SRC == kFromTile || SRC == kFromTileInside) {
        // every LDS read of the patch is issued before the first product.  Each
        // row gets its own base register (the empty asm hides that rows are a
        // constant apart), so the reads of a row pair up into ds_read2 with
        // small offsets instead of one address add per pair.  This needs the
        // tile at the start of the LDS block.
        float z[P * P];
        typedef __attribute__((address_space(3))) const float lds_f32;
        lds_f32 *base = (lds_f32 *)pix;
#pragma unroll
        for (int jv = 0; jv < P; ++jv) {
            lds_f32 *row = base + jv * pitch;
            __asm__("" : "+v"(row));
#pragma unroll
            for (int ju = 0; ju < P; ++ju) z[jv * P + ju] = row[ju];
        }
#pragma unroll
        for (int jv = 0; jv < P; ++jv) {
            float r = 0.f;
#pragma unroll
            for (int ju = 0; ju < P; ++ju) r += gx[ju] * z[jv * P + ju];
            acc += gy[jv] * r;
        }
        const float I = s[4];
        return (I * acc - 0.5f * I * I * (sx2 * sy2)) * L.inv_sn2;
    }
    // frame rows three at a time: bounds the loads in flight (and the registers)
#pragma unroll 3
    for (int jv = 0; jv < P; ++jv) {
        float r = 0.f;
        if (SRC == kFromTile) {
            const float *row = pix + jv * pitch;
#pragma unroll
            for (int ju = 0; ju < P; ++ju) r += gx[ju] * row[ju];
        } else if (SRC == kFromImage) {
            const float *row = pix + (size_t)jv * L.W;
#pragma unroll
            for (int ju = 0; ju < P; ++ju) r += gx[ju] * (row[ju] - L.bg);
        } else {
            const int vv = v0 + jv;
            const float *row = pix + (size_t)min(max(vv, 0), L.H - 1) * L.W;
#pragma unroll
            for (int ju = 0; ju < P; ++ju) {
                const int u = min(max(u0 + ju, 0), L.W - 1);
                const bool in = (unsigned)(u0 + ju) < (unsigned)L.W;
                r += gx[ju] * (in ? (row[u] - L.bg) : 0.f);
            }
        }
        acc += gy[jv] * r;
    }
    const float I = s[4];
    return (I * acc - 0.5f * I * I * (sx2 * sy2)) * L.inv_sn2;
}

// Poisson patch likelihood: pixel counts z ~ Poisson(B + I g), as the
// log-likelihood ratio against the background-only model,
//   l = sum_patch [ z log(1 + I g / B) - I g ],
// pixels outside the image skipped (g = 0 there).  FROM_TILE: `pix` points at
// z - B in the LDS tile (row pitch `pitch`); otherwise at the frame's first
// patch pixel (interior patches) or the frame itself (clamped reads).
template <int HALF, int SRC>
__device__ __forceinline__ float patch_loglik_poisson(const float s[5], int u0, int v0,
                                                      const float *pix, int pitch,
                                                      const Lik &L) {
    constexpr int P = 2 * HALF + 1;
    float gx[P], gy[P];
    profile<HALF>((float)(u0 + HALF) - s[0], L.inv2s2, L.k2, gx);
    profile<HALF>((float)(v0 + HALF) - s[1], L.inv2s2, L.k2, gy);
    const float I = s[4];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        if ((unsigned)(u0 + j) >= (unsigned)L.W) gx[j] = 0.f;
        if ((unsigned)(v0 + j) >= (unsigned)L.H) gy[j] = 0.f;
        gy[j] *= I;
    }
    float acc = 0.f;
#pragma unroll 3
    for (int jv = 0; jv < P; ++jv) {
        float r = 0.f;
#pragma unroll
        for (int ju = 0; ju < P; ++ju) {
            float z;
            if (SRC == kFromTile || SRC == kFromTileInside) {
                z = pix[jv * pitch + ju] + L.bg;
            } else if (SRC == kFromImage) {
                z = pix[(size_t)jv * L.W + ju];
            } else {
                const int v = min(max(v0 + jv, 0), L.H - 1), u = min(max(u0 + ju, 0), L.W - 1);
                z = pix[(size_t)v * L.W + u];
            }
            const float t = gy[jv] * gx[ju];
            r += z * __logf(1.f + t * L.inv_bg) - t;
        }
        acc += r;
    }
    return acc;
}


// Patch log-likelihood and its partial derivatives for the adjoint step:
// g = (dl/dx, dl/dy, dl/dI, dl/dsigma) at the frozen patch origin (u0, v0)
// (the origin is a step function of the position, held fixed).  With the
// profiles gx, gy of the forward step, hx = gx d, kx = gx d^2
// (d = u0 + j - x) and the row sums R0 = sum gx z, R1 = sum hx z,
// R2 = sum kx z over a patch row,
//   A = sum gy R0,  l = (I A - I^2 Sx Sy / 2) / s_n^2,  Sx = sum gx^2,
//   dA/dx = sum gy R1 / s^2,  dA/dy = sum hy R0 / s^2,
//   dA/ds = sum (gy R2 + ky R0) / s^3,
//   dSx/dx = 2 sum gx hx / s^2,  dSx/ds = 2 sum gx kx / s^3  (and in y).
// Pixels outside the image carry no weight.  FROM_TILE: `pix` points at
// z - B of the patch's first pixel in the LDS tile (row pitch `pitch`, zero
// outside the image); otherwise the frame is read with clamped indices.
template <int HALF, bool FROM_TILE>
__device__ __forceinline__ float patch_loglik_grad(const float s[5], int u0, int v0,
                                                   const float *pix, int pitch, const Lik &L,
                                                   float sigma, float g[4]) {
    constexpr int P = 2 * HALF + 1;
    float gx[P], gy[P], hx[P], hy[P], kx[P], ky[P];
    profile<HALF>((float)(u0 + HALF) - s[0], L.inv2s2, L.k2, gx);
    profile<HALF>((float)(v0 + HALF) - s[1], L.inv2s2, L.k2, gy);
    float sx = 0.f, sy = 0.f, sxh = 0.f, syh = 0.f, sxk = 0.f, syk = 0.f;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        if ((unsigned)(u0 + j) >= (unsigned)L.W) gx[j] = 0.f;
        if ((unsigned)(v0 + j) >= (unsigned)L.H) gy[j] = 0.f;
        const float dx = (float)(u0 + j) - s[0], dy = (float)(v0 + j) - s[1];
        hx[j] = gx[j] * dx;
        kx[j] = hx[j] * dx;
        hy[j] = gy[j] * dy;
        ky[j] = hy[j] * dy;
        sx += gx[j] * gx[j];
        sy += gy[j] * gy[j];
        sxh += gx[j] * hx[j];
        syh += gy[j] * hy[j];
        sxk += gx[j] * kx[j];
        syk += gy[j] * ky[j];
    }
    float A = 0.f, Ax = 0.f, Ay = 0.f, As = 0.f;
    // rows unrolled: gy, hy, ky stay in registers (a rolled loop indexes them
    // by row, one of them through scratch memory); 7% off the reverse sweep
#pragma unroll
    for (int jv = 0; jv < P; ++jv) {
        float r0 = 0.f, r1 = 0.f, r2 = 0.f;
        if (FROM_TILE) {
            typedef __attribute__((address_space(3))) const float lds_f32;
            lds_f32 *row = (lds_f32 *)pix + jv * pitch;
#pragma unroll
            for (int ju = 0; ju < P; ++ju) {
                const float z = row[ju];
                r0 += gx[ju] * z;
                r1 += hx[ju] * z;
                r2 += kx[ju] * z;
            }
        } else {
            const int v = min(max(v0 + jv, 0), L.H - 1);
            const float *row = L.img + (size_t)v * L.W;
#pragma unroll
            for (int ju = 0; ju < P; ++ju) {
                const int u = min(max(u0 + ju, 0), L.W - 1);
                const float z = row[u] - L.bg;   // weight 0 where the pixel is outside
                r0 += gx[ju] * z;
                r1 += hx[ju] * z;
                r2 += kx[ju] * z;
            }
        }
        A += gy[jv] * r0;
        Ax += gy[jv] * r1;
        Ay += hy[jv] * r0;
        As += gy[jv] * r2 + ky[jv] * r0;
    }
    const float I = s[4], k = L.inv_sn2;
    const float is2 = 2.f * L.inv2s2;   // 1 / s^2
    g[0] = k * is2 * (I * Ax - I * I * sxh * sy);
    g[1] = k * is2 * (I * Ay - I * I * syh * sx);
    g[2] = k * (A - I * sx * sy);
    g[3] = k * is2 / sigma * (I * As - I * I * (sxk * sy + syk * sx));
    return (I * A - 0.5f * I * I * (sx * sy)) * k;
}

// (U), point mode: Gaussian position observation of filter f.
__device__ __forceinline__ float loglik_point(const float s[5], const Lik &L, uint32_t f) {
    const float dx = s[0] - L.img[2 * f];
    const float dy = s[1] - L.img[2 * f + 1];
    return -(dx * dx + dy * dy) * 0.5f * L.inv_sn2;
}

// ------------------------------------------------------------- DPP wave ops
// gfx9 DPP controls: row_shr:n = 0x110 + n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143.  Lanes without a source take `old` (the identity).
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp(uint32_t v, uint32_t ident) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)v, CTRL, ROWS, 0xF, false);
}

// Inclusive scan over the 64 lanes (Hillis-Steele within rows of 16, then
// row broadcasts).  OP combines two values given as bits.
template <class OP>
__device__ __forceinline__ uint32_t wave_scan_bits(uint32_t v, uint32_t ident, OP op) {
    v = op(v, dpp<0x111, 0xF>(v, ident));
    v = op(v, dpp<0x112, 0xF>(v, ident));
    v = op(v, dpp<0x114, 0xF>(v, ident));
    v = op(v, dpp<0x118, 0xF>(v, ident));
    v = op(v, dpp<0x142, 0xA>(v, ident));
    v = op(v, dpp<0x143, 0xC>(v, ident));
    return v;
}
__device__ __forceinline__ uint32_t lane63(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
    return wave_scan_bits(v, 0u, [](uint32_t a, uint32_t b) { return a + b; });
}
__device__ __forceinline__ float wave_max_f32(float v) {
    const uint32_t r = wave_scan_bits(__float_as_uint(v), 0xFF800000u, [](uint32_t a, uint32_t b) {
        return __float_as_uint(fmaxf(__uint_as_float(a), __uint_as_float(b)));
    });
    return __uint_as_float(lane63(r));
}
// Totals of six doubles over the wave by recursive halving: at each of the
// steps across lane bits 5, 4 and 3 a lane keeps one half of its values and
// adds the partner's copy of that half, so the work halves with the step;
// bits 2..0 then sum the one value left.  Lane l ends with the total of
// v[l >> 3] (l < 48), summed in a fixed order.
__device__ __forceinline__ double wave_total6_f64(const double (&v)[6], const uint32_t lane) {
    double a4[4];
    {
        const bool hi = lane & 32u;
        const double x[8] = {v[0], v[1], v[2], v[3], v[4], v[5], 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double keep = hi ? x[i + 4] : x[i], send = hi ? x[i] : x[i + 4];
            a4[i] = keep + __shfl_xor(send, 32, kWave);
        }
    }
    double a2[2];
    {
        const bool hi = lane & 16u;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const double keep = hi ? a4[i + 2] : a4[i], send = hi ? a4[i] : a4[i + 2];
            a2[i] = keep + __shfl_xor(send, 16, kWave);
        }
    }
    const bool hi = lane & 8u;
    double t = (hi ? a2[1] : a2[0]) + __shfl_xor(hi ? a2[0] : a2[1], 8, kWave);
    t += __shfl_xor(t, 4, kWave);
    t += __shfl_xor(t, 2, kWave);
    t += __shfl_xor(t, 1, kWave);
    return t;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double block_max_d(double v, double *scratch) {
    v = wave_max_d(v);
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) scratch[w] = v;
    __syncthreads();
    double r = scratch[0];
    for (int i = 1; i < nw; ++i) r = fmax(r, scratch[i]);
    return r;
}
// Sum of NV doubles per thread; scratch holds NV doubles per wave.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *scratch) {
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = wave_sum(v[c]);
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) scratch[w * NV + c] = v[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double r = 0.0;
        for (int i = 0; i < nw; ++i) r += scratch[i * NV + c];
        v[c] = r;
    }
}
__device__ __forceinline__ void block_sum_u64(uint64_t (&v)[2], uint64_t *scratch) {
    v[0] = wave_sum_u64(v[0]);
    v[1] = wave_sum_u64(v[1]);
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) {
        scratch[2 * w] = v[0];
        scratch[2 * w + 1] = v[1];
    }
    __syncthreads();
    uint64_t a = 0, b = 0;
    for (int i = 0; i < nw; ++i) {
        a += scratch[2 * i];
        b += scratch[2 * i + 1];
    }
    v[0] = a;
    v[1] = b;
}


// Wave-wide inclusive prefix maximum of unsigned values (identity 0), and the
// exclusive one (the inclusive value of the previous lane, 0 for lane 0).
__device__ __forceinline__ uint32_t wave_incl_max_u32(uint32_t v) {
    return wave_scan_bits(v, 0u, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
}
__device__ __forceinline__ uint32_t wave_shr1(uint32_t v) {   // lane i gets lane i-1
    return dpp<0x138, 0xF>(v, 0u);
}

// floor(num / d) for num < 2^53 and a 32-bit divisor d.
__device__ __forceinline__ uint32_t div_floor_T(uint64_t num, uint32_t d, double inv_d) {
    const uint32_t q = (uint32_t)((double)num * inv_d);
    const uint64_t qd = (uint64_t)q * d;
    const uint32_t down = (uint32_t)(qd > num);
    const uint32_t up = (uint32_t)(qd + d <= num);
    return q - down + up;
}

// First output of particle i in systematic resampling: the number of
// pointers j T + V (j >= 0) below n E_i, where E_i = C_i - Q_i is the
// exclusive cumulative weight: ceil((n E_i - V) / T), or 0 if n E_i <= V.
// Exact for n E_i < 2^53 (a double reciprocal of T and one integer correction).
__device__ __forceinline__ uint32_t first_offspring(uint32_t E, uint32_t n, uint32_t T, uint32_t V,
                                                    double inv_T) {
    const uint64_t nE = (uint64_t)n * E;
    if (nE <= V) return 0;
    return div_floor_T(nE - V + T - 1, T, inv_T);
}

// ------------------------------------------------------- 128-bit integers
struct u128 {
    uint64_t hi, lo;
};
__device__ __forceinline__ u128 mul64(uint64_t a, uint64_t b) {
    return {__umul64hi(a, b), a * b};
}
// a * s for s < 2^32, assuming no overflow of 128 bits.
__device__ __forceinline__ u128 mul_small(u128 a, uint32_t s) {
    return {a.hi * s + __umul64hi(a.lo, s), a.lo * s};
}
__device__ __forceinline__ u128 sub128(u128 a, u128 b) {
    return {a.hi - b.hi - (a.lo < b.lo ? 1u : 0u), a.lo - b.lo};
}
__device__ __forceinline__ bool gt128(u128 a, u128 b) {
    return a.hi > b.hi || (a.hi == b.hi && a.lo > b.lo);
}

// Exchange count of Alg. 3 step 2 from S = sum P, D = sum P^2 (ARNA), or the
// fixed rules.  PE_eff = S^2 / D; Eq. 3 gives
//   N_ex = floor(N_p (M D - S^2) / (2 (M - 1) D)),
// zero above the cut-off PE_eff > (ppm / 10^6) M, zero for M = 1.
__device__ __forceinline__ uint32_t exchange_count(uint64_t S, uint64_t D, uint32_t M,
                                                   uint32_t n_p, uint32_t mode, int first,
                                                   uint32_t fixed_nex, uint32_t initial_nex,
                                                   uint32_t cutoff_ppm) {
    if (M <= 1) return 0;
    if (mode == 0) return fixed_nex;
    if (first) return initial_nex;
    if (D == 0) return n_p / 2;
    const u128 S2 = mul64(S, S);
    const u128 MD = mul64((uint64_t)M, D);
    if (gt128(mul_small(S2, 1000000u), mul_small(MD, cutoff_ppm))) return 0;
    const u128 num = mul_small(sub128(MD, S2), n_p);
    const u128 den = mul64(2ull * (M - 1), D);
    // quotient <= n_p / 2: binary long division over its bits
    uint32_t qt = 0;
    for (int bit = 31 - __clz(n_p | 1); bit >= 0; --bit) {
        const uint32_t cand = qt | (1u << bit);
        if (!gt128(mul_small(den, cand), num)) qt = cand;
    }
    return qt;
}

}  // namespace arna
