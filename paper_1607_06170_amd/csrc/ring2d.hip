// 2D single-ring P-SPIR system matrix, voxel by voxel (paper Sec 2.3).
//
// One workgroup owns one voxel.  In LDS it builds, for the voxel centre v:
//   th   the direction of every sub-segment boundary on every block face
//        (FP64 atan2), so sub-segment s = (crystal g, sub-position p) sees
//        directions I(s) = [th_k, th_k+1);
//   U    the response row of every sub-segment (Sec 2.1, Eq.2-7): FP32 table
//        entries picked with FP64 geometry (angle row, mirror, two-block remap);
//   acc  one FP64 accumulator per crystal-pair bin.
// The homogenization sweep (Eq.11, k -> infinity) pairs each sub-segment s1
// with the sub-segments s2 whose opposite directions overlap I(s1); the line
// set (s1, s2) has weight w = |I(s1) n (I(s2)+pi)| / pi and spreads into the
// bins (g1+a, g2+b) with w U1[a] U2[b] (Eq.10, summed as Eq.12), added to acc
// with LDS FP64 atomics.  The epilogue then counts / compacts (CSR), scatters
// (forward projection) or gathers (back projection) the finished column.
//
// All geometric decisions are taken in FP64 without FMA contraction; the tile
// products are FP32 (or BF16-rounded operands in the precision forms).
#include "common.hpp"

namespace psf {

__device__ __forceinline__ double wrap_2pi(double a) {
    while (a >= 2.0 * kPi) a -= 2.0 * kPi;
    while (a < 0.0) a += 2.0 * kPi;
    return a;
}

__device__ __forceinline__ double wrap_pm_pi(double a) {
    while (a > kPi) a -= 2.0 * kPi;
    while (a <= -kPi) a += 2.0 * kPi;
    return a;
}

// measure of directions in [lo1, lo1+len1) whose opposite lies in [lo2, lo2+len2)
__device__ __forceinline__ double overlap_opposite(double lo1, double len1, double lo2, double len2) {
    const double d = wrap_pm_pi(lo2 + kPi - lo1);
    return fmin(len1, d + len2) - fmax(0.0, d);
}

__device__ __forceinline__ int64_t pair_bin(int64_t i, int64_t j, int64_t n) {
    if (i > j) {
        const int64_t t = i;
        i = j;
        j = t;
    }
    return i * n - i * (i + 1) / 2 + (j - i - 1);
}

__device__ __forceinline__ void voxel_xy(const Ring2D& G, int64_t v, double& x, double& y) {
    const int64_t ix = v % G.nx, iy = v / G.nx;
    x = (ix - 0.5 * (G.nx - 1)) * G.dx + G.cx;
    y = (iy - 0.5 * (G.ny - 1)) * G.dy + G.cy;
}

// direction from (vx, vy) to boundary k of block b's face
__device__ __forceinline__ double boundary_angle(const Ring2D& G, int b, int k, double vx, double vy) {
    const double c = G.frames[2 * b], s = G.frames[2 * b + 1];
    const double xi = -G.half_w + k * (G.lam / G.P);
    const double px = G.rf * c - xi * s - vx;
    const double py = G.rf * s + xi * c - vy;
    return atan2(py, px);
}

__device__ __forceinline__ float bf16_round(float x) {  // round to nearest even, 8 significand bits
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// w * u * v in the requested precision form
__device__ __forceinline__ float tile_product(int prec, float w, float u, float v) {
    if (prec == PSF_FP32) return (w * u) * v;
    if (prec == PSF_BF16) {
        const float x = bf16_round(w * v);  // X = W V in FP32, handed on as BF16
        return bf16_round(u) * x;           // T = U^T X with BF16 operands
    }
    // hi/lo split of each operand: u v ~ uh vh + uh vl + ul vh
    const float uh = bf16_round(u), ul = bf16_round(u - uh);
    const float wv = w * v;
    const float vh = bf16_round(wv), vl = bf16_round(wv - vh);
    return uh * vh + (uh * vl + ul * vh);
}

// Response row of sub-segment (g, p) seen from (vx, vy): out[a+2] for crystal
// g+a.  src[a+2] is the table entry used (-1: zero by construction).  Returns
// 1 if an angle row beyond the table was needed (clamped to the last row).
__device__ int uv_row(const Ring2D& G, double vx, double vy, int g, int p, float* out, int* src) {
    int range = 0;
    const int b = g / G.nc, c = g - b * G.nc;
    const double cs = G.frames[2 * b], sn = G.frames[2 * b + 1];
    const double xi_m = -G.half_w + (c + (p + 0.5) / G.P) * G.lam;  // sub-segment centre
    const double D = G.rf - (cs * vx + sn * vy);                     // voxel to face line
    const double tan_a = (xi_m - (-sn * vx + cs * vy)) / D;
    const double alpha = atan(tan_a);
    const bool mirror = alpha < 0.0;
    const double aa = fabs(alpha);
    int row = (int)floor(aa * 180.0 / kPi / G.step_deg + 0.5);
    if (row > G.n_rows - 1) {
        range = 1;
        row = G.n_rows - 1;
    }
    // frame where the photon leans towards higher crystal index
    const int cm = mirror ? G.nc - 1 - c : c;
    const int pm = mirror ? G.P - 1 - p : p;
    const double nu = mirror ? xi_m + G.half_w : G.half_w - xi_m;  // distance to the approached edge
    // two-block penetration (Eq.2, 4, 5): where the ray meets the next block's face line
    int rowb = -1, p1 = 0, kvirt = 0;
    const double beta = aa - G.two_pi_R;
    if (beta > 0.0 && cm + 2 >= G.nc) {
        const double ap1 = G.sigma + cos(aa) / cos(beta) * (G.sigma + nu);
        const double n = ap1 / G.lam;
        kvirt = (int)ceil(n) - 1;  // virtual crystals ahead of the next block's first crystal
        p1 = (int)floor(((kvirt + 1) - n) * G.P);
        rowb = (int)floor(beta * 180.0 / kPi / G.step_deg + 0.5);
        if (rowb > G.n_rows - 1) {
            range = 1;
            rowb = G.n_rows - 1;
        }
    }
#pragma unroll
    for (int am = -2; am <= 2; ++am) {
        const int a = mirror ? -am : am;
        const int cc = cm + am;
        float v = 0.0f;
        int s = -1;
        if (cc >= 0 && cc < G.nc) {
            s = (row * G.P + pm) * kNb + (am + 2);
            v = G.table[s];
        } else if (cc >= G.nc && rowb >= 0) {
            const int idx = kvirt + 1 + (cc - G.nc);
            if (idx <= 2) {
                s = (rowb * G.P + p1) * kNb + (idx + 2);
                v = G.table[s];
            }
        }
        out[a + 2] = v;
        if (src) src[a + 2] = s;
    }
    return range;
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// block-wide sum; every thread gets the result.  red: LDS of >= 16 doubles
__device__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// ---------------------------------------------------------------------------
// the per-voxel kernel
// ---------------------------------------------------------------------------

constexpr int kBlock2D = 512;

struct Lds2D {
    double* acc;
    double* unw;
    double* th;
    double* gpart;
    double* red;
    float* U;
    int* src;
    unsigned char* uflag;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline size_t smem_layout(const Ring2D& G, int mode, unsigned char* base, Lds2D* L) {
    const int M1 = G.nc * G.P + 1;
    const int64_t tsize = (int64_t)G.n_rows * G.P * kNb;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align16(off + bytes);
        return o;
    };
    const size_t o_acc = take(sizeof(double) * G.nbins);
    const size_t o_unw = take(sizeof(double) * G.nseg);
    const size_t o_th = take(sizeof(double) * G.R * M1);
    const size_t o_gp = take(mode == kModeAdjGrad ? sizeof(double) * tsize : 0);
    const size_t o_red = take(sizeof(double) * 16);
    const size_t o_U = take(sizeof(float) * G.nseg * kNb);
    const size_t o_src = take(mode == kModeAdjGrad ? sizeof(int) * G.nseg * kNb : 0);
    const size_t o_fl = take(G.nseg);
    if (L) {
        L->acc = (double*)(base + o_acc);
        L->unw = (double*)(base + o_unw);
        L->th = (double*)(base + o_th);
        L->gpart = mode == kModeAdjGrad ? (double*)(base + o_gp) : nullptr;
        L->red = (double*)(base + o_red);
        L->U = (float*)(base + o_U);
        L->src = mode == kModeAdjGrad ? (int*)(base + o_src) : nullptr;
        L->uflag = base + o_fl;
    }
    return off;
}

size_t voxel2d_smem_bytes(const Ring2D& G, int mode) { return smem_layout(G, mode, nullptr, nullptr); }

template <int MODE>
__global__ void __launch_bounds__(kBlock2D) k_voxel2d(Ring2D G, VoxArgs2D A) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Lds2D L;
    smem_layout(G, MODE, smem_raw, &L);
    const int tid = threadIdx.x, bs = blockDim.x;
    const int64_t r = blockIdx.x;  // row within the voxel range
    const int64_t v = A.vox_begin + r;
    const int M1 = G.nc * G.P + 1;
    const int segs_per_block = G.nc * G.P;
    double vx, vy;
    voxel_xy(G, v, vx, vy);

    for (int i = tid; i < G.R * M1; i += bs) {
        const int b = i / M1, k = i - b * M1;
        L.th[i] = boundary_angle(G, b, k, vx, vy);
    }
    for (int64_t i = tid; i < G.nbins; i += bs) L.acc[i] = 0.0;
    if (MODE == kModeAdjGrad)
        for (int i = tid; i < G.n_rows * G.P * kNb; i += bs) L.gpart[i] = 0.0;
    __syncthreads();

    const double lo0 = L.th[0];
    for (int s = tid; s < G.nseg; s += bs) {
        const int b = s / segs_per_block, k = s - b * segs_per_block;
        L.unw[s] = lo0 + wrap_2pi(L.th[b * M1 + k] - lo0);
        L.uflag[s] = (unsigned char)uv_row(G, vx, vy, s / G.P, s % G.P, L.U + kNb * s,
                                           MODE == kModeAdjGrad ? L.src + kNb * s : nullptr);
    }
    __syncthreads();

    // table-gradient weights for this voxel: xt[bb][v]
    double xt_b[8];
    if (MODE == kModeAdjGrad) {
        for (int bb = 0; bb < A.batch && bb < 8; ++bb) xt_b[bb] = (double)A.x[(int64_t)bb * G.nvox + v];
    }

    int range_hit = 0;
    // the lines (s1, s2) of weight w spread into the bins (g1 + a, g2 + b)
    auto spread = [&](int s1, int s2, double w) {
        const float wf = (float)w;
        range_hit |= L.uflag[s1] | L.uflag[s2];
        const float* U1 = L.U + kNb * s1;
        const float* U2 = L.U + kNb * s2;
        const int g1 = s1 / G.P, g2 = s2 / G.P;
#pragma unroll
        for (int a = 0; a < kNb; ++a) {
            const float u = U1[a];
            if (MODE != kModeAdjGrad && u == 0.0f) continue;
            int i = g1 + a - 2;
            i = i < 0 ? i + G.Nc : (i >= G.Nc ? i - G.Nc : i);
#pragma unroll
            for (int bq = 0; bq < kNb; ++bq) {
                const float vv = U2[bq];
                if (MODE != kModeAdjGrad && vv == 0.0f) continue;
                int j = g2 + bq - 2;
                j = j < 0 ? j + G.Nc : (j >= G.Nc ? j - G.Nc : j);
                if (i == j) continue;
                const int64_t bin = pair_bin(i, j, G.Nc);
                const float t = tile_product(G.precision, wf, u, vv);
                if (t != 0.0f) {
                    if (G.det) {  // exact integer sums: independent of the order of arrival
                        range_hit |= fix62_ok(t) ? 0 : 1;
                        atomicAdd((unsigned long long*)&L.acc[bin], fix62(t));
                    } else {
                        atomicAdd(&L.acc[bin], (double)t);
                    }
                }
                if (MODE == kModeAdjGrad) {
                    double gsum = 0.0;
                    for (int bb = 0; bb < A.batch && bb < 8; ++bb)
                        gsum += xt_b[bb] * (double)A.y[(int64_t)bb * G.nbins + bin];
                    const double gw = gsum * w;
                    const int su = L.src[kNb * s1 + a], sv = L.src[kNb * s2 + bq];
                    if (su >= 0 && gw != 0.0) atomicAdd(&L.gpart[su], gw * (double)vv);
                    if (sv >= 0 && gw != 0.0) atomicAdd(&L.gpart[sv], gw * (double)u);
                }
            }
        }
    };
    if (G.homog_k > 0) {
        // Eq.11 with finite k: line i at direction theta_i = pi i / k, weight 1 / k,
        // ends on the sub-segments whose direction intervals hold theta_i and
        // theta_i + pi (none through a gap).  The interval is found by bisection
        // on the unwrapped starts; of the candidates around it the last one (in
        // sub-segment order) whose half-open interval holds the direction wins.
        const double w = 1.0 / G.homog_k;
        auto hit = [&](double th) -> int {
            const double x = lo0 + wrap_2pi(th - lo0);
            int lo = 0, hi = G.nseg;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (L.unw[mid] <= x) lo = mid + 1;
                else hi = mid;
            }
            int found = -1;
            for (int d = -1; d <= 1; ++d) {
                int s = lo - 1 + d;
                s = s < 0 ? s + G.nseg : (s >= G.nseg ? s - G.nseg : s);
                const int b = s / segs_per_block, k = s - b * segs_per_block;
                const double lo_s = L.th[b * M1 + k];
                const double len_s = wrap_2pi(L.th[b * M1 + k + 1] - lo_s);
                if (wrap_2pi(th - lo_s) < len_s && s > found) found = s;
            }
            return found;
        };
        for (int i = tid; i < G.homog_k; i += bs) {
            const double th = kPi * i / G.homog_k;
            const int h1 = hit(th), h2 = hit(th + kPi);
            if (h1 < 0 || h2 < 0) continue;
            spread(h1 < h2 ? h1 : h2, h1 < h2 ? h2 : h1, w);
        }
    } else
    // homogenization sweep: thread per s1, candidates s2 found by bisection on
    // the unwrapped interval starts
    for (int s1 = tid; s1 < G.nseg; s1 += bs) {
        const int b1 = s1 / segs_per_block, k1 = s1 - b1 * segs_per_block;
        const double lo1 = L.th[b1 * M1 + k1];
        const double len1 = wrap_2pi(L.th[b1 * M1 + k1 + 1] - lo1);
        double x = L.unw[s1] + kPi;
        if (x >= lo0 + 2.0 * kPi) x -= 2.0 * kPi;
        int lo = 0, hi = G.nseg;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (L.unw[mid] <= x) lo = mid + 1;
            else hi = mid;
        }
        // x can sit an ulp below the first start after the wrap: start at segment 0
        const int j0 = lo > 0 ? lo - 1 : 0;
        for (int c = 0; c < G.nseg; ++c) {
            const int jj = j0 + c;
            const int s2 = jj >= G.nseg ? jj - G.nseg : jj;
            const double base = L.unw[s2] + (jj >= G.nseg ? 2.0 * kPi : 0.0);
            if (c > 0 && base >= x + len1) break;
            if (s2 <= s1) continue;
            const int b2 = s2 / segs_per_block, k2 = s2 - b2 * segs_per_block;
            const double lo2 = L.th[b2 * M1 + k2];
            const double len2 = wrap_2pi(L.th[b2 * M1 + k2 + 1] - lo2);
            const double ov = overlap_opposite(lo1, len1, lo2, len2);
            if (!(ov > kEpsOverlap)) continue;
            spread(s1, s2, ov / kPi);
        }
    }
    if (range_hit) atomicOr(A.status, kStatRange);
    __syncthreads();
    if (G.det) {  // the integer sums back to FP64, in place
        for (int64_t i = tid; i < G.nbins; i += bs) L.acc[i] = unfix62(((const unsigned long long*)L.acc)[i]);
        __syncthreads();
    }

    if (G.top_n > 0) {
        // truncation of the extended bins (Sec 3.3): in every sinogram view, the
        // voxel keeps its top_n largest bins (ties: the lower bin).  View v holds
        // the pairs i < j with (i + j) mod Nc in {2v, 2v + 1}: one thread per view
        // finds the cut (the top_n-th largest) in one pass, then clears the rest.
        const int nview = G.Nc / 2;
        for (int v = tid; v < nview; v += bs) {
            double cv[kTopNMax];
            int cb[kTopNMax];
            int n = 0;
            for (int q = 0; q < 4; ++q) {  // i + j = s, s in {2v, 2v+1, 2v+Nc, 2v+1+Nc}
                const int s = 2 * v + (q & 1) + (q >> 1) * G.Nc;
                for (int i = s - (G.Nc - 1) > 0 ? s - (G.Nc - 1) : 0; 2 * i < s; ++i) {
                    const int64_t bin = pair_bin(i, s - i, G.Nc);
                    const double a = L.acc[bin];
                    if (!(a > 0.0)) continue;
                    // insert (a, bin) into the descending list of at most top_n
                    if (n == G.top_n && !(a > cv[n - 1] || (a == cv[n - 1] && bin < cb[n - 1]))) continue;
                    int k = n < G.top_n ? n++ : n - 1;
                    while (k > 0 && (a > cv[k - 1] || (a == cv[k - 1] && bin < cb[k - 1]))) {
                        cv[k] = cv[k - 1];
                        cb[k] = cb[k - 1];
                        --k;
                    }
                    cv[k] = a;
                    cb[k] = (int)bin;
                }
            }
            if (n < G.top_n) continue;  // the view has at most top_n bins
            const double cut = cv[n - 1];
            const int cutb = cb[n - 1];
            for (int q = 0; q < 4; ++q) {
                const int s = 2 * v + (q & 1) + (q >> 1) * G.Nc;
                for (int i = s - (G.Nc - 1) > 0 ? s - (G.Nc - 1) : 0; 2 * i < s; ++i) {
                    const int64_t bin = pair_bin(i, s - i, G.Nc);
                    const double a = L.acc[bin];
                    if (a < cut || (a == cut && bin > cutb)) L.acc[bin] = 0.0;
                }
            }
        }
        __syncthreads();
    }

    if (MODE == kModeCount) {
        double cnt = 0.0;
        for (int64_t i = tid; i < G.nbins; i += bs) {
            const double a = L.acc[i];
            cnt += (a > 0.0 && a >= A.threshold) ? 1.0 : 0.0;
        }
        cnt = block_sum(cnt, L.red);
        if (tid == 0) {
            A.row_ptr[r + 1] = (int64_t)cnt;
            if (r == 0) A.row_ptr[0] = 0;
        }
    } else if (MODE == kModeFill) {
        __shared__ int wave_tot[kBlock2D / 64];
        const int64_t start = A.row_ptr[r], cap = A.row_ptr[r + 1] - start;
        const int lane = tid & 63, wid = tid >> 6, nw = bs >> 6;
        int64_t running = 0;
        for (int64_t b0 = 0; b0 < G.nbins; b0 += bs) {
            const int64_t bin = b0 + tid;
            const double a = bin < G.nbins ? L.acc[bin] : 0.0;
            const bool keep = a > 0.0 && a >= A.threshold;
            const unsigned long long m = __ballot(keep);
            const int pre = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) wave_tot[wid] = __popcll(m);
            __syncthreads();
            int off = 0, tot = 0;
            for (int w = 0; w < nw; ++w) {
                off += w < wid ? wave_tot[w] : 0;
                tot += wave_tot[w];
            }
            if (keep) {
                const int64_t pos = running + off + pre;
                if (pos < cap) {
                    A.col[start + pos] = (int32_t)bin;
                    A.val[start + pos] = (float)a;
                } else {
                    atomicOr(A.status, kStatOverflow);
                }
            }
            running += tot;
            __syncthreads();
        }
        if (tid == 0 && running != cap) atomicOr(A.status, kStatOverflow);
    } else if (MODE == kModeFwd) {
        for (int64_t i = tid; i < G.nbins; i += bs) {
            const double a = L.acc[i];
            if (a == 0.0) continue;
            for (int bb = 0; bb < A.batch; ++bb) {
                const double xv = (double)A.x[(int64_t)bb * G.nvox + v];
                if (xv != 0.0) atomicAdd(&A.y64[(int64_t)bb * G.nbins + i], a * xv);
            }
        }
    } else {  // back projection (and table gradient)
        for (int bb = 0; bb < A.batch; ++bb) {
            double s = 0.0;
            const float* yb = A.y + (int64_t)bb * G.nbins;
            for (int64_t i = tid; i < G.nbins; i += bs) {
                const double a = L.acc[i];
                if (a != 0.0) s += a * (A.ones ? 1.0 : (double)yb[i]);
            }
            s = block_sum(s, L.red);
            if (tid == 0) {
                float* o = A.xout + (int64_t)bb * G.nvox + v;
                *o = A.accumulate ? *o + (float)s : (float)s;
            }
        }
        if (MODE == kModeAdjGrad) {
            for (int i = tid; i < G.n_rows * G.P * kNb; i += bs) {
                const double gv = L.gpart[i];
                if (gv != 0.0) atomicAdd(&A.grad64[i], gv);
            }
        }
    }
}

hipError_t launch_voxel2d(int mode, const Ring2D& G, const VoxArgs2D& a, hipStream_t st) {
    const size_t smem = voxel2d_smem_bytes(G, mode);
    const dim3 grid((unsigned)a.n_vox_range), block(kBlock2D);
    if (a.n_vox_range <= 0) return hipSuccess;
    switch (mode) {
        case kModeCount:
            hipFuncSetAttribute((const void*)k_voxel2d<kModeCount>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
            hipLaunchKernelGGL(k_voxel2d<kModeCount>, grid, block, smem, st, G, a);
            break;
        case kModeFill:
            hipFuncSetAttribute((const void*)k_voxel2d<kModeFill>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
            hipLaunchKernelGGL(k_voxel2d<kModeFill>, grid, block, smem, st, G, a);
            break;
        case kModeFwd:
            hipFuncSetAttribute((const void*)k_voxel2d<kModeFwd>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
            hipLaunchKernelGGL(k_voxel2d<kModeFwd>, grid, block, smem, st, G, a);
            break;
        case kModeAdj:
            hipFuncSetAttribute((const void*)k_voxel2d<kModeAdj>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
            hipLaunchKernelGGL(k_voxel2d<kModeAdj>, grid, block, smem, st, G, a);
            break;
        case kModeAdjGrad:
            hipFuncSetAttribute((const void*)k_voxel2d<kModeAdjGrad>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
            hipLaunchKernelGGL(k_voxel2d<kModeAdjGrad>, grid, block, smem, st, G, a);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small helpers: row-pointer scan, FP64 -> FP32 finalize, zero fill
// ---------------------------------------------------------------------------

// row_ptr[1..n] holds per-row counts; turn it into the CSR row pointers
__global__ void __launch_bounds__(1024) k_scan_rowptr(int64_t* rp, int64_t n) {
    __shared__ int64_t buf[1024];
    const int tid = threadIdx.x;
    int64_t carry = 0;
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t i = base + tid;
        buf[tid] = i < n ? rp[i + 1] : 0;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t t = tid >= off ? buf[tid - off] : 0;
            __syncthreads();
            buf[tid] += t;
            __syncthreads();
        }
        if (i < n) rp[i + 1] = carry + buf[tid];
        carry += buf[1023];
        __syncthreads();
    }
    if (tid == 0) rp[0] = 0;
}

hipError_t launch_scan_rowptr(int64_t* row_ptr, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_rowptr, dim3(1), dim3(1024), 0, st, row_ptr, n);
    return hipGetLastError();
}

__global__ void k_finalize(const double* src, float* dst, int64_t n, int accumulate) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = accumulate ? dst[i] + (float)src[i] : (float)src[i];
}

hipError_t launch_finalize(const double* src, float* dst, int64_t n, int accumulate, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, st, src, dst, n,
                       accumulate);
    return hipGetLastError();
}

__global__ void k_zero_f64(double* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace psf
