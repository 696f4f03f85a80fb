// Physical-optics aperture sum of Eq. (14) over facet records x frequencies x observations.
//
// For one (incidence, observation, frequency f, k = 2 pi f / c):
//   E_pq = -(j k / 2 pi) exp(-j k (k_i - k_s).c) sum_l A_pq,l sinc(k al_l) sinc(k be_l) exp(-j k D_l)
// with sinc(x) = sin(x)/x and A, al, be, D the frequency-independent record of facet l (the
// scene-frame phase is shifted back to the global origin by the (k_i - k_s).c factor).
//
// Precision (FP64PHASE): the phase k D is formed in fp64 as D * (f / c) revolutions and reduced
// to its fraction in [0, 1) in fp64 before the fp32 sin/cos; each term (fp32 amplitude x fp32 sinc and
// trig) is summed with the other three of its aligned group of four records in fp32, and the
// group sums are accumulated in fp64.  FP64ACC does the same with every term accumulated in
// fp64 on its own (no fp32 groups).  FP32 mode does all of it in fp32.  The sum is
// deterministic: a tile is 1024 records of one
// (segment, slot, observation, frequency tile); lanes own one frequency and stride over the
// tile's records in a fixed order, lanes are combined by a fixed tree, and tiles by a fixed
// loop in the reduction kernel.
#include "pe_device.h"

namespace pe {

constexpr double kC0 = 299792458.0;
constexpr double kTwoPi = 6.283185307179586476925286766559;

__global__ void k_slot_ranges(const uint32_t* __restrict__ list, const uint32_t* __restrict__ n_list,
                              int n_slots, uint32_t* __restrict__ beg, uint32_t* __restrict__ cnt) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slots) return;
    const uint32_t n = *n_list;
    auto lower = [&](uint32_t key) {
        uint32_t lo = 0, hi = n;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (entry_slot(list[mid]) < key) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const uint32_t b = lower((uint32_t)s), e = lower((uint32_t)s + 1);
    beg[s] = b;
    cnt[s] = e - b;
}

void launch_slot_ranges(const uint32_t* list, const uint32_t* n_list, int n_slots,
                        uint32_t* beg, uint32_t* cnt, hipStream_t st) {
    hipLaunchKernelGGL(k_slot_ranges, dim3((n_slots + 255) / 256), dim3(256), 0, st, list,
                       n_list, n_slots, beg, cnt);
}

// Frequency lanes of one slot's tiles: a function of that slot alone, so that the order in
// which a slot's terms are summed does not depend on the other slots of the batch.
__host__ __device__ inline int slot_ft(int n_freq) {
    int p = 1;
    while (p < n_freq && p < 64) p <<= 1;
    return p;
}

__global__ void k_po_tile_count(const SlotDesc* __restrict__ ds, const uint32_t* __restrict__ cnt,
                                int n_seg, int n_slots, uint32_t* __restrict__ out) {
    const int gs = blockIdx.x * blockDim.x + threadIdx.x;
    if (gs >= n_seg * n_slots) return;
    const SlotDesc& d = ds[gs % n_slots];
    const int ft = slot_ft(d.n_freq);
    const uint32_t nrt = (cnt[gs] + kRT - 1) / kRT;
    const uint32_t nft = (d.n_freq + ft - 1) / ft;
    out[gs] = nrt * nft * d.n_obs;
}

void launch_po_tiles(const SlotDesc* d, const uint32_t* seg_cnt, int n_seg, int n_slots, int ft,
                     uint32_t* tmp, uint32_t* tile_prefix, hipStream_t st) {
    const int n = n_seg * n_slots;
    (void)ft;
    hipLaunchKernelGGL(k_po_tile_count, dim3((n + 255) / 256), dim3(256), 0, st, d, seg_cnt, n_seg,
                       n_slots, tmp);
    launch_scan(tmp, tile_prefix, (uint32_t)n, nullptr, 1, tile_prefix + n, st);
}

// sin(x)/x.  The hardware sine is only defined for small arguments, and near-grazing facets
// (area |u' x v'| = pitch^2 / |n . k|) have sinc arguments of 1e4 .. 1e6 rad, so the argument
// is first reduced to [-1/2, 1/2) revolutions.  The division is the hardware reciprocal (1 ulp),
// well inside the error of the fp32 sine itself.
// Both branches are evaluated and one is selected (lanes of a wavefront hold different
// arguments; the small-argument series costs three operations).
// The hardware sine takes its argument in revolutions, so the reduced r goes to it directly.
__device__ inline float sinc_f(float x) {
    const float x2 = x * x;
    const float series = 1.f - x2 * (1.f / 6.f) + x2 * x2 * (1.f / 120.f);
    float r = x * 0.15915494309189535f;
    r -= rintf(r);
    const float full = __builtin_amdgcn_sinf(r) * __builtin_amdgcn_rcpf(x);
    return x2 < 1e-4f ? series : full;
}

// One exit record's fields.
struct PoRec {
    double D;
    float al, be, a[4];
};

// A tile's records from the tile's first record, so that a record is a 32-bit index from a
// wave-uniform base (the loads take the base from scalar registers).
struct PoTileRecs {
    const ExitRec* rec;
};

__device__ inline PoTileRecs po_tile_recs(const ExitRecs& er, uint64_t base) {
    PoTileRecs t;
    t.rec = er.rec + base;
    return t;
}

// r < kRT: the byte offsets fit 32 bits, which lets the loads add them to a scalar base.  A
// record is two 16-byte loads.
__device__ inline PoRec po_rec(const PoTileRecs& t, uint32_t r) {
    typedef unsigned int u4v __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) char GC;
    typedef const __attribute__((address_space(1))) u4v GU;
    const uint32_t o = r * (uint32_t)sizeof(ExitRec);
    const u4v h0 = *(GU*)((GC*)t.rec + o), h1 = *(GU*)((GC*)t.rec + o + 16);
    PoRec q;
    q.D = __hiloint2double((int)h0.y, (int)h0.x);
    q.al = __uint_as_float(h0.z);
    q.be = __uint_as_float(h0.w);
    q.a[0] = __uint_as_float(h1.x);
    q.a[1] = __uint_as_float(h1.y);
    q.a[2] = __uint_as_float(h1.z);
    q.a[3] = __uint_as_float(h1.w);
    return q;
}

// MODE: 0 fp64 phase, fp32 groups of four into fp64; 1 all fp32; 2 fp64 phase, every term into
// fp64.
template <int MODE>
__device__ void po_tile(const SlotDesc& d, uint64_t base, uint32_t rn, int f, int rl, int RL,
                        const double* __restrict__ freq, const ExitRecs& er, double acc[8]) {
    if (f >= d.n_freq || (uint32_t)rl * 4u >= rn) return;
    const double fr = freq[d.freq_base + f];
    const float kf = (float)(kTwoPi * fr / kC0);
    const double rev = fr / kC0;
    const float revf = (float)rev;
    float facc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // Records go in aligned groups of four consecutive ones, each group's loads all issued
    // before any is used (one memory round trip per group instead of three per record).  In
    // the fp64-phase mode a group's four terms are summed in fp32 and the group sums in fp64:
    // the groups are the same whatever the lane layout (ft), so each frequency's result does
    // not depend on the other frequencies of its slot.
    constexpr int kU = 4;
    const PoTileRecs tr = po_tile_recs(er, base);
    const uint32_t n_grp = (rn + kU - 1) / kU;
    for (uint32_t gi = rl; gi < n_grp; gi += RL) {
        const uint32_t r0 = gi * kU;
        float blk[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        PoRec q[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const uint32_t r = r0 + u;
            q[u] = po_rec(tr, r < rn ? r : r0);  // past the end: re-read (in range)
        }
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const PoRec& cur = q[u];
            // a re-read record past the end adds a zero (no branch, so that the compiler does
            // not sink the loads back to their uses)
            const float live = r0 + u < rn ? 1.f : 0.f;
            const float S = sinc_f(kf * cur.al) * sinc_f(kf * cur.be) * live;
            // phase in revolutions, reduced to [0, 1): fp64 product and fraction, except in the
            // all-fp32 mode
            float rf;
            if (MODE == 1) rf = __builtin_amdgcn_fractf((float)cur.D * revf);
            else rf = (float)__builtin_amdgcn_fract(cur.D * rev);
            // cos and sin of 2 pi rf (the hardware takes revolutions)
            const float cs = __builtin_amdgcn_cosf(rf), sn = __builtin_amdgcn_sinf(rf);
            const float wr = S * cs, wi = -S * sn;  // S exp(-j phase)
#pragma unroll
            for (int pq = 0; pq < 4; pq++) {
                const float a = cur.a[pq];
                if (MODE == 1) {
                    facc[2 * pq] += a * wr;
                    facc[2 * pq + 1] += a * wi;
                } else if (MODE == 2) {
                    acc[2 * pq] += (double)(a * wr);
                    acc[2 * pq + 1] += (double)(a * wi);
                } else {
                    blk[2 * pq] += a * wr;
                    blk[2 * pq + 1] += a * wi;
                }
            }
        }
        if (MODE == 0)
            for (int c = 0; c < 8; c++) acc[c] += (double)blk[c];
    }
    if (MODE == 1)
        for (int c = 0; c < 8; c++) acc[c] = facc[c];
}

// Six waves per SIMD (77 VGPRs, no spills) rather than the four its 98 registers allow.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_po_sum(const SlotDesc* __restrict__ ds,
                                                const uint32_t* __restrict__ seg_beg,
                                                const uint32_t* __restrict__ seg_cnt, int n_seg,
                                                int n_slots, const double* __restrict__ freq,
                                                ExitRecs er, uint32_t rec_stride,
                                                const uint32_t* __restrict__ tile_prefix,
                                                int fp32, int FT, double* __restrict__ partial) {
    __shared__ double red[8][256];
    const int n_gs = n_seg * n_slots;
    const uint32_t total = tile_prefix[n_gs];
    const int tid = threadIdx.x;
    for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
        int lo = 0, hi = n_gs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_prefix[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const int gs = lo, g = gs / n_slots, s = gs % n_slots;
        const SlotDesc& d = ds[s];
        const int ft = slot_ft(d.n_freq), RL = 256 / ft, fi = tid & (ft - 1), rl = tid / ft;
        const uint32_t cnt = seg_cnt[gs];
        const uint32_t nrt = (cnt + kRT - 1) / kRT;
        const uint32_t nft = (d.n_freq + ft - 1) / ft;
        const uint32_t local = t - tile_prefix[gs];
        const uint32_t rt = local % nrt, rest = local / nrt;
        const uint32_t ftile = rest % nft, o = rest / nft;
        const uint32_t r0 = seg_beg[gs] + rt * kRT;
        const uint32_t rn = min((uint32_t)kRT, cnt - rt * kRT);
        const uint64_t base = ((uint64_t)o * n_seg + g) * rec_stride + r0;
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const int f = ftile * ft + fi;
        if (fp32 == 1) po_tile<1>(d, base, rn, f, rl, RL, freq, er, acc);
        else if (fp32 == 2) po_tile<2>(d, base, rn, f, rl, RL, freq, er, acc);
        else po_tile<0>(d, base, rn, f, rl, RL, freq, er, acc);
        for (int c = 0; c < 8; c++) red[c][tid] = acc[c];
        __syncthreads();
        for (int stride = RL / 2; stride > 0; stride >>= 1) {
            if (rl < stride) {
                for (int c = 0; c < 8; c++) {
                    if (fp32 == 1) red[c][tid] = (double)((float)red[c][tid] + (float)red[c][tid + stride * ft]);
                    else red[c][tid] += red[c][tid + stride * ft];
                }
            }
            __syncthreads();
        }
        if (rl == 0)
            for (int c = 0; c < 8; c++) partial[((uint64_t)t * FT + fi) * 8 + c] = red[c][tid];
        __syncthreads();
    }
}

void launch_po_sum(const SlotDesc* d, const uint32_t* seg_beg, const uint32_t* seg_cnt,
                   int n_seg, int n_slots, const double* freq, ExitRecs er, uint32_t rec_stride,
                   const uint32_t* tile_prefix, int fp32, int ft, double* partial, int n_blocks,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_po_sum, dim3(n_blocks), dim3(256), 0, st, d, seg_beg, seg_cnt, n_seg,
                       n_slots, freq, er, rec_stride, tile_prefix, fp32, ft, partial);
}

__global__ void k_po_reduce(const SlotDesc* __restrict__ ds, const ObsDesc* __restrict__ obs,
                            int n_slots, int max_obs, int max_freq, int n_seg,
                            const double* __restrict__ freq, const uint32_t* __restrict__ seg_cnt,
                            const uint32_t* __restrict__ tile_prefix, int FT,
                            const double* __restrict__ partial, int fp32,
                            double* __restrict__ E_out, double* __restrict__ rcs_out) {
    const uint64_t total = (uint64_t)n_slots * max_obs * max_freq;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total;
         w += (uint64_t)gridDim.x * blockDim.x) {
        const int f = (int)(w % max_freq);
        const int o = (int)((w / max_freq) % max_obs);
        const int s = (int)(w / ((uint64_t)max_freq * max_obs));
        const SlotDesc& d = ds[s];
        if (o >= d.n_obs || f >= d.n_freq) continue;
        const int ft = slot_ft(d.n_freq);
        const int nft = (d.n_freq + ft - 1) / ft;
        const int ftile = f / ft, fi = f % ft;
        double S[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        float Sf[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int g = 0; g < n_seg; g++) {
            const int gs = g * n_slots + s;
            const uint32_t nrt = (seg_cnt[gs] + kRT - 1) / kRT;
            const uint64_t b = tile_prefix[gs] + ((uint64_t)o * nft + ftile) * nrt;
            for (uint32_t rt = 0; rt < nrt; rt++) {
                const double* p = partial + ((b + rt) * FT + fi) * 8;
                for (int c = 0; c < 8; c++) {
                    if (fp32 == 1) Sf[c] += (float)p[c];
                    else S[c] += p[c];
                }
            }
        }
        if (fp32 == 1)
            for (int c = 0; c < 8; c++) S[c] = Sf[c];
        const ObsDesc& O = obs[d.obs_base + o];
        const double k = kTwoPi * freq[d.freq_base + f] / kC0;
        const double ph = k * O.dc;
        const double cs = cos(ph), sn = sin(ph);
        const double pref = k / kTwoPi;
        const uint64_t out = (uint64_t)d.out_base + (uint64_t)o * d.n_freq + f;
        for (int pq = 0; pq < 4; pq++) {
            const double re = S[2 * pq], im = S[2 * pq + 1];
            const double a = re * cs + im * sn, b = im * cs - re * sn;  // S exp(-j k dc)
            const double Er = pref * b, Ei = -pref * a;                  // -(j k / 2pi) (a + jb)
            E_out[(out * 4 + pq) * 2] = Er;
            E_out[(out * 4 + pq) * 2 + 1] = Ei;
            if (rcs_out) rcs_out[out * 4 + pq] = 10.0 * log10(4.0 * 3.14159265358979323846 *
                                                              (Er * Er + Ei * Ei));
        }
    }
}

void launch_po_reduce(const SlotDesc* d, const ObsDesc* obs, int n_slots, int max_obs,
                      int max_freq, int n_seg, const double* freq, const uint32_t* seg_cnt,
                      const uint32_t* tile_prefix, int ft, const double* partial, int fp32,
                      double* E_out, double* rcs_out, hipStream_t st) {
    const uint64_t total = (uint64_t)n_slots * max_obs * max_freq;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_po_reduce, dim3(blocks), dim3(256), 0, st, d, obs, n_slots, max_obs,
                       max_freq, n_seg, freq, seg_cnt, tile_prefix, ft, partial, fp32, E_out,
                       rcs_out);
}

}  // namespace pe
