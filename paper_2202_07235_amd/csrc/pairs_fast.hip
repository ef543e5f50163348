// Host side of the fused Hermitian pair kernel: support checks, argument
// marshalling and dispatch to the per-precision instantiations.
#include <string.h>

#include "pairs_fast.h"

namespace radsvd {


static bool fast_q_ok(int Q) {
    return Q == 64 || Q == 96 || Q == 128 || Q == 192 || Q == 256 || Q == 384 || Q == 512;
}

bool fast_path_supported(const radsvd_plan *p, int flags) {
    if (!p->herm || p->prec == RADSVD_FP64 || !p->Af || !p->Bf) return false;
    if (flags & ~(RADSVD_OUT_BEST | RADSVD_OUT_LSE | RADSVD_OUT_FULL)) return false;
    return fast_q_ok(p->Q);
}

bool fast_band_ok(int band) { return band == 0 || band == 1 || band == 2 || band == 4 || band == 8 || band == 16; }

static int plan_kind(const radsvd_plan *p) {
    if (p->prec == RADSVD_FP32) return 0;
    if (p->prec == RADSVD_BF16) return 1;
    return p->products == 3 ? 2 : 3;
}

int fast_plan_wpc(const radsvd_plan *p) {
    if (p->waves == 4) return 1;
    if (p->waves == 8) return 2;
    return fastk::fast_default_wpc(plan_kind(p), p->Q, p->H8);
}

bool fast_waves_ok(const radsvd_plan *p, int waves) {
    if (waves == 0) return true;
    if ((waves != 4 && waves != 8) || !fast_path_supported(p, RADSVD_OUT_BEST)) return false;
    // the eight-wave kernel's plans have their operands in its layout only
    if (wide_plan(p->prec, p->products, p->herm, p->Q)) return waves == 8;
    const int def = fastk::fast_default_wpc(plan_kind(p), p->Q, p->H8);
    return waves == 4 * def || fastk::fast_alt_q(p->Q);
}

hipError_t launch_pairs_fast(const radsvd_plan *p, int flags, float inv_s2, float *best_score,
                             int32_t *best_m, int32_t *best_t, float *lse_pair, void *X_full, hipStream_t s) {
    fastk::Args a;
    memset(&a, 0, sizeof(a));
    a.Af = p->Af;
    a.Bf = p->Bf;
    a.n_img = p->n_img;
    a.n_tgt = p->n_tgt;
    a.T = p->T;
    a.nTA = p->na_pad / kFastTA;
    a.nTB = p->nb_pad / kFastTB;
    a.band = p->band ? p->band : kDefaultBand;
    a.H8 = p->H8;
    a.nplanes = p->nplanes_a;
    a.flags = flags;
    a.inv_s2 = inv_s2;
    a.best_score = best_score;
    a.best_m = best_m;
    a.best_t = best_t;
    a.lse_pair = lse_pair;
    a.X_full = reinterpret_cast<cx<float> *>(X_full);
    const int nwg = a.nTA * a.nTB;
    if (wide_plan(p->prec, p->products, p->herm, p->Q)) return fastk::launch_wide(a, p->Q, nwg, p->H8, s);
    const int kind = plan_kind(p);
    if (flags & RADSVD_OUT_FULL) {   // the FULL instantiations run at the default occupancy
        switch (kind) {
        case 0: return fastk::launch_fast_full_fp32(a, p->Q, nwg, p->H8, s);
        case 1: return fastk::launch_fast_full_bf16(a, p->Q, nwg, p->H8, s);
        case 2: return fastk::launch_fast_full_bf16x3(a, p->Q, nwg, p->H8, s);
        default: return fastk::launch_fast_full_bf16x3_6(a, p->Q, nwg, p->H8, s);
        }
    }
    if (fast_plan_wpc(p) != fastk::fast_default_wpc(kind, p->Q, p->H8)) {
        switch (kind) {
        case 0: return fastk::launch_fast_alt_fp32(a, p->Q, nwg, p->H8, s);
        case 1: return fastk::launch_fast_alt_bf16(a, p->Q, nwg, p->H8, s);
        case 2: return fastk::launch_fast_alt_bf16x3(a, p->Q, nwg, p->H8, s);
        default: return fastk::launch_fast_alt_bf16x3_6(a, p->Q, nwg, p->H8, s);
        }
    }
    switch (kind) {
    case 0: return fastk::launch_fast_fp32(a, p->Q, nwg, p->H8, s);
    case 1: return fastk::launch_fast_bf16(a, p->Q, nwg, p->H8, s);
    case 2: return fastk::launch_fast_bf16x3(a, p->Q, nwg, p->H8, s);
    default: return fastk::launch_fast_bf16x3_6(a, p->Q, nwg, p->H8, s);
    }
}

}  // namespace radsvd
