/* Sanitizer driver for the host side of the C ABI (test infrastructure):
 * code handles from CSR and QC tables, their info and row levels, option
 * defaults, workspace sizing, the argument checks of every entry point that
 * fail before any device work, and handle release, under AddressSanitizer and
 * UndefinedBehaviorSanitizer, on a machine without a GPU.  Exit status 0 when
 * every call returns what include/cbp.h documents. */
#include <stdio.h>
#include <stdlib.h>

#include "cbp.h"

static int bad = 0;
#define EXPECT(cond)                                                    \
    do {                                                                \
        if (!(cond)) {                                                  \
            fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #cond, cbp_last_error()); \
            bad = 1;                                                    \
        }                                                               \
    } while (0)

int main(void) {
    /* 4 x 8 base, Z = 16: dual-diagonal parity part */
    int32_t sh[4 * 8];
    for (int i = 0; i < 32; ++i) sh[i] = -1;
    for (int r = 0; r < 4; ++r)
        for (int b = 0; b < 4; ++b) sh[r * 8 + b] = (3 * r + 5 * b + 1) % 16;
    for (int r = 0; r < 4; ++r) {
        sh[r * 8 + 4 + r] = 0;
        if (r > 0) sh[r * 8 + 4 + r - 1] = 0;
    }
    sh[0 * 8 + 4 + 3] = 1;  /* weight-1 shift closing the staircase */
    cbp_code_t *q = NULL;
    EXPECT(cbp_code_from_qc(4, 8, 16, sh, &q) == CBP_OK && q);
    int32_t M = 0, N = 0, Z = 0, kern = 0, nlev = 0;
    int64_t E = 0;
    EXPECT(cbp_code_info(q, &M, &N, &E, &Z, &kern) == CBP_OK && M == 64 && N == 128 && Z == 16);
    EXPECT(cbp_code_levels(q, &nlev, NULL, NULL) == CBP_OK && nlev > 0);
    int32_t *lp = malloc(sizeof(int32_t) * (nlev + 1)), *rows = malloc(sizeof(int32_t) * M);
    EXPECT(cbp_code_levels(q, &nlev, lp, rows) == CBP_OK && lp[nlev] == M);
    cbp_opts_t o;
    cbp_opts_default(&o);
    EXPECT(o.lmax == 20.0f && o.alpha == 0.75f);
    size_t ws = 0;
    for (int d = 0; d <= 4; ++d) {
        o.kernel = d >= 3 ? CBP_KERNEL_SPARSE : CBP_KERNEL_AUTO;
        EXPECT(cbp_workspace_size(q, d, 1000, &o, &ws) == CBP_OK && ws > 0);
    }
    cbp_opts_default(&o);
    EXPECT(cbp_workspace_size(q, 9, 10, &o, &ws) == CBP_EINVAL);
    /* CSR: the lifted code's rows, and malformed tables */
    int32_t rp[4] = {0, 3, 6, 9}, ci[9] = {0, 2, 4, 1, 3, 5, 0, 3, 5};
    cbp_code_t *c = NULL;
    EXPECT(cbp_code_from_csr(3, 6, rp, ci, &c) == CBP_OK && c);
    int32_t ci_bad[9] = {0, 4, 2, 1, 3, 5, 0, 3, 5};
    cbp_code_t *c2 = NULL;
    EXPECT(cbp_code_from_csr(3, 6, rp, ci_bad, &c2) == CBP_EINVAL && !c2);
    int32_t ci_oor[9] = {0, 2, 9, 1, 3, 5, 0, 3, 5};
    EXPECT(cbp_code_from_csr(3, 6, rp, ci_oor, &c2) == CBP_EINVAL);
    EXPECT(cbp_code_from_csr(0, 6, rp, ci, &c2) == CBP_EINVAL);
    int32_t sh_bad[4 * 8];
    for (int i = 0; i < 32; ++i) sh_bad[i] = sh[i];
    sh_bad[3] = 16;
    EXPECT(cbp_code_from_qc(4, 8, 16, sh_bad, &c2) == CBP_EINVAL);
    EXPECT(cbp_code_from_qc(4, 8, 16, NULL, &c2) == CBP_EINVAL);
    /* decoders: empty batches succeed, bad arguments fail, all before device work */
    EXPECT(cbp_decode(q, NULL, NULL, NULL, 10, 0, NULL, NULL) == CBP_OK);
    EXPECT(lbp_nms_decode(q, NULL, NULL, NULL, 10, 0, NULL, NULL) == CBP_OK);
    EXPECT(cbp_decode(q, NULL, NULL, NULL, 10, 5, NULL, NULL) == CBP_EINVAL);
    EXPECT(fbp_nms_decode(q, NULL, NULL, NULL, -1, 5, NULL, NULL) == CBP_EINVAL);
    EXPECT(cbp_decode(NULL, NULL, NULL, NULL, 10, 5, NULL, NULL) == CBP_EINVAL);
    EXPECT(cbp_decode_static(q, 7, NULL, NULL, NULL, 1, 1, NULL, NULL) == CBP_EINVAL);
    EXPECT(cbp_decode_static(q, 0, NULL, NULL, NULL, 1, 0, NULL, NULL) == CBP_OK);
    EXPECT(cbp_syndrome(q, NULL, NULL, 0, NULL) == CBP_OK);
    size_t uws = 0;
    EXPECT(cbp_unrolled_workspace_size(q, 10, 100, &uws) == CBP_OK && uws > 0);
    EXPECT(cbp_unrolled_workspace_size(q, 0, 100, &uws) == CBP_EINVAL);
    const cbp_code_t *codes[2] = {q, q};
    cbp_mix_t *mix = NULL;
    EXPECT(cbp_mix_create(codes, 2, &mix) == CBP_OK && mix);
    cbp_mix_schedule_t sc;
    EXPECT(cbp_mix_get_schedule(mix, &sc) == CBP_OK && sc.lanes % 16 == 0);
    {   /* sized on the current device: no device here is CBP_EHIP */
        const int rc = cbp_mix_workspace_size(mix, 0, 1000, NULL, &ws);
        EXPECT(rc == CBP_OK || rc == CBP_EHIP);
    }
    cbp_mix_t *mix2 = NULL;
    EXPECT(cbp_mix_create(codes, 0, &mix2) == CBP_EINVAL && !mix2);
    cbp_mix_free(mix);
    EXPECT(cbp_strerror(CBP_EUNSUPPORTED) != NULL && cbp_version() >= 100);
    free(lp);
    free(rows);
    cbp_code_free(c);
    cbp_code_free(q);
    printf("abi host driver: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
