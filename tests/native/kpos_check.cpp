// Host driver of tests/test_kpos_cpu.py: the incremental K position of the
// implicit-GEMM kernels (struct KPos, extracted from conv.hip into kpos.h by
// the test) against the direct decoding of the packed K order.

#include <cstdio>
#include <cstdlib>
#include <initializer_list>
#include "kpos.h"

static int esize(int dt) { return dt == 0 ? 4 : dt == 1 ? 2 : 1; }
int main() {
    long checked = 0;
    int cins[] = {4, 8, 16, 24, 32, 40, 48, 64, 96, 128, 192, 256, 512, 1024};
    for (int dt = 0; dt < 3; ++dt)
    for (int spr : {8, 4})
    for (int cin_p : cins)
    for (int R : {1, 2, 3, 4})
    for (int S : {1, 2, 3}) {
        const int ES = esize(dt), SEG = 16 / ES, BKE = spr * SEG, RS = R * S;
        if ((cin_p * ES) % 16) continue;
        const bool blk = RS > 1 && cin_p * ES > 128 && (cin_p * ES) % 128 == 0;
        const int cbsh = blk ? 7 - (ES >> 1) : -1;
        if (blk && ((1 << cbsh) % BKE)) continue;
        const int K = RS * cin_p, k_pad = (K + BKE - 1) / BKE * BKE + 2 * BKE;  // two padding tiles past K
        const int nkt = k_pad / BKE;
        for (int kt0 = 0; kt0 < nkt; kt0 += 3)
        for (int sc = 0; sc < spr; ++sc) {
            KPos kp;
            kp.init(kt0 * BKE + sc * SEG, cin_p, RS, S, cbsh);
            for (int kt = kt0; kt < nkt; ++kt) {
                const int k0 = kt * BKE + sc * SEG;
                int tap, c0;
                if (cbsh < 0) { tap = k0 / cin_p; c0 = k0 - tap * cin_p; }
                else { const int b = k0 >> cbsh, cb = b / RS; tap = b - cb * RS; c0 = (cb << cbsh) + (k0 & ((1 << cbsh) - 1)); }
                const int r = tap / S, s = tap - r * S;
                const bool kv = tap < RS && c0 < cin_p;
                const bool kv2 = kp.r < R && kp.c0 < cin_p;
                if (kv != kv2 || (kv && (kp.r != r || kp.s != s || kp.c0 != c0))) {
                    printf("MISMATCH dt %d spr %d cin %d R %d S %d kt0 %d kt %d sc %d: direct r%d s%d c%d kv%d incr r%d s%d c%d kv%d\n",
                           dt, spr, cin_p, R, S, kt0, kt, sc, r, s, c0, kv, kp.r, kp.s, kp.c0, kv2);
                    return 1;
                }
                ++checked;
                kp.next(BKE, cin_p, R, S, cbsh);
            }
        }
    }
    printf("ok %ld positions\n", checked);
    return 0;
}
