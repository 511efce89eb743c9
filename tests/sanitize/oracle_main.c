/* Drives the CPU oracle (oracle/lt_oracle.c) on random label images for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer: every call must return 0,
 * and the results must satisfy D >= 0, D = 0 exactly on background, LT >= D on
 * objects and LT = 0 on background.  Prints "oracle sanitizer run ok" at the end. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_edt(const int64_t* lab, int ndim, const int64_t* shape, const int64_t* w, int64_t* D);
int oracle_lt(const int64_t* D, int ndim, const int64_t* shape, const int64_t* w, int64_t* LT, int64_t* work);

static uint64_t state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64(void) {                 /* splitmix64 */
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

int main(void) {
    const int64_t shapes[][3] = {{1, 1, 1}, {1, 7, 9}, {5, 6, 7}, {9, 4, 13}, {3, 17, 2}, {12, 12, 12}};
    const int64_t weights[][3] = {{1, 1, 1}, {4, 1, 1}, {2, 3, 5}, {1, 9, 1}};
    int cases = 0;
    for (int s = 0; s < 6; ++s)
        for (int nd = 2; nd <= 3; ++nd)
            for (int wi = 0; wi < 4; ++wi) {
                const int64_t* sh = nd == 3 ? shapes[s] : shapes[s] + 1;
                const int64_t* w = nd == 3 ? weights[wi] : weights[wi] + 1;
                int64_t n = 1;
                for (int a = 0; a < nd; ++a) n *= sh[a];
                int64_t* lab = malloc((size_t)n * sizeof(int64_t));
                int64_t* D = malloc((size_t)n * sizeof(int64_t));
                int64_t* LT = malloc((size_t)n * sizeof(int64_t));
                for (int64_t i = 0; i < n; ++i) {
                    /* blocks of 3 along x with relabelling noise and background */
                    const uint64_t r = next_u64();
                    lab[i] = (r % 5 == 0) ? 0 : (int64_t)((i / 3) % 4) + 1;
                }
                int64_t work = 0;
                if (oracle_edt(lab, nd, sh, wi ? w : NULL, D) || oracle_lt(D, nd, sh, wi ? w : NULL, LT, &work)) {
                    printf("oracle call failed\n");
                    return 1;
                }
                for (int64_t i = 0; i < n; ++i) {
                    const int bad = D[i] < 0 || (lab[i] == 0) != (D[i] == 0) || (lab[i] != 0 && LT[i] < D[i]) ||
                                    (lab[i] == 0 && LT[i] != 0);
                    if (bad) {
                        printf("invariant broken at %lld\n", (long long)i);
                        return 1;
                    }
                }
                free(lab);
                free(D);
                free(LT);
                ++cases;
            }
    if (oracle_edt(NULL, 3, shapes[2], NULL, NULL) != -1) return 1;
    printf("oracle sanitizer run ok (%d cases)\n", cases);
    return 0;
}
