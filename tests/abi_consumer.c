/* A plain C99 consumer of the library's C ABI (include/ks.h): reads a raw
 * volume from a file, runs ks_detect on it and prints one line per region.
 *
 *   abi_consumer volume.raw dtype X Y Z bins spacing s_min s_max method max_iter capacity
 *
 * dtype: 0 u8, 1 u16, 2 i16.  Output: "n_found N" then, per written region,
 * "x y z scale seed saliency entropy pdf_change" (floats as %.9g).  Exit status 0
 * on KS_OK, 1 on a library error (its name on stderr), 2 on bad arguments. */
#include <stdio.h>
#include <stdlib.h>

#include "ks.h"

int main(int argc, char** argv) {
    if (argc != 13) {
        fprintf(stderr, "usage: %s volume.raw dtype X Y Z bins spacing s_min s_max method max_iter capacity\n",
                argv[0]);
        return 2;
    }
    const int dtype = atoi(argv[2]);
    const int32_t dims[3] = {atoi(argv[3]), atoi(argv[4]), atoi(argv[5])};
    const int32_t bins = atoi(argv[6]), spacing = atoi(argv[7]);
    const int32_t scales[2] = {atoi(argv[8]), atoi(argv[9])};
    const int32_t method = atoi(argv[10]), max_iter = atoi(argv[11]), capacity = atoi(argv[12]);
    if (dtype < 0 || dtype > 2 || dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || capacity < 1) return 2;
    const size_t n = (size_t)dims[0] * dims[1] * dims[2] * (dtype == 0 ? 1u : 2u);
    void* vol = malloc(n);
    ks_region* out = (ks_region*)malloc(sizeof(ks_region) * (size_t)capacity);
    FILE* f = fopen(argv[1], "rb");
    if (!vol || !out || !f || fread(vol, 1, n, f) != n) return 2;
    fclose(f);
    int32_t n_found = 0;
    const ks_status st = ks_detect(vol, (ks_dtype)dtype, dims, bins, spacing, scales, (ks_method)method, max_iter,
                                   out, capacity, &n_found);
    if (st != KS_OK) {
        fprintf(stderr, "ks_detect: %s\n", ks_status_str(st));
        return 1;
    }
    printf("n_found %d\n", n_found);
    const int w = n_found < capacity ? n_found : capacity;
    for (int i = 0; i < w; ++i)
        printf("%d %d %d %d %d %.9g %.9g %.9g\n", out[i].x, out[i].y, out[i].z, out[i].scale, out[i].seed,
               out[i].saliency, out[i].entropy, out[i].pdf_change);
    free(vol);
    free(out);
    return 0;
}
