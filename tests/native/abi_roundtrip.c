/* A plain C program using only the C ABI (include/lc.h) and the HIP runtime:
 * compress, parse the header, decompress, decompress a range, access and
 * lower_bound, each checked against the keys on the host.  Exit status 0
 * on success; prints the first mismatch otherwise. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lc.h"

#define CHECK(x)                                                          \
    do {                                                                  \
        if (!(x)) {                                                       \
            fprintf(stderr, "FAIL line %d: %s\n", __LINE__, #x);          \
            return 1;                                                     \
        }                                                                 \
    } while (0)

int main(void)
{
    const uint64_t n = 300000;
    uint64_t* keys = (uint64_t*)malloc(n * 8);
    uint64_t x = 77, state = 12345;
    for (uint64_t i = 0; i < n; i++) {
        state = state * 6364136223846793005ull + 1442695040888963407ull;
        x += 1 + (state >> 54);  /* gaps 1 .. 1024 */
        keys[i] = x;
    }
    lc_params p;
    memset(&p, 0, sizeof p);
    p.key_bytes = 8;
    p.log2_block = LC_DEFAULT_LOG2_BLOCK;
    p.frac_bits = LC_DEFAULT_FRAC_BITS;
    p.eps = 63;
    uint64_t blob_max = 0, ws_bytes = 0;
    CHECK(lc_compress_bound(n, &p, &blob_max, &ws_bytes) == LC_OK);

    void *d_keys, *d_blob, *d_ws, *d_out, *d_idx, *d_pos;
    uint64_t* d_bytes;
    uint32_t* d_flags;
    const uint64_t m = 5000;
    CHECK(hipMalloc(&d_keys, n * 8) == hipSuccess);
    CHECK(hipMalloc(&d_blob, blob_max) == hipSuccess);
    CHECK(hipMalloc(&d_ws, ws_bytes) == hipSuccess);
    CHECK(hipMalloc(&d_out, n * 8) == hipSuccess);
    CHECK(hipMalloc(&d_idx, m * 8) == hipSuccess);
    CHECK(hipMalloc(&d_pos, m * 8) == hipSuccess);
    CHECK(hipMalloc((void**)&d_bytes, 8) == hipSuccess);
    CHECK(hipMalloc((void**)&d_flags, 4) == hipSuccess);
    CHECK(hipMemcpy(d_keys, keys, n * 8, hipMemcpyHostToDevice) == hipSuccess);
    CHECK(hipMemset(d_flags, 0, 4) == hipSuccess);

    CHECK(lc_compress(d_keys, n, &p, d_blob, blob_max, d_ws, ws_bytes, d_bytes, d_flags, NULL) == LC_OK);
    uint64_t blob_bytes = 0;
    uint32_t flags = 1;
    CHECK(hipMemcpy(&blob_bytes, d_bytes, 8, hipMemcpyDeviceToHost) == hipSuccess);
    CHECK(hipMemcpy(&flags, d_flags, 4, hipMemcpyDeviceToHost) == hipSuccess);
    CHECK(flags == 0);
    unsigned char header[LC_HEADER_BYTES];
    CHECK(hipMemcpy(header, d_blob, LC_HEADER_BYTES, hipMemcpyDeviceToHost) == hipSuccess);
    lc_blob_info info;
    CHECK(lc_info(header, LC_HEADER_BYTES, &info) == LC_OK);
    CHECK(info.n == n && info.blob_bytes == blob_bytes && info.eps == 63);

    uint64_t* back = (uint64_t*)malloc(n * 8);
    CHECK(lc_decompress(d_blob, &info, d_out, NULL) == LC_OK);
    CHECK(hipMemcpy(back, d_out, n * 8, hipMemcpyDeviceToHost) == hipSuccess);
    CHECK(memcmp(back, keys, n * 8) == 0);

    const uint64_t b = 12345, e = 200001;
    CHECK(lc_decompress_range(d_blob, &info, b, e, d_out, NULL) == LC_OK);
    CHECK(hipMemcpy(back, d_out, (e - b) * 8, hipMemcpyDeviceToHost) == hipSuccess);
    CHECK(memcmp(back, keys + b, (e - b) * 8) == 0);

    uint64_t* idx = (uint64_t*)malloc(m * 8);
    uint64_t* q = (uint64_t*)malloc(m * 8);
    for (uint64_t i = 0; i < m; i++) {
        state = state * 6364136223846793005ull + 1442695040888963407ull;
        idx[i] = (state >> 11) % n;
        q[i] = keys[idx[i]] + (i % 3) - 1; /* key - 1, key, key + 1 */
    }
    CHECK(hipMemcpy(d_idx, idx, m * 8, hipMemcpyHostToDevice) == hipSuccess);
    CHECK(lc_access(d_blob, &info, (const uint64_t*)d_idx, m, d_out, d_flags, NULL) == LC_OK);
    CHECK(hipMemcpy(back, d_out, m * 8, hipMemcpyDeviceToHost) == hipSuccess);
    for (uint64_t i = 0; i < m; i++) CHECK(back[i] == keys[idx[i]]);

    CHECK(hipMemcpy(d_idx, q, m * 8, hipMemcpyHostToDevice) == hipSuccess);
    CHECK(lc_lower_bound(d_blob, &info, d_idx, m, (uint64_t*)d_pos, NULL) == LC_OK);
    CHECK(hipMemcpy(back, d_pos, m * 8, hipMemcpyDeviceToHost) == hipSuccess);
    for (uint64_t i = 0; i < m; i++) {
        uint64_t lo = 0, hi = n; /* first k with keys[k] >= q[i] */
        while (lo < hi) {
            const uint64_t mid = (lo + hi) / 2;
            if (keys[mid] >= q[i]) hi = mid;
            else lo = mid + 1;
        }
        CHECK(back[i] == lo);
    }
    printf("abi roundtrip ok: n=%lu blob=%lu bytes\n", (unsigned long)n, (unsigned long)blob_bytes);
    return 0;
}
