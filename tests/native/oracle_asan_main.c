/*
 * Test driver that links the FP64 oracle's C source into a standalone
 * program, so that it can be built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only).  It reads one binary request,
 * runs the scan image, meshification, both coverage modes of the brute-force
 * renderer and the contract's sub-triangle listing, and writes every result
 * so that the caller can compare it with the shared-library build.
 *
 * Request (native byte order):
 *   int32 H, W; camera {f32 fx, fy, cx, cy; i32 width, height; f32 z_near, z_far};
 *   f64 T_map[12]; f64 T_query[12]; i32 stride, radius; f32 z_min, z_max, max_edge;
 *   f32 depth[H * W]
 * Reply: d_s f32[H*W], c_s u8[H*W], i64 nv, i64 nt, xyz f32[nv*3], tri i32[nt*3],
 *   cls u8[nt], then for mode 0 and 1: z f64[n], id i32[n], z2 f64[n], ncov i32[n],
 *   nrm f64[3n], i64 dropped (n = width * height of the camera); then i64 nsub and
 *   the sub-triangle records i64[7 * nsub].
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    float fx, fy, cx, cy;
    int32_t width, height;
    float z_near, z_far;
} drv_camera;

void or_scan_image(const float* depth, int32_t H, int32_t W, float z_min, float z_max, float* d_out,
                   uint8_t* c_out);
int64_t or_meshify(const float* depth, int32_t H, int32_t W, const drv_camera* cam, const double* T, int32_t s,
                   int32_t R, float z_min, float z_max, float max_edge, float* xyz, int32_t* tri, uint8_t* cls,
                   int64_t cap_t, int64_t* n_v_out);
int64_t or_render(const float* xyz, int64_t nv, const int32_t* tri, int64_t nt, const double* T,
                  const drv_camera* cam, int32_t mode, const int64_t* pix, int64_t npix, double* z_out,
                  int32_t* id_out, double* z2_out, int32_t* ncov_out, double* nrm_out);
int64_t or_contract_subs(const float* xyz, const int32_t* tri, int64_t nt, const double* T, const drv_camera* cam,
                         int64_t* out, int64_t cap);

static void must_read(FILE* f, void* p, size_t n) {
    if (fread(p, 1, n, f) != n) { fprintf(stderr, "short request\n"); exit(2); }
}

static void put(FILE* f, const void* p, size_t n) {
    if (n && fwrite(p, 1, n, f) != n) { fprintf(stderr, "short write\n"); exit(3); }
}

static void* alloc(size_t n) {
    void* p = malloc(n ? n : 1);
    if (!p) { fprintf(stderr, "out of memory\n"); exit(4); }
    return p;
}

int main(int argc, char** argv) {
    if (argc != 3) { fprintf(stderr, "usage: %s request reply\n", argv[0]); return 1; }
    FILE* in = fopen(argv[1], "rb");
    if (!in) return 1;
    int32_t H, W, s, R;
    drv_camera cam;
    double Tm[12], Tq[12];
    float z_min, z_max, max_edge;
    must_read(in, &H, 4); must_read(in, &W, 4); must_read(in, &cam, sizeof cam);
    must_read(in, Tm, sizeof Tm); must_read(in, Tq, sizeof Tq);
    must_read(in, &s, 4); must_read(in, &R, 4);
    must_read(in, &z_min, 4); must_read(in, &z_max, 4); must_read(in, &max_edge, 4);
    const size_t npx = (size_t)H * (size_t)W;
    float* depth = alloc(4 * npx);
    must_read(in, depth, 4 * npx);
    fclose(in);

    FILE* out = fopen(argv[2], "wb");
    if (!out) return 1;
    float* d = alloc(4 * npx);
    uint8_t* c = alloc(npx);
    or_scan_image(depth, H, W, z_min, z_max, d, c);
    put(out, d, 4 * npx); put(out, c, npx);

    const int64_t gh = (H + s - 1) / s, gw = (W + s - 1) / s;
    const int64_t cap_t = 2 * (gh > 1 ? gh - 1 : 0) * (gw > 1 ? gw - 1 : 0);
    float* xyz = alloc(sizeof(float) * 3 * (size_t)(gh * gw));
    int32_t* tri = alloc(sizeof(int32_t) * 3 * (size_t)cap_t);
    uint8_t* cls = alloc((size_t)cap_t);
    int64_t nv = 0;
    const int64_t nt = or_meshify(depth, H, W, &cam, Tm, s, R, z_min, z_max, max_edge, xyz, tri, cls, cap_t, &nv);
    if (nt < 0) return 5;
    put(out, &nv, 8); put(out, &nt, 8);
    put(out, xyz, sizeof(float) * 3 * (size_t)nv); put(out, tri, sizeof(int32_t) * 3 * (size_t)nt);
    put(out, cls, (size_t)nt);

    const int64_t n = (int64_t)cam.width * cam.height;
    double* z = alloc(8 * (size_t)n);
    double* z2 = alloc(8 * (size_t)n);
    double* nrm = alloc(24 * (size_t)n);
    int32_t* id = alloc(4 * (size_t)n);
    int32_t* ncov = alloc(4 * (size_t)n);
    for (int32_t mode = 0; mode < 2; ++mode) {
        const int64_t dropped = or_render(xyz, nv, tri, nt, Tq, &cam, mode, NULL, n, z, id, z2, ncov, nrm);
        put(out, z, 8 * (size_t)n); put(out, id, 4 * (size_t)n); put(out, z2, 8 * (size_t)n);
        put(out, ncov, 4 * (size_t)n); put(out, nrm, 24 * (size_t)n); put(out, &dropped, 8);
    }
    const int64_t cap = 2 * nt + 1;
    int64_t* subs = alloc(sizeof(int64_t) * 7 * (size_t)cap);
    const int64_t nsub = or_contract_subs(xyz, tri, nt, Tq, &cam, subs, cap);
    put(out, &nsub, 8); put(out, subs, sizeof(int64_t) * 7 * (size_t)(nsub < cap ? nsub : cap));
    fclose(out);
    free(depth); free(d); free(c); free(xyz); free(tri); free(cls);
    free(z); free(z2); free(nrm); free(id); free(ncov); free(subs);
    return 0;
}
