/*
 * The C-ABI used from plain C99, with the HIP runtime only (no Python, no
 * torch): a canvas of one root refined once into 8 equal leaves (colour
 * (1, 128/255, 0), optical depth 1 per leaf edge) is uploaded, one view
 * looking down +z through the whole canvas is rendered on a stream this
 * program creates, and every pixel is compared with the closed form of the
 * emission-absorption model: a ray of unit direction d crosses the two
 * leaves along z over 1 / d_z canvas units = 2 / d_z leaf edges, so
 * A = 1 - exp(-2 / d_z) and RGB = c A.  Also checks an error path.
 * Prints "ok" and exits 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "cvx.h"

#define IMG_W 16
#define IMG_H 16
#define TAN_HALF 0.05

static int fails = 0;

static void check(int ok, const char* what) {
  if (!ok) {
    fprintf(stderr, "FAILED: %s\n", what);
    ++fails;
  }
}

int main(void) {
  cvx_node nodes[16];
  cvx_leaf_rgba8_f16 leaves[8];
  for (int i = 0; i < 16; ++i) {
    nodes[i].child = 0u;
    nodes[i].parent = 0u;
  }
  nodes[0].child = 8u; /* the root's 8 children start at node 8 */
  nodes[0].parent = 0xffffffffu;
  for (int i = 0; i < 8; ++i) {
    nodes[8 + i].child = 0x80000000u | (uint32_t)i;
    nodes[8 + i].parent = 0u;
    leaves[i].r = 255;
    leaves[i].g = 128;
    leaves[i].b = 0;
    leaves[i].a = 161;              /* round(255 (1 - e^-1)); not read */
    leaves[i].kappa_f16 = 0x3c00u;  /* 1.0 in IEEE half */
    leaves[i].pad = 0;
  }
  cvx_canvas_desc desc = {{0.0, 0.0, 0.0}, 1.0, 1u, 1u, CVX_LEAF_RGBA8_F16, 0u};

  cvx_view view = {0};
  view.canvas_id = 0;
  view.W = IMG_W;
  view.H = IMG_H;
  view.alpha_stop = 1.0f;
  view.eye[0] = 0.5; view.eye[1] = 0.5; view.eye[2] = -1.0;
  view.right[0] = 1.0;
  view.up[1] = 1.0;
  view.fwd[2] = 1.0;
  view.tan_half_fov_x = TAN_HALF;
  view.tan_half_fov_y = TAN_HALF;
  view.out_offset_px = 0;

  hipStream_t stream;
  if (hipStreamCreate(&stream) != hipSuccess) {
    fprintf(stderr, "no HIP stream\n");
    return 2;
  }
  float* out_dev = NULL;
  if (hipMalloc((void**)&out_dev, sizeof(float) * 4 * IMG_W * IMG_H) != hipSuccess) return 2;

  cvx_ctx* ctx = NULL;
  int rc = cvx_create(&ctx, 0, (void*)stream);
  check(rc == CVX_OK, "cvx_create");
  if (rc != CVX_OK) return 1;
  rc = cvx_upload_pool(ctx, 0, &desc, nodes, 16, leaves, 8);
  check(rc == CVX_OK, "cvx_upload_pool");
  if (rc != CVX_OK) fprintf(stderr, "%s\n", cvx_last_error(ctx));

  cvx_render_opts opts = {0};
  opts.variant = CVX_VARIANT_FP32_REBASED;
  rc = cvx_render(ctx, &view, 1, out_dev, &opts);
  check(rc == CVX_OK, "cvx_render");
  if (rc != CVX_OK) fprintf(stderr, "%s\n", cvx_last_error(ctx));

  float img[4 * IMG_W * IMG_H];
  check(hipStreamSynchronize(stream) == hipSuccess, "hipStreamSynchronize");
  check(hipMemcpy(img, out_dev, sizeof img, hipMemcpyDeviceToHost) == hipSuccess, "hipMemcpy");
  double worst = 0.0;
  for (int y = 0; y < IMG_H; ++y) {
    for (int x = 0; x < IMG_W; ++x) {
      const double u = (2.0 * (x + 0.5) / IMG_W - 1.0) * TAN_HALF;
      const double v = (1.0 - 2.0 * (y + 0.5) / IMG_H) * TAN_HALF;
      const double dz = 1.0 / sqrt(1.0 + u * u + v * v);
      const double a = 1.0 - exp(-2.0 / dz);
      const double want[4] = {a, a * 128.0 / 255.0, 0.0, a};
      for (int c = 0; c < 4; ++c) {
        const double e = fabs((double)img[4 * (y * IMG_W + x) + c] - want[c]);
        worst = e > worst ? e : worst;
      }
    }
  }
  check(worst <= 1e-4, "pixels against the closed form");

  /* an unknown canvas is an error with a message, and changes nothing */
  view.canvas_id = 5;
  rc = cvx_render(ctx, &view, 1, out_dev, &opts);
  check(rc != CVX_OK && cvx_last_error(ctx)[0] != '\0', "render of a missing canvas fails");
  check(cvx_status_str(CVX_ERR_NOT_FOUND)[0] != '\0', "status string");

  check(cvx_free_pool(ctx, 0) == CVX_OK, "cvx_free_pool");
  cvx_destroy(ctx);
  (void)hipFree(out_dev);
  (void)hipStreamDestroy(stream);
  printf("max |rgba - closed form| = %.3g over %d pixels\n", worst, IMG_W * IMG_H);
  if (fails) return 1;
  printf("ok\n");
  return 0;
}
