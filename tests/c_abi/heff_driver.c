/* A plain C user of the library: no Python, no PyTorch in the process, only
 * include/mrdmrg.h, libmrdmrg.so and the HIP runtime.  Test infrastructure.
 *
 *   heff_driver <input> <output>
 *
 * input (little-endian): int32 ly, prec, max_iter; bond a; bond c; MPO site w1; MPO
 * site w2; then L, R and theta as int64 n followed by n complex128 (interleaved) in the
 * canonical layouts; then bond b (between the two orbitals) and the site tensors A
 * (SITE layout of a, b) and B (SITE layout of b, c), each as int64 n + n complex128.
 * bond = int32 nsec, nsec x (int32 n, int32 k), nsec x int32 dim;
 * site = int32 dl, dr, dl x charge, dr x charge, 2 x charge (qs), dl*2*2*dr complex128.
 * output: int64 n, n complex128 (H_eff theta), float64 energy, int32 iterations of
 * lanczos_ground started from theta; int64 n + n complex128 of env_update_left(L, A)
 * and of env_update_right(R, B) (sizes from dm_layout); float64 energy and int32
 * iterations of each of the two instances of a two-plan lanczos_ground_batched started
 * from theta.  Exit status 0 on success; on a library error the message of
 * dm_last_error() goes to stderr and the status is 2. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mrdmrg.h"

static FILE* in;

static void rd(void* p, size_t n) {
  if (fread(p, 1, n, in) != n) {
    fprintf(stderr, "short input\n");
    exit(3);
  }
}
static int32_t rd_i32(void) {
  int32_t v;
  rd(&v, 4);
  return v;
}
static int64_t rd_i64(void) {
  int64_t v;
  rd(&v, 8);
  return v;
}
static void* rd_array(size_t n) {
  void* p = malloc(n > 0 ? n : 1);
  if (!p) exit(3);
  rd(p, n);
  return p;
}

static void read_bond(dm_bond* b) {
  b->nsec = rd_i32();
  b->q = (const dm_charge*)rd_array((size_t)b->nsec * sizeof(dm_charge));
  b->dim = (const int32_t*)rd_array((size_t)b->nsec * 4);
}

static void read_site(dm_mpo_site* w) {
  w->dl = rd_i32();
  w->dr = rd_i32();
  w->ql = (const dm_charge*)rd_array((size_t)w->dl * sizeof(dm_charge));
  w->qr = (const dm_charge*)rd_array((size_t)w->dr * sizeof(dm_charge));
  rd(w->qs, sizeof(w->qs));
  w->w = (const double*)rd_array((size_t)w->dl * 4 * w->dr * 16);
}

/* n complex128 from the input into a new device buffer */
static void* read_device(int64_t* n) {
  *n = rd_i64();
  void* h = rd_array((size_t)*n * 16);
  void* d = NULL;
  if (hipMalloc(&d, (size_t)(*n > 0 ? *n : 1) * 16) != hipSuccess ||
      hipMemcpy(d, h, (size_t)*n * 16, hipMemcpyHostToDevice) != hipSuccess) {
    fprintf(stderr, "device copy failed\n");
    exit(3);
  }
  free(h);
  return d;
}

#define CHECK(call)                                              \
  do {                                                           \
    const int rc_ = (call);                                      \
    if (rc_ != DM_OK) {                                          \
      fprintf(stderr, "%s: %d %s\n", #call, rc_, dm_last_error()); \
      return 2;                                                  \
    }                                                            \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: heff_driver <input> <output>\n");
    return 1;
  }
  in = fopen(argv[1], "rb");
  if (!in) return 3;
  const int32_t ly = rd_i32(), prec = rd_i32(), max_iter = rd_i32();
  dm_bond a, c;
  dm_mpo_site w1, w2;
  read_bond(&a);
  read_bond(&c);
  read_site(&w1);
  read_site(&w2);
  int64_t nl, nr, nt;
  void* L = read_device(&nl);
  void* R = read_device(&nr);
  void* th = read_device(&nt);
  dm_bond b;
  read_bond(&b);
  int64_t na, nb;
  void* A = read_device(&na);
  void* B = read_device(&nb);
  fclose(in);
  /* a second copy of theta: the Lanczos calls overwrite their start vector */
  void* th2 = NULL;
  void* th3 = NULL;
  if (hipMalloc(&th2, (size_t)(nt > 0 ? nt : 1) * 16) != hipSuccess ||
      hipMalloc(&th3, (size_t)(nt > 0 ? nt : 1) * 16) != hipSuccess ||
      hipMemcpy(th2, th, (size_t)nt * 16, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(th3, th, (size_t)nt * 16, hipMemcpyDeviceToDevice) != hipSuccess)
    return 3;

  dm_heff_plan* plan = NULL;
  CHECK(dm_heff_plan_create(ly, &a, &c, &w1, &w2, L, R, prec, NULL, &plan));
  int64_t n = 0;
  double flops[3];
  CHECK(dm_heff_info(plan, &n, flops));
  if (n != nt) {
    fprintf(stderr, "theta has %lld elements, the plan %lld\n", (long long)nt, (long long)n);
    return 2;
  }
  void* y = NULL;
  if (hipMalloc(&y, (size_t)(n > 0 ? n : 1) * 16) != hipSuccess) return 3;
  CHECK(heff_apply(plan, th, y, NULL));
  double* hy = (double*)malloc((size_t)(n > 0 ? n : 1) * 16);
  if (hipMemcpy(hy, y, (size_t)n * 16, hipMemcpyDeviceToHost) != hipSuccess) return 3;
  double energy = 0.0;
  int32_t iters = 0;
  CHECK(lanczos_ground(plan, th, max_iter, 1e-14, &energy, &iters, NULL));

  /* environment updates through the window: output sizes from the layout query */
  dm_layout_desc dl_desc;
  memset(&dl_desc, 0, sizeof(dl_desc));
  dl_desc.kind = DM_LAYOUT_ENV_L;
  dl_desc.ly = ly;
  dl_desc.x = &b;
  dl_desc.nw = w1.dr;
  dl_desc.qw = w1.qr;
  int64_t nblk = 0, nlo = 0, nro = 0;
  CHECK(dm_layout(&dl_desc, &nblk, &nlo, NULL));
  dl_desc.kind = DM_LAYOUT_ENV_R;
  dl_desc.nw = w2.dl;
  dl_desc.qw = w2.ql;
  CHECK(dm_layout(&dl_desc, &nblk, &nro, NULL));
  void *Lo = NULL, *Ro = NULL;
  if (hipMalloc(&Lo, (size_t)(nlo > 0 ? nlo : 1) * 16) != hipSuccess ||
      hipMalloc(&Ro, (size_t)(nro > 0 ? nro : 1) * 16) != hipSuccess)
    return 3;
  CHECK(env_update_left(ly, &a, &b, &w1, L, A, Lo, prec, NULL));
  CHECK(env_update_right(ly, &b, &c, &w2, R, B, Ro, prec, NULL));
  double* hl = (double*)malloc((size_t)(nlo > 0 ? nlo : 1) * 16);
  double* hr = (double*)malloc((size_t)(nro > 0 ? nro : 1) * 16);
  if (hipMemcpy(hl, Lo, (size_t)nlo * 16, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hr, Ro, (size_t)nro * 16, hipMemcpyDeviceToHost) != hipSuccess)
    return 3;

  /* two plans of the same window in one batch */
  dm_heff_plan* plan2 = NULL;
  CHECK(dm_heff_plan_create(ly, &a, &c, &w1, &w2, L, R, prec, NULL, &plan2));
  dm_heff_plan* pair[2];
  pair[0] = plan;
  pair[1] = plan2;
  dm_batch* batch = NULL;
  CHECK(dm_batch_create(2, pair, NULL, &batch));
  void* thetas[2];
  thetas[0] = th2;
  thetas[1] = th3;
  double eb[2];
  int32_t kb[2];
  CHECK(lanczos_ground_batched(batch, thetas, max_iter, 1e-14, eb, kb, NULL, NULL));
  dm_batch_destroy(batch);
  dm_heff_plan_destroy(plan2);
  dm_heff_plan_destroy(plan);

  FILE* out = fopen(argv[2], "wb");
  if (!out) return 3;
  fwrite(&n, 8, 1, out);
  fwrite(hy, 16, (size_t)n, out);
  fwrite(&energy, 8, 1, out);
  fwrite(&iters, 4, 1, out);
  fwrite(&nlo, 8, 1, out);
  fwrite(hl, 16, (size_t)nlo, out);
  fwrite(&nro, 8, 1, out);
  fwrite(hr, 16, (size_t)nro, out);
  fwrite(eb, 8, 2, out);
  fwrite(kb, 4, 2, out);
  fclose(out);
  void* bufs[] = {L, R, th, th2, th3, y, A, B, Lo, Ro};
  for (size_t i = 0; i < sizeof(bufs) / sizeof(bufs[0]); ++i) (void)hipFree(bufs[i]);
  free(hy);
  free(hl);
  free(hr);
  return 0;
}
