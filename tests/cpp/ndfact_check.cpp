// CPU check of the host factorisation data (test infrastructure only): reads a
// CSR matrix P and a block of right-hand sides, factorises P with nd_factor,
// then runs the two level-scheduled block solves on the CPU with the stored
// inverted-block data, exactly in the order the GPU kernels use, and writes
// Z = P^{-1} R.  The Python test compares Z with a SciPy sparse solve.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "ndfact.h"

int main(int argc, char** argv) {
  if (argc < 4) { fprintf(stderr, "usage: in.bin out.bin leaf\n"); return 2; }
  FILE* f = fopen(argv[1], "rb");
  int64_t n, nnz, k;
  if (fread(&n, 8, 1, f) != 1 || fread(&nnz, 8, 1, f) != 1) return 3;
  lrc::CsrHost P;
  P.n = n;
  P.rowptr.resize(n + 1);
  P.col.resize(nnz);
  P.val.resize(nnz);
  if (fread(P.rowptr.data(), 8, n + 1, f) != size_t(n + 1)) return 3;
  if (fread(P.col.data(), 4, nnz, f) != size_t(nnz)) return 3;
  if (fread(P.val.data(), 8, nnz, f) != size_t(nnz)) return 3;
  if (fread(&k, 8, 1, f) != 1) return 3;
  std::vector<double> R(n * k);
  if (fread(R.data(), 8, n * k, f) != size_t(n * k)) return 3;
  fclose(f);
  lrc::SupernodalFactor F;
  std::string err;
  int rc = lrc::nd_factor(P, atoi(argv[3]), 0, &F, &err);
  if (rc != 0) { printf("{\"rc\": %d, \"err\": \"%s\"}\n", rc, err.c_str()); return 0; }
  const int S = F.nsn;
  std::vector<double> y(n * k, 0.0), x(n * k, 0.0), cb(F.cb_off[S] * k, 0.0), Z(n * k, 0.0);
  // forward, by height
  for (int h = 0; h < F.nlev_fwd; ++h)
    for (int s = 0; s < S; ++s) {
      if (F.height[s] != h) continue;
      const int64_t ns = F.ns[s], nb = F.nb[s], fr = ns + nb, j0 = F.j0[s];
      std::vector<double> front(fr * k, 0.0);
      for (int64_t p = 0; p < fr; ++p) {
        for (int64_t c = 0; c < k; ++c) {
          double v = (p < ns) ? R[int64_t(F.perm[j0 + p]) * k + c] : 0.0;
          for (int64_t e = F.asm_ptr[F.front_off[s] + p]; e < F.asm_ptr[F.front_off[s] + p + 1]; ++e)
            v += cb[F.asm_src[e] * k + c];
          front[p * k + c] = v;
        }
      }
      const double* fw = F.fw.data() + F.fw_off[s];
      for (int64_t r = 0; r < fr; ++r)
        for (int64_t c = 0; c < k; ++c) {
          double acc = (r >= ns) ? front[r * k + c] : 0.0;
          for (int64_t i = 0; i < ns; ++i) acc += fw[i * fr + r] * front[i * k + c];
          if (r < ns) y[(j0 + r) * k + c] = acc;
          else cb[(F.cb_off[s] + r - ns) * k + c] = acc;
        }
    }
  // backward, by depth
  for (int dpt = 0; dpt < F.nlev_bwd; ++dpt)
    for (int s = 0; s < S; ++s) {
      if (F.depth[s] != dpt) continue;
      const int64_t ns = F.ns[s], nb = F.nb[s], fr = ns + nb, j0 = F.j0[s];
      const double* bw = F.bw.data() + F.bw_off[s];
      const int32_t* B = F.bnd.data() + F.bnd_off[s];
      for (int64_t r = 0; r < ns; ++r)
        for (int64_t c = 0; c < k; ++c) {
          double acc = 0.0;
          for (int64_t i = 0; i < fr; ++i) {
            double in = (i < ns) ? y[(j0 + i) * k + c] : x[int64_t(B[i - ns]) * k + c];
            acc += bw[i * ns + r] * in;
          }
          x[(j0 + r) * k + c] = acc;
          Z[int64_t(F.perm[j0 + r]) * k + c] = acc;
        }
    }
  FILE* o = fopen(argv[2], "wb");
  fwrite(Z.data(), 8, n * k, o);
  fclose(o);
  printf("{\"rc\": 0, \"nsn\": %d, \"nlev_fwd\": %d, \"nlev_bwd\": %d, \"max_front\": %ld, "
         "\"dense_entries\": %.0f, \"t_order\": %.4f, \"t_factor\": %.4f, \"t_post\": %.4f}\n",
         S, F.nlev_fwd, F.nlev_bwd, (long)F.max_front, F.dense_entries, F.seconds_order,
         F.seconds_factor, F.seconds_post);
  return 0;
}
