// Diffusion-synthetic acceleration of the scattering iteration on gfx950.
//
// The paper runs its outer GMRES on Phi without a preconditioner (Sec. 4.2)
// and names acceleration as needed for scattering-dominated problems
// (Sec. 6).  Here the outer GMRES is preconditioned from the right with the
// diffusion approximation of the scattering correction, built from the
// direction-independent blocks already integrated (same pattern, same test
// functions):  P^-1 v = v + C^-1 (Ms v).
#include "internal.hpp"

namespace mlpg {

namespace {

struct DsaSigma {
    double t[kMaxMat], a[kMaxMat], s[kMaxMat];
};

// One thread per row: sigma_t,i is the mass-weighted mean of the materials'
// effective sigma_t over row i and D_i = 1 / (3 sigma_t,i);
//   C[p]  = D_i sum_a K^aa[p] + sum_g sigma_a,g Mass_g[p] + 1/2 sum_f S_f[p]
//   Ms[p] = sum_g sigma_s,g Mass_g[p],   dinv[i] = 1 / C[diag(i)]
// (the face term is the Marshak vacuum condition).
__global__ void dsa_assemble_kernel(int64_t n, int dim, int G, int64_t nnz, const int64_t *__restrict__ row_off,
                                    const int64_t *__restrict__ diag_pos, const double *__restrict__ blocks,
                                    DsaSigma sg, double *__restrict__ C, double *__restrict__ Ms,
                                    double *__restrict__ dinv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int kb = G * (1 + dim), sb = kb + dim * dim;
    double mt = 0.0, m1 = 0.0;
    for (int g = 0; g < G; ++g) {
        double mg = 0.0;
        for (int64_t p = row_off[i]; p < row_off[i + 1]; ++p) mg += blocks[(int64_t)(g * (1 + dim)) * nnz + p];
        mt += sg.t[g] * mg;
        m1 += mg;
    }
    const double st = (m1 != 0.0 && mt > 0.0) ? mt / m1 : 1.0;
    const double D = 1.0 / (3.0 * st);
    for (int64_t p = row_off[i]; p < row_off[i + 1]; ++p) {
        double k = 0.0, a = 0.0, sc = 0.0, sf = 0.0;
        for (int al = 0; al < dim; ++al) k += blocks[(int64_t)(kb + al * dim + al) * nnz + p];
        for (int g = 0; g < G; ++g) {
            const double mg = blocks[(int64_t)(g * (1 + dim)) * nnz + p];
            a += sg.a[g] * mg;
            sc += sg.s[g] * mg;
        }
        for (int f = 0; f < 2 * dim; ++f) sf += blocks[(int64_t)(sb + f) * nnz + p];
        C[p] = D * k + a + 0.5 * sf;
        Ms[p] = sc;
    }
    const double d = C[diag_pos[i]];
    dinv[i] = d != 0.0 ? 1.0 / d : 1.0;
}

// y[i] = sum_p vals[p] (dinv .* x)[col[p]] for one vector, a wave per row
// (lanes stride the row, then a fixed-order shuffle reduction).
__global__ __launch_bounds__(256) void csr_spmv_kernel(int64_t n, const int64_t *__restrict__ row_off,
                                                       const int32_t *__restrict__ col,
                                                       const double *__restrict__ vals,
                                                       const double *__restrict__ x,
                                                       const double *__restrict__ dinv, double *__restrict__ y,
                                                       const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= n) return;
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
    for (int64_t p = row_off[i] + lane; p < row_off[i + 1]; p += 64) {
        const int32_t j = col[p];
        acc += vals[p] * (dinv ? dinv[j] * x[j] : x[j]);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) y[i] = acc;
}

}  // namespace

hipError_t launch_dsa_assemble(Problem &P, const double *sig_t_eff, const double *sig_a_eff, const double *sig_s,
                               hipStream_t s)
{
    if (P.n_mat > kMaxMat) return hipErrorInvalidValue;
    DsaSigma sg = {};
    for (int g = 0; g < P.n_mat; ++g) {
        sg.t[g] = sig_t_eff[g];
        sg.a[g] = sig_a_eff[g];
        sg.s[g] = sig_s[g];
    }
    dsa_assemble_kernel<<<(unsigned)((P.n + 255) / 256), 256, 0, s>>>(P.n, P.dim, P.n_mat, P.nnz, P.row_off.p,
                                                                       P.diag_pos.p, P.blocks.p, sg, P.dsaC.p,
                                                                       P.dsaMs.p, P.dsa_dinv.p);
    return hipGetLastError();
}

hipError_t launch_csr_spmv(Problem &P, const double *vals, const double *x, const double *dinv, double *y,
                           const int *gate, hipStream_t s)
{
    csr_spmv_kernel<<<(unsigned)((P.n + 3) / 4), 256, 0, s>>>(P.n, P.row_off.p, P.col.p, vals, x, dinv, y, gate);
    return hipGetLastError();
}

}  // namespace mlpg
