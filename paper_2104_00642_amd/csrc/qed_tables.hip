// qed_tables.hip -- rate and inverse-CDF tables of the QED module, computed
// on the GPU in FP64 from the spectra of Sec. IV:
//   nonlinear Compton (Eq. 23): bracket_c(u) = (u^2-2u+2)/(1-u) K_{2/3}(y) - int_y^inf K_{1/3},
//                               y = 2u / (3 (1-u) chi)
//   nonlinear Breit-Wheeler (Eq. 24): bracket_p(x) = (x^2+(1-x)^2)/(x(1-x)) K_{2/3}(y) + int_y^inf K_{1/3},
//                               y = 2 / (3 chi x (1-x))
// F(chi) = int_0^1 bracket; the normalized rates are W = alpha/(sqrt3 pi) (m c^2/hbar w_r) F / eps.
// Bessel functions from K_nu(y) = int_0^inf exp(-y cosh t) cosh(nu t) dt and
// int_y^inf K_{1/3} = int_0^inf exp(-y cosh t) cosh(t/3)/cosh t dt (trapezoidal
// rule in t).  The energy fraction is reached through the smoothstep
// u = 10v^3 - 15v^4 + 6v^5, which removes the u^(-2/3) behaviour at u -> 0 and
// the (1-u)^(-1/3) tail at u -> 1; cumulative integrals use the midpoint
// rule on a fine uniform grid in v.  Method II reads the normalized
// differential spectra at (chi, sigma) nodes.
#include "device_common.h"
#include "pic_internal.h"
#include "qed_internal.h"

namespace pic {

__device__ double trap_bessel(double y, double nu, int mode) {
    const double h = 1.0 / 48.0;
    double sum = 0.0;
    for (int k = 0; k < 100000; ++k) {
        const double t = k * h;
        const double ch = cosh(t);
        const double e = exp(-y * ch);
        const double term = mode == 0 ? e * cosh(nu * t) : e * cosh(t / 3.0) / ch;
        sum += (k == 0 ? 0.5 : 1.0) * term;
        if (y * sinh(t) > nu + 1.0 && term < 1e-17 * sum) break;
    }
    return sum * h;
}

__device__ double bracket(int proc, double x, double chi) {
    if (x <= 0.0 || x >= 1.0) return 0.0;
    if (proc == QED_COMPTON) {
        const double y = 2.0 * x / (3.0 * (1.0 - x) * chi);
        if (y > 700.0) return 0.0;
        return (x * x - 2.0 * x + 2.0) / (1.0 - x) * trap_bessel(y, 2.0 / 3.0, 0) - trap_bessel(y, 0.0, 1);
    }
    const double y = 2.0 / (3.0 * chi * x * (1.0 - x));
    if (y > 700.0) return 0.0;
    return (x * x + (1.0 - x) * (1.0 - x)) / (x * (1.0 - x)) * trap_bessel(y, 2.0 / 3.0, 0) +
           trap_bessel(y, 0.0, 1);
}

__device__ __forceinline__ double smoothstep5(double v) { return v * v * v * (10.0 + v * (-15.0 + 6.0 * v)); }
__device__ __forceinline__ double dsmoothstep5(double v) { return 30.0 * v * v * (1.0 - v) * (1.0 - v); }

// integrand in v at the midpoints of the fine grid, bracket(u(v)) du/dv, one
// thread per (chi, interval); the midpoint rule never evaluates the endpoint
// v = 0, where the integrand has a finite limit but bracket(0) is undefined
__global__ void qed_integrand_kernel(int proc, const double *chis, int nchi, double *out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nchi * QED_NV) return;
    const int i = (int)(e / QED_NV), j = (int)(e % QED_NV);
    if (j == QED_NV - 1) {
        out[e] = 0.0;
        return;
    }
    const double v = ((double)j + 0.5) / (QED_NV - 1);
    out[e] = bracket(proc, smoothstep5(v), chis[i]) * dsmoothstep5(v);
}

// per chi: cumulative midpoint-rule integral at the grid nodes (in place),
// returns the total
__global__ void qed_cumulate_kernel(double *f, int nchi, double *total) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nchi) return;
    double *row = f + (int64_t)i * QED_NV;
    const double h = 1.0 / (QED_NV - 1);
    double acc = 0.0, prev = row[0];
    row[0] = 0.0;
    for (int j = 1; j < QED_NV; ++j) {
        const double cur = row[j];
        acc += h * prev;
        prev = cur;
        row[j] = acc;
    }
    total[i] = acc;
}

// inverse CDF: for each (chi_i, r_k) find u with C(u) = r C(1); stored as
// u^(1/3) (Compton) or x (pairs)
__global__ void qed_invert_kernel(int proc, const double *cum, const double *total, int nchi,
                                  float *table) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nchi * QED_NR) return;
    const int i = e / QED_NR, k = e % QED_NR;
    const double r = qed_r_of_rho(proc, (double)k / (QED_NR - 1));
    const double *row = cum + (int64_t)i * QED_NV;
    const double target = r * total[i];
    int lo = 0, hi = QED_NV - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (row[mid] < target) lo = mid;
        else hi = mid;
    }
    const double c0 = row[lo], c1 = row[hi];
    const double fr = c1 > c0 ? (target - c0) / (c1 - c0) : 0.0;
    const double v = ((double)lo + fr) / (QED_NV - 1);
    const double u = smoothstep5(v);
    table[e] = (float)(proc == QED_COMPTON ? cbrt(u) : u);
}

// log-rate tables with the known asymptotic factor removed:
//   Compton  g = ln(F / chi);  pairs  g = ln F + 8 / (3 chi)
__global__ void qed_logrates_kernel(int proc, const double *chis, const double *total, int nchi,
                                    float *g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nchi) return;
    const double F = total[i];
    const double chi = chis[i];
    g[i] = (float)(proc == QED_COMPTON ? log(F / chi) : log(F) + 8.0 / (3.0 * chi));
}

// Method II densities at the (chi_i, sigma_k) nodes: 3 s^2 bracket_c(s^3) / F
// in s for emission (finite as s -> 0; the node s = 0 takes s = 1e-6, where
// the next term of the expansion is 1e-12 of the limit), bracket_p(x) / F in x
// for pairs
__global__ void qed_density_kernel(int proc, const double *chis, const double *total, int nchi,
                                   float *table) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nchi * QED_NS) return;
    const int i = e / QED_NS, k = e % QED_NS;
    const double sig = 0.5 * (1.0 - cos(3.14159265358979323846 * k / (QED_NS - 1)));
    double v;
    if (proc == QED_COMPTON) {
        const double s = fmax(sig, 1e-6);
        v = 3.0 * s * s * bracket(proc, s * s * s, chis[i]);
    } else {
        v = bracket(proc, sig, chis[i]);
    }
    table[e] = total[i] > 0.0 ? (float)(v / total[i]) : 0.0f;
}

__global__ void qed_chigrid_kernel(double lo, double hi, int n, double *chis) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) chis[i] = exp10(lo + (hi - lo) * i / (n - 1));
}

hipError_t build_qed_tables(QedTables *t, hipStream_t s) {
    double *chis = nullptr, *f = nullptr, *total = nullptr;
    hipError_t e = hipMalloc(&chis, sizeof(double) * QED_NCHI);
    if (e == hipSuccess) e = hipMalloc(&f, sizeof(double) * QED_NCHI * QED_NV);
    if (e == hipSuccess) e = hipMalloc(&total, sizeof(double) * QED_NCHI);
    if (e == hipSuccess) e = hipMalloc(&t->dev, sizeof(float) * QED_TABLE_FLOATS);
    for (int proc = 0; proc < 2 && e == hipSuccess; ++proc) {
        const double lo = proc == QED_COMPTON ? QED_LOG_CHI_MIN_C : QED_LOG_CHI_MIN_P;
        qed_chigrid_kernel<<<1, QED_NCHI, 0, s>>>(lo, QED_LOG_CHI_MAX, QED_NCHI, chis);
        const int64_t ne = (int64_t)QED_NCHI * QED_NV;
        qed_integrand_kernel<<<(unsigned)((ne + 255) / 256), 256, 0, s>>>(proc, chis, QED_NCHI, f);
        qed_cumulate_kernel<<<1, QED_NCHI, 0, s>>>(f, QED_NCHI, total);
        float *rate = t->dev + (proc == QED_COMPTON ? QED_OFF_RATE_C : QED_OFF_RATE_P);
        float *inv = t->dev + (proc == QED_COMPTON ? QED_OFF_INV_C : QED_OFF_INV_P);
        qed_logrates_kernel<<<1, QED_NCHI, 0, s>>>(proc, chis, total, QED_NCHI, rate);
        qed_invert_kernel<<<(QED_NCHI * QED_NR + 255) / 256, 256, 0, s>>>(proc, f, total, QED_NCHI, inv);
        float *den = t->dev + (proc == QED_COMPTON ? QED_OFF_DEN_C : QED_OFF_DEN_P);
        qed_density_kernel<<<(QED_NCHI * QED_NS + 255) / 256, 256, 0, s>>>(proc, chis, total, QED_NCHI, den);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(chis);
    hipFree(f);
    hipFree(total);
    return e;
}

}  // namespace pic
