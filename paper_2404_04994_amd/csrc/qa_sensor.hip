// qa_sensor.hip -- charge-sensor response (Sec. 5.1) after the array's
// charges are known.
//
// The problem's last S dots are sensor dots.  The array dots' charges n_a
// come from the array's own ground state or softargmin (computed with the
// array block of C_dd and C_gd: the sensors left out, every gate's
// cross-talk kept).  With n_a fixed, each pixel's sensor charges minimise
// U(n) = 1/2 (n - x_u)^T A (n - x_u), A = C_dd^{-1} of the whole system, over
// the floor/ceil box around the sensors' continuous minimum (clipped at 0:
// one sensor is then exact, a 1-D convex quadratic); the sensor potentials
// are v = A (n - x_u) (Eq. for the potential).  Adding a carrier to sensor s
// costs v_s + A_ss/2, removing one -v_s + A_ss/2; the response is the peak
// profile (Lorentzian or Gaussian, width gamma) of each, summed (the removal
// term only for an occupied sensor), so it peaks at the Coulomb-peak
// conditions on either side.  Noise on top, from draws passed in:
// white (amplitude x a standard-normal draw per sample), 1/f (Voss-McCartney:
// K octave sources, source k redrawn every 2^k samples, summed over sqrt K)
// and random telegraph jumps (the state flips where a uniform draw falls
// below the rate; amplitude x state), samples in pixel order.
#include "qa_device.h"

namespace qa {

constexpr int kMaxSensor = 4;

// one thread per pixel; the block first inverts the whole C_dd
__global__ __launch_bounds__(kPrepThreads) void k_sensor(
    const DiagRec *__restrict__ dr, int n_sensor, int shape, double gamma, const double *__restrict__ V,
    int64_t P, const int32_t *__restrict__ n_int, const double *__restrict__ n_dbl,
    const double *__restrict__ white_draws, double white, const double *__restrict__ pink_draws,
    double pink, int octaves, double *__restrict__ signal)
{
    __shared__ double sCdd[kMaxDot * kMaxDot];
    __shared__ double sA[kMaxDot * kMaxDot];
    __shared__ double cvec[kMaxDot];
    __shared__ double red[8];
    __shared__ double sG[kMaxGate * kMaxDot];   // C_gd transposed: sG[j * kMaxDot + i]
    __shared__ double sB[kMaxSensor * kMaxSensor];  // (A_ss)^{-1}
    const int n = dr->n, g = dr->g;
    const int S = n_sensor, Na = n - n_sensor;
    sCdd[threadIdx.x] = dr->Cdd[threadIdx.x];
    for (int e = threadIdx.x; e < kMaxGate * kMaxDot; e += blockDim.x) {
        const int j = e / kMaxDot, i = e % kMaxDot;
        sG[e] = dr->Cgd[i * kMaxGate + j];
    }
    __syncthreads();
    prep_inverse(sCdd, n, sA, cvec, red);
    if (threadIdx.x == 0) {
        // inverse of the sensor block of A by Gauss-Jordan (S <= 4; positive
        // definite, no pivoting)
        double m[kMaxSensor][2 * kMaxSensor];
        for (int i = 0; i < S; ++i)
            for (int j = 0; j < 2 * S; ++j)
                m[i][j] = (j < S) ? sA[(Na + i) * kMaxDot + Na + j] : (j - S == i ? 1.0 : 0.0);
        for (int k = 0; k < S; ++k) {
            const double r = 1.0 / m[k][k];
            for (int j = 0; j < 2 * S; ++j) m[k][j] *= r;
            for (int i = 0; i < S; ++i) {
                if (i == k) continue;
                const double f = m[i][k];
                for (int j = 0; j < 2 * S; ++j) m[i][j] -= f * m[k][j];
            }
        }
        for (int i = 0; i < S; ++i)
            for (int j = 0; j < S; ++j) sB[i * kMaxSensor + j] = m[i][S + j];
    }
    __syncthreads();

    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    // x_u = C_gd V of every dot
    double xu[kMaxDot];
#pragma unroll
    for (int i = 0; i < kMaxDot; ++i) xu[i] = 0.0;
    for (int j = 0; j < g; ++j) {
        const double v = V[p * g + j];
#pragma unroll
        for (int i = 0; i < kMaxDot; ++i) xu[i] += sG[j * kMaxDot + i] * v;
    }
    // w = A_sa (n_a - x_u,a): the array's pull on each sensor
    double w[kMaxSensor] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < Na; ++i) {
        const double na = n_int ? (double)n_int[p * Na + i] : n_dbl[p * Na + i];
        const double za = na - xu[i];
        for (int s = 0; s < S; ++s) w[s] += sA[(Na + s) * kMaxDot + i] * za;
    }
    // continuous minimum over the sensor charges and its box
    int base[kMaxSensor] = {0, 0, 0, 0};
    for (int s = 0; s < S; ++s) {
        double xs = xu[Na + s];
        for (int r = 0; r < S; ++r) xs -= sB[s * kMaxSensor + r] * w[r];
        base[s] = (int)floor(fmax(xs, 0.0));
    }
    // the sensor-dependent part of U: d^T w + 1/2 d^T A_ss d, d = n_s - x_u,s;
    // ties to the lexicographically smallest charges (sensor 0 most
    // significant): candidates in that order, strict improvement only
    double best = INFINITY;
    int bits = 0;
    for (int c = 0; c < (1 << S); ++c) {
        double d[kMaxSensor];
        for (int s = 0; s < S; ++s) d[s] = (double)(base[s] + ((c >> (S - 1 - s)) & 1)) - xu[Na + s];
        double e = 0.0;
        for (int s = 0; s < S; ++s) {
            double q = 0.0;
            for (int r = 0; r < S; ++r) q += sA[(Na + s) * kMaxDot + Na + r] * d[r];
            e += d[s] * (w[s] + 0.5 * q);
        }
        if (e < best) { best = e; bits = c; }
    }
    for (int s = 0; s < S; ++s) {
        const int ns = base[s] + ((bits >> (S - 1 - s)) & 1);
        // sensor potential v_s = w_s + (A_ss d)_s
        double vs = w[s];
        for (int r = 0; r < S; ++r) {
            const double dr_ = (double)(base[r] + ((bits >> (S - 1 - r)) & 1)) - xu[Na + r];
            vs += sA[(Na + s) * kMaxDot + Na + r] * dr_;
        }
        const double half = 0.5 * sA[(Na + s) * kMaxDot + Na + s];
        const double xp = (vs + half) / gamma, xm = (-vs + half) / gamma;
        double r;
        if (shape == 0) {
            r = 1.0 / (1.0 + xp * xp) + (ns > 0 ? 1.0 / (1.0 + xm * xm) : 0.0);
        } else {
            r = exp(-0.5 * xp * xp) + (ns > 0 ? exp(-0.5 * xm * xm) : 0.0);
        }
        if (white_draws) r += white * white_draws[p * S + s];
        if (pink_draws) {
            // octave k of sensor s starts after the earlier sources' draws
            double sum = 0.0;
            int64_t off = 0;
            for (int s2 = 0; s2 < S; ++s2)
                for (int k = 0; k < octaves; ++k) {
                    const int64_t len = (P + ((int64_t)1 << k) - 1) >> k;
                    if (s2 == s) sum += pink_draws[off + (p >> k)];
                    off += len;
                }
            r += pink * sum / sqrt((double)octaves);
        }
        signal[p * S + s] = r;
    }
}

// random telegraph noise, one block of 1024 threads per sensor: the flips
// (uniform draw below the rate) are prefix-counted over the samples in
// chunks of 1024 (wave ballots, then the 16 wave totals), and amplitude x
// (count mod 2) is added to the signal
__global__ __launch_bounds__(1024) void k_sensor_jumps(int64_t P, int n_sensor,
                                                       const double *__restrict__ u, double rate,
                                                       double amp, double *__restrict__ signal)
{
    __shared__ int wsum[16];
    __shared__ int carry_s;
    const int s = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < P; c0 += 1024) {
        const int64_t t = c0 + threadIdx.x;
        const bool flip = t < P && u[t * n_sensor + s] < rate;
        const unsigned long long b = __ballot(flip);
        const int incl = __popcll(b & (~0ull >> (63 - lane)));  // flips up to this lane
        if (lane == 63) wsum[wv] = __popcll(b);
        __syncthreads();
        int before = carry_s;
        for (int k = 0; k < wv; ++k) before += wsum[k];
        if (t < P && ((before + incl) & 1)) signal[t * n_sensor + s] += amp;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int k = 0; k < 16; ++k) tot += wsum[k];
            carry_s += tot;
        }
        __syncthreads();
    }
}

hipError_t launch_sensor(const DiagRec *dr, int n_sensor, int shape, double gamma, const double *V,
                         int64_t P, const int32_t *n_int, const double *n_dbl,
                         const double *white_draws, double white, const double *pink_draws,
                         double pink, int octaves, double *signal, hipStream_t s)
{
    if (P <= 0) return hipSuccess;
    if (n_sensor < 1 || n_sensor > kMaxSensor) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((P + kPrepThreads - 1) / kPrepThreads);
    hipLaunchKernelGGL(k_sensor, dim3(blocks), dim3(kPrepThreads), 0, s, dr, n_sensor, shape, gamma,
                       V, P, n_int, n_dbl, white_draws, white, pink_draws, pink, octaves, signal);
    return hipGetLastError();
}

hipError_t launch_sensor_jumps(int64_t P, int n_sensor, const double *u, double rate, double amp,
                               double *signal, hipStream_t s)
{
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sensor_jumps, dim3(n_sensor), dim3(1024), 0, s, P, n_sensor, u, rate, amp,
                       signal);
    return hipGetLastError();
}

}  // namespace qa
