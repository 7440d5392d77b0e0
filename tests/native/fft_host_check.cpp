// Host-side check of the FFT building blocks of the HIP library: the same
// header, compiled for the CPU, transforms lines that the test compares with
// numpy's FFT.
#include <cmath>
#include <vector>
#include "../../paper_1307_8052_amd/csrc/fft.hpp"

using rpa::cplx;

extern "C" int fft_lines_host(int N, int dir, int nlines, const double* in, double* out) {
    rpa::FftPlan plan;
    if (!rpa::make_plan(N, &plan)) return -1;
    std::vector<cplx<double>> a(nlines * N), b(nlines * N), tw(N);
    for (int t = 0; t < N; ++t) tw[t] = rpa::mk(std::cos(2 * M_PI * t / N), -std::sin(2 * M_PI * t / N));
    for (int i = 0; i < nlines * N; ++i) a[i] = rpa::mk(in[2 * i], in[2 * i + 1]);
    auto addr = [N](int l, int e) { return l * N + e; };
    cplx<double>* src = a.data();
    cplx<double>* dst = b.data();
    int Ns = 1;
    for (int s = 0; s < plan.nstages; ++s) {
        int R = plan.radix[s];
        if (dir < 0)
            rpa::stockham_dispatch<-1>(R, src, dst, N, Ns, nlines, (s & 1) != 0, addr, tw.data(), 0, 1);
        else
            rpa::stockham_dispatch<+1>(R, src, dst, N, Ns, nlines, (s & 1) == 0, addr, tw.data(), 0, 1);
        std::swap(src, dst);
        Ns *= R;
    }
    for (int i = 0; i < nlines * N; ++i) { out[2 * i] = src[i].x; out[2 * i + 1] = src[i].y; }
    return 0;
}

// One line through the register-resident transform of the same header.
template <int N>
static void reg_line(int dir, const double* in, double* out) {
    cplx<double> v[N];
    for (int i = 0; i < N; ++i) v[i] = rpa::mk(in[2 * i], in[2 * i + 1]);
    if (dir < 0) rpa::RegFft<N, -1, double>::run(v);
    else rpa::RegFft<N, +1, double>::run(v);
    for (int i = 0; i < N; ++i) { out[2 * i] = v[i].x; out[2 * i + 1] = v[i].y; }
}

extern "C" int fft_reg_sizes(int* out, int cap) {
    int n = 0;
#define RPA_LIST(N) if (n < cap) out[n] = N; ++n;
    RPA_REG_SIZES(RPA_LIST)
#undef RPA_LIST
    return n;
}

extern "C" int fft_reg_host(int N, int dir, const double* in, double* out) {
    switch (N) {
#define RPA_CASE(L) case L: reg_line<L>(dir, in, out); return 0;
        RPA_REG_SIZES(RPA_CASE)
#undef RPA_CASE
        default: return -1;
    }
}

// FP32 versions of the same transforms: the twiddle table holds the FP32 values and then their low parts,
// as the library builds it.
extern "C" int fft_lines_host_f32(int N, int dir, int nlines, const float* in, float* out) {
    rpa::FftPlan plan;
    if (!rpa::make_plan(N, &plan)) return -1;
    std::vector<cplx<float>> a(nlines * N), b(nlines * N), tw(rpa::twiddle_len<float>(N));
    for (int t = 0; t < N; ++t) {
        const double c = std::cos(2 * M_PI * t / N), s = -std::sin(2 * M_PI * t / N);
        tw[t] = rpa::mk((float)c, (float)s);
        tw[N + t] = rpa::mk((float)(c - (double)tw[t].x), (float)(s - (double)tw[t].y));
    }
    for (int i = 0; i < nlines * N; ++i) a[i] = rpa::mk(in[2 * i], in[2 * i + 1]);
    auto addr = [N](int l, int e) { return l * N + e; };
    cplx<float>* src = a.data();
    cplx<float>* dst = b.data();
    int Ns = 1;
    for (int s = 0; s < plan.nstages; ++s) {
        int R = plan.radix[s];
        if (dir < 0)
            rpa::stockham_dispatch<-1>(R, src, dst, N, Ns, nlines, (s & 1) != 0, addr, tw.data(), 0, 1);
        else
            rpa::stockham_dispatch<+1>(R, src, dst, N, Ns, nlines, (s & 1) == 0, addr, tw.data(), 0, 1);
        std::swap(src, dst);
        Ns *= R;
    }
    for (int i = 0; i < nlines * N; ++i) { out[2 * i] = src[i].x; out[2 * i + 1] = src[i].y; }
    return 0;
}

template <int N>
static void reg_lines_f32(int dir, int nlines, const float* in, float* out) {
    for (int l = 0; l < nlines; ++l) {
        cplx<float> v[N];
        for (int i = 0; i < N; ++i) v[i] = rpa::mk(in[2 * (l * N + i)], in[2 * (l * N + i) + 1]);
        if (dir < 0) rpa::RegFft<N, -1, float>::run(v);
        else rpa::RegFft<N, +1, float>::run(v);
        for (int i = 0; i < N; ++i) { out[2 * (l * N + i)] = v[i].x; out[2 * (l * N + i) + 1] = v[i].y; }
    }
}

extern "C" int fft_reg_host_f32(int N, int dir, int nlines, const float* in, float* out) {
    switch (N) {
#define RPA_CASE(L) case L: reg_lines_f32<L>(dir, nlines, in, out); return 0;
        RPA_REG_SIZES(RPA_CASE)
#undef RPA_CASE
        default: return -1;
    }
}
