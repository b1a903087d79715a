// Momentum-residual assembly: kernels and the lesasm_assemble_momentum_rhs entry.
//
// Algorithm 1, step "Element assembly", run once per Runge-Kutta stage:
// every element gathers its nodes, computes its residual at the Gauss points
// (Section 3.2, equation (momentum), EMAC + viscous + Vreman terms) and
// scatter-adds it into the nodal right-hand side (Section 3.4.3).  One launch
// per element category (type); in colour mode one launch per colour, so no two
// threads of a launch touch the same node and the scatter is a plain
// read-modify-write with a fixed summation order.
#include "element.hpp"

namespace lesasm {

template <int T, typename R, bool ATOMIC, bool HAS_P>
__global__ __launch_bounds__(256) void k_assemble(CatView c, const double *__restrict__ xyz,
                                                  const double *__restrict__ u, const double *__restrict__ p,
                                                  double nu, double cv, double *__restrict__ rhs) {
    constexpr int nn = Ref<T>::nn;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int local = b * blockDim.x + threadIdx.x;
    if (local >= c.n) return;
    const int e = c.off + local;
    ElementData<T, R> d;
    gather<T, R, HAS_P>(d, c, e, xyz, u, p);
    const double dl = c.delta[e];
    R acc[nn][3];
    element_residual<T, R, HAS_P>(d, (R)nu, (R)(cv * dl * dl), acc);
#pragma unroll
    for (int a = 0; a < nn; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double *dst = rhs + 3 * (size_t)d.fid[a] + i;
            if (ATOMIC)
                unsafeAtomicAdd(dst, (double)acc[a][i]);
            else
                *dst += (double)acc[a][i];
        }
}

__global__ void k_fill(double *__restrict__ a, size_t n, double v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] = v;
}

// rhs <- dt * M_L^-1 rhs
__global__ void k_increment(double *__restrict__ rhs, const double *__restrict__ mass, double dt, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double s = dt / mass[i];
        rhs[3 * i + 0] *= s;
        rhs[3 * i + 1] *= s;
        rhs[3 * i + 2] *= s;
    }
}

__global__ void k_check_finite(const double *__restrict__ a, size_t n, int *flag) {
    int bad = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        bad |= !isfinite(a[i]);
    if (bad) atomicOr(flag, 1);
}

int grid_for(size_t n, int block) {
    size_t g = (n + block - 1) / block;
    return (int)(g < 8192 ? (g ? g : 1) : 8192);
}

template <int T, typename R, bool ATOMIC, bool HAS_P>
static void launch_cat(const CatView &v, int block, hipStream_t s, const double *xyz, const double *u,
                       const double *p, double nu, double cv, double *rhs) {
    const int nb = (v.n + block - 1) / block;
    hipLaunchKernelGGL((k_assemble<T, R, ATOMIC, HAS_P>), dim3(nb), dim3(block), 0, s, v, xyz, u, p, nu, cv, rhs);
}

template <int T, typename R>
static void dispatch_scatter(const CatView &v, bool atomic, bool has_p, int block, hipStream_t s,
                             const double *xyz, const double *u, const double *p, double nu, double cv,
                             double *rhs) {
    if (atomic) {
        if (has_p) launch_cat<T, R, true, true>(v, block, s, xyz, u, p, nu, cv, rhs);
        else launch_cat<T, R, true, false>(v, block, s, xyz, u, p, nu, cv, rhs);
    } else {
        if (has_p) launch_cat<T, R, false, true>(v, block, s, xyz, u, p, nu, cv, rhs);
        else launch_cat<T, R, false, false>(v, block, s, xyz, u, p, nu, cv, rhs);
    }
}

ProfileScope::ProfileScope(lesasm_mesh *m_, int slot_, hipStream_t s_) : m(m_), slot(slot_), s(s_) {
    if (!m->profile) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        a = b = nullptr;
        return;
    }
    (void)hipEventRecord(a, s);
}

ProfileScope::~ProfileScope() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    m->pending[slot].push_back({a, b});
}

template <typename R>
static void dispatch_type(int type, const CatView &v, bool atomic, bool has_p, int block, hipStream_t s,
                          const double *xyz, const double *u, const double *p, double nu, double cv, double *rhs) {
    switch (type) {
    case LESASM_TET04: dispatch_scatter<LESASM_TET04, R>(v, atomic, has_p, block, s, xyz, u, p, nu, cv, rhs); break;
    case LESASM_PYR05: dispatch_scatter<LESASM_PYR05, R>(v, atomic, has_p, block, s, xyz, u, p, nu, cv, rhs); break;
    case LESASM_PEN06: dispatch_scatter<LESASM_PEN06, R>(v, atomic, has_p, block, s, xyz, u, p, nu, cv, rhs); break;
    case LESASM_HEX08: dispatch_scatter<LESASM_HEX08, R>(v, atomic, has_p, block, s, xyz, u, p, nu, cv, rhs); break;
    }
}

// Launches every element kernel of one assembly on stream s (rhs already zeroed).
int launch_assembly(lesasm_mesh *m, const double *u, const double *p, double nu, double *rhs, hipStream_t s) {
    const bool atomic = !(m->flags & LESASM_MESH_SCATTER_COLOUR);
    for (int k = 0; k < kNumCat; ++k) {
        const Category &c = m->cat[k];
        if (c.n == 0) continue;
        const size_t nranges = atomic ? 1 : c.colour_off.size() - 1;
        for (size_t r = 0; r < nranges; ++r) {
            CatView v;
            v.cg = c.d_cg;
            v.cf = c.d_cf;
            v.delta = c.d_delta;
            v.ld = (int32_t)c.n;
            v.off = atomic ? 0 : (int32_t)c.colour_off[r];
            v.n = atomic ? (int32_t)c.n : (int32_t)(c.colour_off[r + 1] - c.colour_off[r]);
            if (v.n == 0) continue;
            ProfileScope ps(m, LESASM_KERNEL_TET04 + k, s);
            if (m->precision == LESASM_PREC_FP32)
                dispatch_type<float>(c.type, v, atomic, p != nullptr, m->block, s, m->d_xyz, u, p, nu, m->vreman_c, rhs);
            else
                dispatch_type<double>(c.type, v, atomic, p != nullptr, m->block, s, m->d_xyz, u, p, nu, m->vreman_c, rhs);
        }
    }
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

}  // namespace lesasm

using namespace lesasm;

static bool misaligned(const void *p) { return ((uintptr_t)p & 7u) != 0; }

extern "C" int lesasm_assemble_momentum_rhs(lesasm_mesh *m, const double *d_u, const double *d_p, double nu,
                                            double dt, double *d_rhs, void *stream) {
    if (!m) return fail(LESASM_E_INVALID_ARG, "assemble: mesh is NULL");
    if (m->n_field > 0 && (!d_u || !d_rhs)) return fail(LESASM_E_INVALID_ARG, "assemble: u or rhs is NULL");
    if (misaligned(d_u) || misaligned(d_p) || misaligned(d_rhs))
        return fail(LESASM_E_INVALID_ARG, "assemble: pointers must be 8-byte aligned");
    if (d_rhs && (d_rhs == d_u || (d_p && d_rhs == d_p)))
        return fail(LESASM_E_INVALID_ARG, "assemble: rhs aliases an input");
    int dev = -1;
    LESASM_HIP_TRY(hipGetDevice(&dev));
    if (dev != m->device) return fail(LESASM_E_STATE, "assemble: current device differs from the mesh's device");
    hipStream_t s = (hipStream_t)stream;
    if (m->n_field == 0) return LESASM_OK;
    const size_t n3 = 3 * (size_t)m->n_field;

    if (m->check_finite) {
        int zero = 0, flag = 0;
        LESASM_HIP_TRY(hipMemcpyAsync(m->d_flag, &zero, sizeof(int), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n3, 256)), dim3(256), 0, s, d_u, n3, m->d_flag);
        if (d_p)
            hipLaunchKernelGGL(k_check_finite, dim3(grid_for(m->n_field, 256)), dim3(256), 0, s, d_p,
                               (size_t)m->n_field, m->d_flag);
        LESASM_HIP_TRY(hipMemcpyAsync(&flag, m->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
        LESASM_HIP_TRY(hipStreamSynchronize(s));
        if (flag) return fail(LESASM_E_NONFINITE, "assemble: u or p holds NaN/Inf");
    }

    {
        ProfileScope ps(m, LESASM_KERNEL_FILL, s);
        hipLaunchKernelGGL(k_fill, dim3(grid_for(n3, 256)), dim3(256), 0, s, d_rhs, n3, 0.0);
    }
    int st = launch_assembly(m, d_u, d_p, nu, d_rhs, s);
    if (st) return st;
    if (m->rhs_mode == LESASM_RHS_INCREMENT) {
        ProfileScope ps(m, LESASM_KERNEL_INCREMENT, s);
        hipLaunchKernelGGL(k_increment, dim3(grid_for(m->n_field, 256)), dim3(256), 0, s, d_rhs, m->d_mass, dt,
                           (size_t)m->n_field);
    }
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_mesh_kernel_times(lesasm_mesh *m, double *ms, int64_t *launches, int reset) {
    if (!m || !ms || !launches) return fail(LESASM_E_INVALID_ARG, "kernel_times: NULL argument");
    for (int k = 0; k < LESASM_NUM_KERNEL_SLOTS; ++k) {
        for (auto &ev : m->pending[k]) {
            float t = 0.0f;
            LESASM_HIP_TRY(hipEventSynchronize(ev.second));
            LESASM_HIP_TRY(hipEventElapsedTime(&t, ev.first, ev.second));
            m->prof_ms[k] += t;
            m->prof_n[k] += 1;
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
        m->pending[k].clear();
        ms[k] = m->prof_ms[k];
        launches[k] = m->prof_n[k];
        if (reset) {
            m->prof_ms[k] = 0.0;
            m->prof_n[k] = 0;
        }
    }
    return LESASM_OK;
}
