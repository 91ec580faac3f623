// Device-side stencil operators on the structured right-diagonal mesh and
// block reductions, shared by the solver and problem translation units.
#pragma once

#include "common.h"

namespace hinv {

// ------------------------------------------------------------ reductions ---
__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over a workgroup of kBlock threads, fixed order; result valid in thread 0.
// Call at most once per kernel (the LDS slot is not reused).
__device__ inline double block_sum(double v) {
    __shared__ double part[kBlock / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) part[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) r += part[i];
    return r;
}

// ------------------------------------------------------- state operator ---
// A(m) restricted to the free nodes (0 < j < N): the P1 stiffness with the
// per-triangle coefficient c_T is a five-point stencil on this mesh (the
// diagonal edge is opposite a right angle).  wE[k] is the weight of edge
// (i,j)-(i+1,j) = (c_lower(i,j) + c_upper(i,j-1)) / 2, wN[k] the weight of edge
// (i,j)-(i,j+1) = (c_upper(i,j) + c_lower(i-1,j)) / 2 (absent triangles count
// zero); the diagonal is the sum of the four incident edge weights.
// Several instances of one mesh size can share a launch: their coefficient
// arrays are stacked cs elements apart and column c belongs to instance
// c / cpi (cs = 0: one instance).
template <typename T>
struct OpA {
    int N;
    const T* wE;
    const T* wN;
    const T* dinv;  // 1 / diagonal on free nodes, 0 on Dirichlet nodes
    long long cs = 0;
    int cpi = 1;
    // the operator of the instance that owns column c
    __device__ OpA at(int c) const {
        OpA o = *this;
        if (cs) {
            const long long off = (long long)(c / cpi) * cs;
            o.wE += off;
            o.wN += off;
            o.dinv += off;
        }
        return o;
    }
    __device__ bool is_free(int, int j) const { return j > 0 && j < N; }
    __device__ T inv_diag(int, int, int k) const { return dinv[k]; }
    // diagonal of a free row: sum of the four incident edge weights
    __device__ T diag(int i, int, int k) const {
        return (i < N ? wE[k] : (T)0) + (i > 0 ? wE[k - 1] : (T)0) + wN[k] + wN[k - N - 1];
    }
    // Row k of A_FF applied to the vector given by xat(i, j, k); call on free nodes only.
    template <class F>
    __device__ T apply(int i, int j, int k, F xat) const {
        T s = 0, d = 0;
        if (i < N) {
            const T w = wE[k];
            d += w;
            s += w * xat(i + 1, j, k + 1);
        }
        if (i > 0) {
            const T w = wE[k - 1];
            d += w;
            s += w * xat(i - 1, j, k - 1);
        }
        {
            const T w = wN[k];
            d += w;
            if (j + 1 < N) s += w * xat(i, j + 1, k + N + 1);
        }
        {
            const T w = wN[k - N - 1];
            d += w;
            if (j - 1 > 0) s += w * xat(i, j - 1, k - N - 1);
        }
        return d * xat(i, j, k) - s;
    }
    // Straight-line form of apply() for kernels that overlap the loads of
    // several rows: row() and gather() issue every load of row k (an absent
    // neighbour reads node k itself), combine() gives it weight zero.  Same
    // operation order as apply(), so on finite vectors the two agree bit for bit.
    struct Row {
        T we, ww, wn, ws;
    };
    struct Nb {
        T c, e, w, n, s;
    };
    __device__ Row row(int i, int j, int k) const {
        const int N1 = N + 1;
        return Row{wE[k], wE[i > 0 ? k - 1 : k], wN[k], wN[j > 0 ? k - N1 : k]};
    }
    __device__ Nb gather(int i, int j, int k, const T* __restrict__ x) const {
        const int N1 = N + 1;
        return Nb{x[k], x[i < N ? k + 1 : k], x[i > 0 ? k - 1 : k], x[j + 1 < N ? k + N1 : k],
                  x[j > 1 ? k - N1 : k]};
    }
    __device__ T combine(int i, int j, const Row& r, const Nb& v) const {
        const T we = i < N ? r.we : (T)0, ww = i > 0 ? r.ww : (T)0;
        T s = 0, d = 0;
        d += we;
        s += we * v.e;
        d += ww;
        s += ww * v.w;
        d += r.wn;
        s += (j + 1 < N ? r.wn : (T)0) * v.n;
        d += r.ws;
        s += (j - 1 > 0 ? r.ws : (T)0) * v.s;
        return d * v.c - s;
    }
};

// ------------------------------------------------------- prior operator ---
// K_A = g K + dl M + bt M_boundary with Theta = I (every node is a dof).
// K: unit five-point stiffness (edge weight = number of adjacent triangles / 2).
// M: P1 mass, |T|/12 (1 + delta_vw) per triangle, |T| = h^2/2; couples the
//    four axis neighbours and the two diagonal neighbours (i+-1, j+-1).
// M_boundary: (h/6) [[2,1],[1,2]] on every boundary edge.
// Constant coefficients: the rows of the 9 node classes travel as kernel
// arguments, so applying K_A reads no coefficient array.
// Row of the prior operator: diagonal, the six neighbour couplings and 1/diagonal.
template <typename T>
struct KARow {
    T c, e, w, n, s, ne, sw, dinv;
};

// The row of node (i, j) depends only on which sides of the square the node
// lies on: 9 classes, class = ci + 3 cj with ci = 0 (interior column),
// 1 (i = 0), 2 (i = N) and cj likewise for rows.
__host__ __device__ inline int ka_class(int i, int j, int N) {
    return (i == 0 ? 1 : (i == N ? 2 : 0)) + 3 * (j == 0 ? 1 : (j == N ? 2 : 0));
}

template <typename T, class F>
__device__ inline T ka_apply(const KARow<T>& r, int N, int i, int j, int k, F xat) {
    const int N1 = N + 1;
    T acc = r.c * xat(i, j, k);
    if (i < N) acc += r.e * xat(i + 1, j, k + 1);
    if (i > 0) acc += r.w * xat(i - 1, j, k - 1);
    if (j < N) acc += r.n * xat(i, j + 1, k + N1);
    if (j > 0) acc += r.s * xat(i, j - 1, k - N1);
    if (i < N && j < N) acc += r.ne * xat(i + 1, j + 1, k + N1 + 1);
    if (i > 0 && j > 0) acc += r.sw * xat(i - 1, j - 1, k - N1 - 1);
    return acc;
}

// Straight-line gather of the seven values a prior row reads (an absent
// neighbour reads node k itself; its coupling is zero).
template <typename T>
struct KANb {
    T c, e, w, n, s, ne, sw;
};
template <typename T>
__device__ inline KANb<T> ka_gather(int N, int i, int j, int k, const T* __restrict__ x) {
    const int N1 = N + 1;
    const bool hE = i < N, hW = i > 0, hN = j < N, hS = j > 0;
    return KANb<T>{x[k], x[hE ? k + 1 : k], x[hW ? k - 1 : k], x[hN ? k + N1 : k], x[hS ? k - N1 : k],
                   x[hE && hN ? k + N1 + 1 : k], x[hW && hS ? k - N1 - 1 : k]};
}
// Same order of operations as ka_apply (absent neighbours add a zero product).
template <typename T>
__device__ inline T ka_combine(const KARow<T>& r, const KANb<T>& v) {
    return r.c * v.c + r.e * v.e + r.w * v.w + r.n * v.n + r.s * v.s + r.ne * v.ne + r.sw * v.sw;
}

// Row tables travel by value (kernel arguments).  Interior nodes (class 0,
// all but the boundary) read row 0 at a constant index, which the compiler
// keeps in scalar registers; only boundary nodes index the table per lane.
template <typename T>
struct OpKA {
    int N;
    KARow<T> rows[9];
    __device__ const OpKA& at(int) const { return *this; }
    __device__ bool is_free(int, int) const { return true; }
    __device__ T inv_diag(int i, int j, int) const {
        const int c = ka_class(i, j, N);
        return c == 0 ? rows[0].dinv : rows[c].dinv;
    }
    __device__ T diag(int i, int j, int) const {
        const int c = ka_class(i, j, N);
        return c == 0 ? rows[0].c : rows[c].c;
    }
    template <class F>
    __device__ T apply(int i, int j, int k, F xat) const {
        const int c = ka_class(i, j, N);
        if (c == 0) {
            // interior: all six neighbours exist
            const int N1 = N + 1;
            const KARow<T>& r = rows[0];
            return r.c * xat(i, j, k) + r.e * xat(i + 1, j, k + 1) + r.w * xat(i - 1, j, k - 1) +
                   r.n * xat(i, j + 1, k + N1) + r.s * xat(i, j - 1, k - N1) +
                   r.ne * xat(i + 1, j + 1, k + N1 + 1) + r.sw * xat(i - 1, j - 1, k - N1 - 1);
        }
        return ka_apply(rows[c], N, i, j, k, xat);
    }
    // straight-line form (see OpA): the row is the node class, its table
    // entry is read when combining
    struct Row {
        int c;
    };
    using Nb = KANb<T>;
    __device__ Row row(int i, int j, int) const { return Row{ka_class(i, j, N)}; }
    __device__ Nb gather(int i, int j, int k, const T* __restrict__ x) const { return ka_gather(N, i, j, k, x); }
    __device__ T combine(int, int, const Row& r, const Nb& v) const {
        return r.c == 0 ? ka_combine(rows[0], v) : ka_combine(rows[r.c], v);
    }
};

// Same operator reading its row table through a pointer (staged in LDS, or in
// global memory with 9 rows per stacked instance, column c -> instance c / cpi).
template <typename T>
struct OpKARef {
    int N;
    const KARow<T>* rows;
    int cpi = 0;  // 0: one instance
    __device__ OpKARef at(int c) const {
        OpKARef o = *this;
        if (cpi) o.rows += 9 * (c / cpi);
        return o;
    }
    __device__ bool is_free(int, int) const { return true; }
    __device__ T inv_diag(int i, int j, int) const { return rows[ka_class(i, j, N)].dinv; }
    __device__ T diag(int i, int j, int) const { return rows[ka_class(i, j, N)].c; }
    template <class F>
    __device__ T apply(int i, int j, int k, F xat) const {
        return ka_apply(rows[ka_class(i, j, N)], N, i, j, k, xat);
    }
    // straight-line form (see OpA): the table entry is loaded with the row
    using Row = KARow<T>;
    using Nb = KANb<T>;
    __device__ Row row(int i, int j, int) const { return rows[ka_class(i, j, N)]; }
    __device__ Nb gather(int i, int j, int k, const T* __restrict__ x) const { return ka_gather(N, i, j, k, x); }
    __device__ T combine(int, int, const Row& r, const Nb& v) const { return ka_combine(r, v); }
};

// Straight-line form of either prior operator with its 9 rows staged in LDS
// by the kernel (a boundary node then reads its row there, after its loads,
// instead of a per-lane load from kernel arguments or global memory).
template <typename T>
struct OpKALds {
    int N;
    const KARow<T>* rows;  // LDS
    struct Row {
        int c;
    };
    using Nb = KANb<T>;
    __device__ bool is_free(int, int) const { return true; }
    __device__ Row row(int i, int j, int) const { return Row{ka_class(i, j, N)}; }
    __device__ Nb gather(int i, int j, int k, const T* __restrict__ x) const { return ka_gather(N, i, j, k, x); }
    __device__ T combine(int, int, const Row& r, const Nb& v) const { return ka_combine(rows[r.c], v); }
};

// Row c (0..8) of the operator a column uses, for staging into LDS.
template <typename T>
__device__ inline KARow<T> ka_row(const OpKA<T>& o, int c) { return o.rows[c]; }
template <typename T>
__device__ inline KARow<T> ka_row(const OpKARef<T>& o, int c) { return o.rows[c]; }

// Prior operator of a level: the 9 row classes from the element matrices.
//   K_Theta: per triangle |T| grad(phi_v) . Theta grad(phi_w) with |T| = h^2/2;
//      on both triangles of a cell the gradients are (-1, 0), (1, -1), (0, 1)
//      / h (lower) and (0, -1), (-1, 1), (1, 0) / h (upper), so every
//      triangle couples its horizontal edge with (t12 - t11)/2, its vertical
//      edge with (t12 - t22)/2 and its diagonal edge with -t12/2 (Theta = I:
//      axis edges -1/2 per triangle, diagonal 0), and the rows sum to zero;
//   M: |T|/12 (1 + delta_vw) per triangle, so an axis edge adjacent to t
//      triangles couples with t h^2/24, the diagonal edge (2 triangles) with
//      h^2/12 and the diagonal is (number of incident triangles) h^2/12;
//   M_boundary: (h/6) [[2,1],[1,2]] per boundary edge.
template <typename T>
inline OpKA<T> make_prior_op(int N, const PriorParams& pp) {
    const double g = pp.gamma, dl = pp.delta, bt = pp.beta;
    const double kh = 0.5 * (pp.t12 - pp.t11), kv = 0.5 * (pp.t12 - pp.t22), kd = -pp.t12;  // K couplings
    OpKA<T> o;
    o.N = N;
    const double h = 1.0 / N, h2 = h * h;
    const int reps_i[3] = {N / 2, 0, N}, reps_j[3] = {N / 2, 0, N};
    for (int cj = 0; cj < 3; ++cj)
        for (int ci = 0; ci < 3; ++ci) {
            const int i = reps_i[ci], j = reps_j[cj];
            const int hasE = i < N, hasW = i > 0, hasN = j < N, hasS = j > 0;
            const int jin = (j < N) + (j > 0);  // triangles on a horizontal edge at row j
            const int iin = (i < N) + (i > 0);  // triangles on a vertical edge at column i
            const int bh = (j == 0 || j == N);  // horizontal edges at row j are boundary edges
            const int bv = (i == 0 || i == N);  // vertical edges at column i are boundary edges
            const int ne = hasE && hasN, sw = hasW && hasS;  // diagonal edges (2 triangles each)
            const double eh = g * kh * jin + dl * jin * h2 / 24.0 + bt * (h / 6.0) * bh;
            const double ev = g * kv * iin + dl * iin * h2 / 24.0 + bt * (h / 6.0) * bv;
            const double ed = g * kd + dl * h2 / 12.0;
            const int ntri = 2 * ne + (hasW && hasN) + (hasE && hasS) + 2 * sw;
            const int nbe = bh * (hasE + hasW) + bv * (hasN + hasS);
            // K_Theta's diagonal: minus its couplings (zero row sums)
            const double cK = -(kh * jin * (hasE + hasW) + kv * iin * (hasN + hasS) + kd * (ne + sw));
            const double c = g * cK + dl * ntri * h2 / 12.0 + bt * (h / 3.0) * nbe;
            KARow<T>& r = o.rows[ci + 3 * cj];
            r.c = (T)c;
            r.e = (T)(hasE ? eh : 0.0);
            r.w = (T)(hasW ? eh : 0.0);
            r.n = (T)(hasN ? ev : 0.0);
            r.s = (T)(hasS ? ev : 0.0);
            r.ne = (T)(ne ? ed : 0.0);
            r.sw = (T)(sw ? ed : 0.0);
            r.dinv = (T)(1.0 / c);
        }
    return o;
}

// ---------------------------------------------------------- tile stencil ---
// Both operators are symmetric with couplings to the east, north and (prior
// only) north-east neighbours, so an LDS tile of either is five arrays per
// node: diagonal c, east e, north n, north-east g and 1/diagonal dv, with
//   (A x)_l = c_l x_l + e_l x_{l+1} + e_{l-1} x_{l-1} + n_l x_{l+TW} + n_{l-TW} x_{l-TW}
//             + g_l x_{l+TW+1} + g_{l-TW-1} x_{l-TW-1}
// (l = local index, TW = tile width).  Absent neighbours carry zero
// couplings, nodes outside the mesh are zero everywhere, and dv is zero on
// Dirichlet rows, so the tile stencil needs no boundary branches: the vectors
// it is applied to are zero on Dirichlet rows.
template <class Op>
constexpr bool kNorthEast = true;  // the prior operator couples (i+1, j+1)
template <typename T>
constexpr bool kNorthEast<OpA<T>> = false;

template <typename T>
struct TileStencil {
    T* c;   // unused (size 1) for the state operator: see tile_center
    T* e;
    T* n;
    T* g;   // unused (size 1) for the state operator
    T* dv;
};

// Stages the rows of the TW x TW tile whose local (0, 0) is node (ox, oy),
// NT threads.  Every global load of a thread is issued before its first LDS
// store, so the load latencies of its NT-strided elements overlap.
// The state operator stages its two edge weights and 1/d per node; the
// diagonal is summed from the staged weights of the node and of its west and
// south neighbours where it is used (tile_center), so no diagonal array is
// staged (three loads a node instead of five, one LDS array fewer).
template <int TW, int NT, typename T>
__device__ inline void stage_stencil(const OpA<T>& op, const TileStencil<T>& s, int ox, int oy) {
    constexpr int NN = TW * TW, E = (NN + NT - 1) / NT;
    const int N = op.N, N1 = N + 1;
    T we[E], wn[E], dv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int t = threadIdx.x + e * NT;
        const int i = ox + t % TW, j = oy + t / TW;
        const bool in = t < NN && i >= 0 && i <= N && j >= 0 && j <= N;
        const int k = j * N1 + i;
        we[e] = in ? op.wE[k] : (T)0;
        wn[e] = in ? op.wN[k] : (T)0;
        dv[e] = in ? op.dinv[k] : (T)0;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int t = threadIdx.x + e * NT;
        if (t < NN) {
            s.e[t] = -we[e];
            s.n[t] = -wn[e];
            s.dv[t] = dv[e];
        }
    }
}

template <int TW, int NT, typename T, class OpK>
__device__ inline void stage_stencil(const OpK& op, const TileStencil<T>& s, int ox, int oy) {
    constexpr int NN = TW * TW, E = (NN + NT - 1) / NT;
    const int N = op.N;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int t = threadIdx.x + e * NT;
        if (t >= NN) break;
        const int i = ox + t % TW, j = oy + t / TW;
        T c = 0, ee = 0, n = 0, g = 0, dv = 0;
        if (i >= 0 && i <= N && j >= 0 && j <= N) {
            const KARow<T>& r = op.rows[ka_class(i, j, N)];
            c = r.c;
            ee = r.e;
            n = r.n;
            g = r.ne;
            dv = r.dinv;
        }
        s.c[t] = c;
        s.e[t] = ee;
        s.n[t] = n;
        s.g[t] = g;
        s.dv[t] = dv;
    }
}

// Identifies the problem instance an operator belongs to (stacked
// hierarchies): a staged tile is reused while the key stays the same.
template <typename T>
__device__ inline const void* instance_key(const OpA<T>& o) { return o.wE; }
template <typename T>
__device__ inline const void* instance_key(const OpKARef<T>& o) { return o.rows; }
template <typename T>
__device__ inline const void* instance_key(const OpKA<T>&) { return reinterpret_cast<const void*>(1); }

// The prior operator on a tile through its 9-row class table (staged in LDS)
// instead of per-node staged rows: the coefficients of a node depend only on
// which sides of the square it lies on, so a tile of interior nodes uses row 0
// throughout, and a tile at the boundary computes each node's class.  Same
// couplings in the same order as the staged form: a node's own c, e, n, ne,
// its west neighbour's e, its south neighbour's n and its south-west
// neighbour's ne (zero for nodes outside the mesh).
template <typename T, int TW>
struct TileKA {
    const KARow<T>* rows;
    int ox, oy, N;
    bool interior;  // every node of the tile has class 0
    __device__ int cls(int l) const {
        const int i = ox + l % TW, j = oy + l / TW;
        if (i < 0 || i > N || j < 0 || j > N) return -1;
        return ka_class(i, j, N);
    }
    __device__ T dinv(int l) const {
        if (interior) return rows[0].dinv;
        const int c = cls(l);
        return c < 0 ? (T)0 : rows[c].dinv;
    }
    __device__ T center(int l) const {
        if (interior) return rows[0].c;
        const int c = cls(l);
        return c < 0 ? (T)0 : rows[c].c;
    }
    __device__ T apply(int l, const T* v) const {
        if (interior) {
            const KARow<T>& r = rows[0];
            return r.c * v[l] + r.e * v[l + 1] + r.e * v[l - 1] + r.n * v[l + TW] + r.n * v[l - TW] +
                   r.ne * v[l + TW + 1] + r.ne * v[l - TW - 1];
        }
        const int c0 = cls(l), cw = cls(l - 1), cs = cls(l - TW), csw = cls(l - TW - 1);
        const KARow<T> z{};
        const KARow<T>& r = c0 < 0 ? z : rows[c0];
        const T ew = cw < 0 ? (T)0 : rows[cw].e;
        const T ns = cs < 0 ? (T)0 : rows[cs].n;
        const T gsw = csw < 0 ? (T)0 : rows[csw].ne;
        return r.c * v[l] + r.e * v[l + 1] + ew * v[l - 1] + r.n * v[l + TW] + ns * v[l - TW] + r.ne * v[l + TW + 1] +
               gsw * v[l - TW - 1];
    }
};

// Diagonal of row l on a staged tile (l must have its west and south
// neighbours inside the tile): the prior operator's staged value; for the
// state operator the sum w_E + w_N + w_W + w_S of the four incident edge
// weights, in that order (off the mesh, and for absent edges, the staged
// weights are zero).
template <bool NE, typename T>
__device__ inline T tile_center(const TileStencil<T>& s, int TW, int l) {
    if constexpr (NE) return s.c[l];
    else return -s.e[l] + -s.n[l] + -s.e[l - 1] + -s.n[l - TW];
}

// (A v)_l with row r at every node (a tile of interior prior-operator
// nodes), in the operation order of tile_apply<true> on staged rows.
template <typename T>
__device__ inline T row_apply(const KARow<T>& r, int TW, int l, const T* v) {
    T a = r.c * v[l] + r.e * v[l + 1] + r.e * v[l - 1] + r.n * v[l + TW] + r.n * v[l - TW];
    a += r.ne * v[l + TW + 1] + r.ne * v[l - TW - 1];
    return a;
}

// (A v)_l on a staged tile; l must have all eight neighbours inside the tile.
template <bool NE, typename T>
__device__ inline T tile_apply(const TileStencil<T>& s, int TW, int l, const T* v) {
    T a = tile_center<NE>(s, TW, l) * v[l] + s.e[l] * v[l + 1] + s.e[l - 1] * v[l - 1] + s.n[l] * v[l + TW] +
          s.n[l - TW] * v[l - TW];
    if constexpr (NE) a += s.g[l] * v[l + TW + 1] + s.g[l - TW - 1] * v[l - TW - 1];
    return a;
}

// ------------------------------------------------------------ triangles ---
// Node indices (a, r, b) of triangle s (0 lower, 1 upper) of cell (ci, cj).
__device__ inline void tri_nodes(int N, int ci, int cj, int s, int& ka, int& kr, int& kb) {
    ka = knode(ci, cj, N);
    kb = knode(ci + 1, cj + 1, N);
    kr = s == 0 ? knode(ci + 1, cj, N) : knode(ci, cj + 1, N);
}

// Unit-coefficient element bilinear form |T| grad v . grad w on a right
// triangle with legs h, in (a, r, b) order:
// 1/2 [(v_a - v_r)(w_a - w_r) + (v_r - v_b)(w_r - w_b)].
__device__ inline double tri_form(double va, double vr, double vb, double wa, double wr,
                                  double wb) {
    return 0.5 * ((va - vr) * (wa - wr) + (vr - vb) * (wr - wb));
}

// Visits the (up to 6) triangles incident to node (i, j): f(ci, cj, s, role)
// with role 0/1/2 = the node is vertex a/r/b of the triangle.
template <class F>
__device__ inline void for_incident_triangles(int N, int i, int j, F f) {
    if (i < N && j < N) {
        f(i, j, 0, 0);
        f(i, j, 1, 0);
    }
    if (i > 0 && j < N) f(i - 1, j, 0, 1);  // lower of cell (i-1, j): r = (i, j)
    if (i < N && j > 0) f(i, j - 1, 1, 1);  // upper of cell (i, j-1): r = (i, j)
    if (i > 0 && j > 0) {
        f(i - 1, j - 1, 0, 2);
        f(i - 1, j - 1, 1, 2);
    }
}

}  // namespace hinv
