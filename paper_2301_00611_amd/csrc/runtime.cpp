// runtime.cpp -- host side of libdem_hip.so: scene/world management, device
// buffers, the broad-phase run (host-orchestrated, a few small read-backs),
// the stepping loop (HIP graphs of `chunk` steps that stop themselves when a
// broad-phase run is needed), read-back and the extern "C" API of dem.h.
//
// A World holds one or more independent scenes in one set of arrays: bodies
// of all scenes live in one structure-of-arrays arena and are advanced by
// the same kernels; each body carries its scene index (batched mode only).
// Internally every body (wall or sphere) of the world has a global index
// (gid); each scene maps its own ids (0, 1, ... in insertion order) to gids.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <fstream>
#include <sstream>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "dem_internal.hpp"

namespace dem {
namespace {

thread_local std::string g_err;

struct Error {
    dem_status code;
    std::string msg;
};

[[noreturn]] void fail(dem_status code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess) fail(DEM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPC(x) ::dem::hip_check((x), #x)

// Growable device allocation.
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void ensure(size_t need)
    {
        if (need <= bytes && p) return;
        size_t nb = std::max<size_t>(need + need / 2, 256);
        void* q = nullptr;
        if (hipMalloc(&q, nb) != hipSuccess) fail(DEM_ENOMEM, "device allocation of " + std::to_string(nb) + " bytes failed");
        if (p) (void)hipFree(p);
        p = q;
        bytes = nb;
    }
    // grow keeping the first `keep` bytes
    void ensure_keep(size_t need, size_t keep, hipStream_t st)
    {
        if (need <= bytes && p) return;
        size_t nb = std::max<size_t>(need + need / 2, 256);
        void* q = nullptr;
        if (hipMalloc(&q, nb) != hipSuccess) fail(DEM_ENOMEM, "device allocation failed");
        if (p && keep) HIPC(hipMemcpyAsync(q, p, std::min(keep, bytes), hipMemcpyDeviceToDevice, st));
        if (p) {
            HIPC(hipStreamSynchronize(st));
            (void)hipFree(p);
        }
        p = q;
        bytes = nb;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

struct BodySet {
    DBuf xr, vm, w, q, mat, blocked, id, scene, period;
    void ensure(size_t n)
    {
        for (DBuf* b : {&xr, &vm, &w, &q}) b->ensure(n * sizeof(double4));
        mat.ensure(n * 2);
        blocked.ensure(n);
        id.ensure(n * 4);
        scene.ensure(n * 2);
        period.ensure(n * 4);
    }
    Bodies view() const
    {
        Bodies b;
        b.xr = xr.as<double4>();
        b.vm = vm.as<double4>();
        b.w = w.as<double4>();
        b.q = q.as<double4>();
        b.mat = mat.as<uint16_t>();
        b.blocked = blocked.as<uint8_t>();
        b.id = id.as<int32_t>();
        b.scene = scene.as<uint16_t>();
        b.period = period.as<int32_t>();
        return b;
    }
    void release()
    {
        for (DBuf* b : {&xr, &vm, &w, &q, &mat, &blocked, &id, &scene, &period}) b->release();
    }
};

// A growable pinned host buffer: a device-to-host copy into it is one DMA
// transfer (pageable memory is copied through a staging buffer, piece by
// piece, each piece waited for).
struct HBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void ensure(size_t need)
    {
        if (need <= bytes && p) return;
        size_t nb = std::max<size_t>(need + need / 2, 256);
        void* q = nullptr;
        if (hipHostMalloc(&q, nb, hipHostMallocDefault) != hipSuccess)
            fail(DEM_ENOMEM, "pinned host allocation of " + std::to_string(nb) + " bytes failed");
        if (p) (void)hipHostFree(p);
        p = q;
        bytes = nb;
    }
    void release()
    {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T* as() const
    {
        return static_cast<T*>(p);
    }
};

struct PairSet {
    DBuf a, b, cell, pid, real, ea, eb, hist, frec;  // partitioned order (touching pairs first)
    DBuf hpid, hcell, hmap;                     // canonical (owner-sorted) order, for the next run's lookup
    DBuf own_begin, own_count;  // by gid, into the canonical order
    size_t cap = 0;
    void ensure(size_t n, bool fp32)
    {
        n = std::max<size_t>(n, 1);
        for (DBuf* d : {&a, &b, &cell, &pid, &ea, &eb, &hpid, &hcell, &hmap}) d->ensure(n * 4);
        real.ensure(n);
        hist.ensure(n * hist_bytes(fp32 ? DEM_FP32_MIXED : DEM_FP64));
        frec.ensure(n * kForceWords * (fp32 ? sizeof(float) : sizeof(double)));
        cap = n;
    }
    Pairs view() const
    {
        Pairs p;
        p.a = a.as<int32_t>();
        p.b = b.as<int32_t>();
        p.cell = cell.as<int32_t>();
        p.pid = pid.as<int32_t>();
        p.real = real.as<uint8_t>();
        p.ea = ea.as<int32_t>();
        p.eb = eb.as<int32_t>();
        p.h = hist.as<HistRec>();
        p.frec = frec.as<double>();
        p.frecf = frec.as<float>();
        return p;
    }
    History history() const
    {
        History h;
        h.own_begin = own_begin.as<int32_t>();
        h.own_count = own_count.as<int32_t>();
        h.pid = hpid.as<int32_t>();
        h.cell = hcell.as<int32_t>();
        h.map = hmap.as<int32_t>();
        h.h = hist.as<HistRec>();
        return h;
    }
    void release()
    {
        for (DBuf* d : {&a, &b, &cell, &pid, &real, &ea, &eb, &hist, &frec, &hpid, &hcell, &hmap, &own_begin,
                        &own_count})
            d->release();
        cap = 0;
    }
};

// kind 0: FrictMat; kind 1: ViscElMat given by contact time and restitution
// coefficients (young and poisson then hold the class's defaults, used only by
// the P-wave step)
struct HostMaterial {
    double density, young, poisson, friction;
    int kind = 0;
    double tc = 0.0, en = 0.0, et = 0.0;
};

struct HostScene {
    dem_params p;
    std::vector<int32_t> gids;  // local id -> gid
    int64_t n_spheres = 0, n_walls = 0;
    int64_t iter = 0;
    double time = 0.0;
    double verlet = 0.0;        // Delta L in use
    double rmax = 0.0;          // largest radius at the last broad-phase run
    double r_lo = INFINITY;     // smallest and largest sphere radius (radii never change)
    double r_hi = 0.0;
    // two-level grid: radii above r_split go on the coarse level (0 = one
    // level), n_large of them
    double r_split = 0.0;
    int64_t n_large = 0;
};

// Host copy of everything per gid (kept in step only when bodies are added
// or the state is overwritten; the device holds the truth while stepping).
struct HostBody {
    int kind;  // 0 sphere, 1 wall
    int scene;
    int wall;  // wall index when kind == 1
    double x[3], v[3], w[3], q[4];
    double r, m;
    int mat;
    uint8_t blocked;
};

struct KernelTimer {
    double total_ms = 0.0;
    int64_t launches = 0;
};

struct World {
    // asynchronous stepping: while `busy` is set every call but dem_wait is
    // refused; the worker's outcome is handed to dem_wait
    std::thread worker;
    std::atomic<int> busy{0};
    dem_status async_rc = DEM_OK;
    std::string async_msg;

    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int precision = DEM_FP64;
    bool periodic = false;
    bool track_energy = false;
    std::vector<HostScene> scenes;
    std::vector<HostMaterial> mats;
    std::vector<Wall> walls;           // global wall table (ordered by scene)
    std::vector<int> wall_scene;
    std::vector<HostBody> bodies;      // by gid (authoritative only while host_dirty)
    bool host_dirty = false;           // bodies added / state set: upload before stepping
    bool on_device = false;            // device arrays hold the current state
    bool need_rebuild = true;
    bool contacts_valid = false;

    // device
    BodySet bs[2];
    int active = 0;
    PairSet ps[2];
    int pactive = 0;
    int npairs = 0;
    int nslots = 0;
    int ngids_dev = 0;                 // number of gids the device arrays were built for
    int old_ngids = 0;                 // gids covered by the active own arrays
    DBuf slot_of_id, keys, vals, keys_alt, vals_alt, cell_start, cell_end, counts, row_start;
    DBuf ent_slot, ent_pid, ent_cell, ent_own, own_scan, rows_ent, scan_tmp, radix_tmp;
    DBuf d_ve;
    DBuf d_scenes, d_walls, d_mats, d_tanphi, d_ctr, d_part_c, d_part_i, d_bounds, d_total, d_tmp3, d_args;
    DBuf d_ctrl_cfg, d_ctrl_state, d_acc_ctrl, d_acc_ctrl2;  // the controlled cell (device-resident)
    DBuf pb_ca, pb_cb, pb_found, pb_flag, pb_scan;  // pair build scratch (canonical order)
    int grid_c = 1, grid_i = 1;        // step-kernel grids (contact sized with headroom)
    int acc_c_n = 0, acc_i_n = 0;      // slots currently in use in d_part_c / d_part_i
    int next_parity = 0;               // parity of the next step (stall flags alternate)
    // running sums folded from the per-block slots (fixed block order)
    double base_plast = 0.0, base_grav = 0.0, base_damp = 0.0, base_visc = 0.0;
    unsigned long long base_contact_steps = 0;
    // last-step values kept across a fold until the next step runs
    double last_el = 0.0, last_kin = 0.0, last_rot = 0.0;
    unsigned long long last_ss = 0, last_sw = 0;
    bool slots_fresh = true;           // no step has written the slots since the last fold
    std::vector<SceneParams> sp;       // host copy of the scene table
    Counters* h_ctr = nullptr;         // pinned
    HBuf h_slots_c, h_slots_i;         // the per-block slots as read back
    // pinned: what the host writes into the counters before a launch chain
    // (steps_done = 0, halt = 0, iter0), the 16 bytes from steps_done on
    struct ChunkStart {
        int32_t steps_done, halt;
        int64_t iter0;
    };
    ChunkStart* h_chunk = nullptr;
    int ncells = 0;
    DBuf d_flag;                       // broad phase: a body's period out of the packed range
    DBuf lflag, lscan, keys2, vals2, keys2_alt, vals2_alt;  // level 1 of a two-level grid
    DBuf raw_slot, raw_pid, raw_cell, ent_body;              // row entries in the order found, and their rows
    int morton_bits = 1, scene_bits = 0;
    int64_t rebuilds = 0;
    int64_t iter_at_rebuild = 0;       // scene 0's iteration count at the last broad-phase run
    double last_rebuild_ms = 0.0;      // wall time of the last broad-phase run
    double rebuild_ms_total = 0.0;
    DBuf d_acct;
    int64_t n_candidates = 0;
    int block_contact = 256, block_integrate = 256;
    int chunk = 32;
    double tuned_ms = 0.0;             // ms per step measured by the autotuner
    bool use_graph = true;

    // graphs
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;
        std::vector<hipEvent_t> ev;
    };
    std::map<std::string, GraphEntry> graphs;

    // timing
    bool timing = false;
    std::map<std::string, KernelTimer> timers;

    ~World()
    {
        if (worker.joinable()) worker.join();
        release();
    }
    void release()
    {
        for (auto& kv : graphs) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            for (auto e : kv.second.ev) (void)hipEventDestroy(e);
        }
        graphs.clear();
        for (auto& b : bs) b.release();
        for (auto& p : ps) p.release();
        for (DBuf* d : {&slot_of_id, &keys, &vals, &keys_alt, &vals_alt, &cell_start, &cell_end, &counts, &row_start,
                        &ent_slot, &ent_pid, &ent_cell, &ent_own, &own_scan, &rows_ent, &scan_tmp, &radix_tmp,
                        &d_scenes, &d_walls, &d_mats, &d_tanphi, &d_ctr, &d_part_c, &d_part_i, &d_bounds, &d_total,
                        &d_tmp3, &d_args, &d_ctrl_cfg, &d_ctrl_state, &d_acc_ctrl, &d_acc_ctrl2, &pb_ca, &pb_cb, &pb_found,
                        &pb_flag, &pb_scan, &d_flag, &lflag, &lscan, &keys2, &vals2, &keys2_alt, &vals2_alt, &raw_slot, &raw_pid,
                        &raw_cell, &ent_body, &d_acct})
            d->release();
        if (h_ctr) (void)hipHostFree(h_ctr);
        h_ctr = nullptr;
        h_slots_c.release();
        h_slots_i.release();
        if (h_chunk) (void)hipHostFree(h_chunk);
        h_chunk = nullptr;
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
    }

    bool batched() const { return scenes.size() > 1; }
    // a box or a facet among the boundaries: the contact kernel with their geometry
    bool has_prims() const
    {
        for (const Wall& w : walls)
            if (w.kind != kPlane) return true;
        return false;
    }

    void invalidate_graphs()
    {
        for (auto& kv : graphs) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            for (auto e : kv.second.ev) (void)hipEventDestroy(e);
        }
        graphs.clear();
    }

    // ------------------------------------------------------------ setup
    void init(int nsc, const dem_params* p)
    {
        device = p[0].device;
        HIPC(hipSetDevice(device));
        if (p[0].stream) {
            stream = static_cast<hipStream_t>(p[0].stream);
        } else {
            HIPC(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
            own_stream = true;
        }
        precision = p[0].precision;
        periodic = p[0].periodic != 0;
        track_energy = p[0].track_energy != 0;
        scenes.resize(nsc);
        for (int i = 0; i < nsc; ++i) scenes[i].p = p[i];
        HIPC(hipHostMalloc(reinterpret_cast<void**>(&h_ctr), sizeof(Counters), hipHostMallocDefault));
        std::memset(h_ctr, 0, sizeof(Counters));
        d_ctr.ensure(sizeof(Counters));
        HIPC(hipMemsetAsync(d_ctr.p, 0, sizeof(Counters), stream));
        static_assert(offsetof(Counters, halt) == offsetof(Counters, steps_done) + 4 &&
                          offsetof(Counters, iter0) == offsetof(Counters, steps_done) + 8,
                      "the chunk-start fields are contiguous");
        HIPC(hipHostMalloc(reinterpret_cast<void**>(&h_chunk), sizeof(ChunkStart), hipHostMallocDefault));
        std::memset(h_chunk, 0, sizeof(ChunkStart));
        d_ctrl_cfg.ensure(sizeof(CtrlConfig));
        d_ctrl_state.ensure(sizeof(CtrlState));
        HIPC(hipMemsetAsync(d_ctrl_cfg.p, 0, sizeof(CtrlConfig), stream));
        HIPC(hipMemsetAsync(d_ctrl_state.p, 0, sizeof(CtrlState), stream));
        sp.resize(nsc);
        for (int i = 0; i < nsc; ++i) {
            SceneParams& s = sp[i];
            std::memset(&s, 0, sizeof s);
            const dem_params& q = p[i];
            s.dt = q.dt;
            for (int k = 0; k < 3; ++k) s.gravity[k] = q.gravity[k];
            s.damping = q.damping;
            s.damp_rot = q.damp_rot;
            s.homo_deform = q.homo_deform;
            s.periodic = q.periodic;
            for (int k = 0; k < 9; ++k) {
                s.H[k] = q.periodic ? q.hsize[k] : (k % 4 == 0 ? 1.0 : 0.0);
                s.L[k] = q.periodic ? q.velgrad[k] : 0.0;
                s.trsf[k] = (k % 4 == 0 ? 1.0 : 0.0);
            }
            if (q.periodic) invert(s.H, s.Hinv);
        }
        d_scenes.ensure(sizeof(SceneParams) * nsc);
        HIPC(hipMemcpyAsync(d_scenes.p, sp.data(), sizeof(SceneParams) * nsc, hipMemcpyHostToDevice, stream));
        HIPC(hipStreamSynchronize(stream));
        if (const char* c = std::getenv("DEM_CHUNK")) chunk = std::max(1, std::atoi(c));
        if (const char* g = std::getenv("DEM_NO_GRAPH")) use_graph = std::atoi(g) == 0;
    }

    static bool invert(const double* M, double* out)
    {
        const double a = M[0], b = M[1], c = M[2], d = M[3], e = M[4], f = M[5], g = M[6], h = M[7], i = M[8];
        const double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
        const double det = a * A + b * B + c * C;
        if (!(std::fabs(det) > 0.0)) return false;
        out[0] = A / det;
        out[1] = -(b * i - c * h) / det;
        out[2] = (b * f - c * e) / det;
        out[3] = B / det;
        out[4] = (a * i - c * g) / det;
        out[5] = -(a * f - c * d) / det;
        out[6] = C / det;
        out[7] = -(a * h - b * g) / det;
        out[8] = (a * e - b * d) / det;
        return true;
    }

    int add_material(double density, double young, double poisson, double friction)
    {
        if (!(density > 0.0) || !(young > 0.0) || !(poisson > -1.0 && poisson <= 0.5) ||
            !(friction >= 0.0 && friction < 1.5707963267948966))
            fail(DEM_EINVAL, "dem_add_material: need density > 0, young > 0, -1 < poisson <= 0.5, 0 <= friction < pi/2");
        if (mats.size() >= 1024) fail(DEM_EINVAL, "dem_add_material: at most 1024 materials");
        HostMaterial m;
        m.density = density;
        m.young = young;
        m.poisson = poisson;
        m.friction = friction;
        mats.push_back(m);
        upload_materials();
        return (int)mats.size() - 1;
    }
    int add_viscel_material(double density, double tc, double en, double et, double friction)
    {
        if (!(tc > 0.0) || !std::isfinite(tc) || !(en > 0.0 && en <= 1.0) || !(et > 0.0 && et <= 1.0))
            fail(DEM_EINVAL, "dem_add_viscel_material: need tc > 0 and restitution coefficients in (0, 1]");
        const int id = add_material(density, 1e9, 0.25, friction);
        mats[id].kind = 1;
        mats[id].tc = tc;
        mats[id].en = en;
        mats[id].et = et;
        upload_materials();
        return id;
    }
    bool has_viscel() const
    {
        for (const HostMaterial& m : mats)
            if (m.kind == 1) return true;
        return false;
    }
    // The laws pair materials of one kind: a scene whose bodies mix FrictMat
    // and ViscElMat has no law for some pairs and is refused at its next step.
    bool kinds_checked = false;
    void check_material_kinds()
    {
        if (kinds_checked || !has_viscel()) return;
        std::vector<int> kind(scenes.size(), -1);
        for (const HostBody& b : bodies) {
            const int k = mats[b.mat].kind;
            int& sk = kind[b.scene];
            if (sk >= 0 && sk != k) fail(DEM_EINVAL, "dem_step: bodies of elastic and visco-elastic materials in one scene");
            sk = k;
        }
        kinds_checked = true;
    }

    void upload_materials()
    {
        const int n = (int)mats.size();
        std::vector<Material> m(n);
        std::vector<double> tp((size_t)n * n);
        std::vector<ViscElPair> ve((size_t)n * n);
        for (int i = 0; i < n; ++i) {
            std::memset(&m[i], 0, sizeof m[i]);
            m[i].young = mats[i].young;
            m[i].young_poisson = mats[i].young * mats[i].poisson;
            m[i].density = mats[i].density;
            m[i].viscel = mats[i].kind == 1 ? 1 : 0;
            for (int j = 0; j < n; ++j) {
                tp[(size_t)i * n + j] = std::tan(mats[i].friction < mats[j].friction ? mats[i].friction : mats[j].friction);
                // the pair's tc and restitution coefficients: the means of the two materials'
                ViscElPair& P = ve[(size_t)i * n + j];
                std::memset(&P, 0, sizeof P);
                if (mats[i].kind == 1 && mats[j].kind == 1) {
                    P.tc = 0.5 * (mats[i].tc + mats[j].tc);
                    P.len = std::log(0.5 * (mats[i].en + mats[j].en));
                    P.let = std::log(0.5 * (mats[i].et + mats[j].et));
                }
            }
        }
        d_mats.ensure(sizeof(Material) * std::max(n, 1));
        d_tanphi.ensure(sizeof(double) * std::max(n * n, 1));
        d_ve.ensure(sizeof(ViscElPair) * std::max(n * n, 1));
        HIPC(hipMemcpyAsync(d_mats.p, m.data(), sizeof(Material) * n, hipMemcpyHostToDevice, stream));
        HIPC(hipMemcpyAsync(d_tanphi.p, tp.data(), sizeof(double) * n * n, hipMemcpyHostToDevice, stream));
        HIPC(hipMemcpyAsync(d_ve.p, ve.data(), sizeof(ViscElPair) * n * n, hipMemcpyHostToDevice, stream));
        HIPC(hipStreamSynchronize(stream));
        if (d_args.p) upload_args();
    }

    // Bring the host copy up to date with the device (before adding bodies).
    void pull_bodies()
    {
        if (!on_device || host_dirty) return;
        std::vector<double> buf(4 * (size_t)nslots);
        std::vector<int32_t> ids((size_t)nslots);
        const BodySet& B = bs[active];
        HIPC(hipMemcpyAsync(ids.data(), B.id.p, 4 * (size_t)nslots, hipMemcpyDeviceToHost, stream));
        HIPC(hipStreamSynchronize(stream));
        // packed 4-vectors: component c of slot i is buf[4 i + c]
        auto pull = [&](const DBuf& d, double* (*field)(HostBody&), int ncomp) {
            HIPC(hipMemcpyAsync(buf.data(), d.p, 32 * (size_t)nslots, hipMemcpyDeviceToHost, stream));
            HIPC(hipStreamSynchronize(stream));
            for (int i = 0; i < nslots; ++i) {
                double* dst = field(bodies[ids[i]]);
                for (int c = 0; c < ncomp; ++c) dst[c] = buf[4 * (size_t)i + c];
            }
        };
        pull(B.xr, [](HostBody& b) { return b.x; }, 3);
        pull(B.vm, [](HostBody& b) { return b.v; }, 3);
        pull(B.w, [](HostBody& b) { return b.w; }, 3);
        pull(B.q, [](HostBody& b) { return b.q; }, 4);
    }

    int64_t add_spheres(int s, int64_t n, const double* pos3, const double* radius, const double* vel3,
                        const double* angvel3, const int32_t* mat, int32_t default_mat, const uint8_t* blocked)
    {
        if (n < 0 || (n > 0 && (!pos3 || !radius))) fail(DEM_EINVAL, "dem_add_spheres: need pos3 and radius");
        kinds_checked = false;
        for (int64_t i = 0; i < n; ++i) {
            const int mi = mat ? mat[i] : default_mat;
            if (mi < 0 || mi >= (int)mats.size()) fail(DEM_EINVAL, "dem_add_spheres: unknown material");
            if (!(radius[i] > 0.0) || !std::isfinite(radius[i])) fail(DEM_EINVAL, "dem_add_spheres: radius must be > 0");
            for (int k = 0; k < 3; ++k)
                if (!std::isfinite(pos3[3 * i + k])) fail(DEM_EINVAL, "dem_add_spheres: non-finite position");
        }
        if ((int64_t)bodies.size() + n > 0x7ffffff0LL) fail(DEM_EINVAL, "dem_add_spheres: too many bodies");
        pull_bodies();
        HostScene& S = scenes[s];
        const int64_t first = (int64_t)S.gids.size();
        for (int64_t i = 0; i < n; ++i) {
            HostBody b;
            std::memset(&b, 0, sizeof b);
            b.kind = 0;
            b.scene = s;
            b.mat = mat ? mat[i] : default_mat;
            b.r = radius[i];
            for (int k = 0; k < 3; ++k) {
                b.x[k] = pos3[3 * i + k];
                b.v[k] = vel3 ? vel3[3 * i + k] : 0.0;
                b.w[k] = angvel3 ? angvel3[3 * i + k] : 0.0;
            }
            b.q[0] = 1.0;
            b.blocked = blocked ? (uint8_t)(blocked[i] & 63u) : 0;
            const double rho = mats[b.mat].density;
            const double r = b.r;
            b.m = 4.0 / 3.0 * M_PI * r * r * r * rho;
            S.r_lo = std::min(S.r_lo, r);
            S.r_hi = std::max(S.r_hi, r);
            S.gids.push_back((int32_t)bodies.size());
            bodies.push_back(b);
        }
        S.n_spheres += n;
        split_levels(s);
        host_dirty = true;
        need_rebuild = true;
        return first;
    }

    // Size ratio above 2.5: two grid levels, split at the largest radius not
    // above half the largest (small spheres then search cells sized for
    // themselves, and the large ones search both levels); else one level.
    void split_levels(int s)
    {
        HostScene& S = scenes[s];
        S.r_split = 0.0;
        S.n_large = 0;
        if (!(S.r_hi > 2.5 * S.r_lo)) return;
        double rs = 0.0;
        for (int32_t g : S.gids) {
            const HostBody& b = bodies[g];
            if (b.kind == 0 && b.r <= 0.5 * S.r_hi) rs = std::max(rs, b.r);
        }
        int64_t nl = 0;
        for (int32_t g : S.gids)
            if (bodies[g].kind == 0 && bodies[g].r > rs) ++nl;
        S.r_split = rs;
        S.n_large = nl;
    }

    int64_t add_wall(int s, int axis, double position, int sense, int mat)
    {
        if (axis < 0 || axis > 2 || sense < -1 || sense > 1 || !std::isfinite(position))
            fail(DEM_EINVAL, "dem_add_wall: axis in 0..2, sense in -1..1, finite position");
        Wall w;
        std::memset(&w, 0, sizeof w);
        w.kind = kPlane;
        w.axis = axis;
        w.sense = sense;
        w.pos = position;
        return add_boundary(s, w, mat, "dem_add_wall");
    }
    int64_t add_box(int s, const double* c3, const double* h3, int mat)
    {
        if (!c3 || !h3) fail(DEM_EINVAL, "dem_add_box: null argument");
        Wall w;
        std::memset(&w, 0, sizeof w);
        w.kind = kBox;
        for (int k = 0; k < 3; ++k) {
            if (!std::isfinite(c3[k]) || !(h3[k] > 0.0) || !std::isfinite(h3[k]))
                fail(DEM_EINVAL, "dem_add_box: finite centre and half-sizes > 0");
            w.g[k] = c3[k] - h3[k];
            w.g[3 + k] = c3[k] + h3[k];
        }
        return add_boundary(s, w, mat, "dem_add_box");
    }
    int64_t add_facet(int s, const double* v0, const double* v1, const double* v2, int mat)
    {
        if (!v0 || !v1 || !v2) fail(DEM_EINVAL, "dem_add_facet: null argument");
        Wall w;
        std::memset(&w, 0, sizeof w);
        w.kind = kFacet;
        const double* v[3] = {v0, v1, v2};
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) {
                if (!std::isfinite(v[i][k])) fail(DEM_EINVAL, "dem_add_facet: non-finite vertex");
                w.g[3 * i + k] = v[i][k];
            }
        const double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
        const double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
        const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        if (!((c[0] * c[0] + c[1] * c[1]) + c[2] * c[2] > 0.0)) fail(DEM_EINVAL, "dem_add_facet: degenerate triangle");
        return add_boundary(s, w, mat, "dem_add_facet");
    }
    // A fixed boundary (plane, box, facet) of scene s.
    int64_t add_boundary(int s, Wall w, int mat, const char* who)
    {
        if (mat < 0 || mat >= (int)mats.size()) fail(DEM_EINVAL, std::string(who) + ": unknown material");
        if (scenes[s].p.periodic) fail(DEM_EINVAL, std::string(who) + ": boundaries are not supported in a periodic cell");
        if (scenes[s].n_walls >= kMaxWallsPerScene) fail(DEM_EINVAL, std::string(who) + ": too many boundaries in one scene");
        pull_bodies();
        HostScene& S = scenes[s];
        HostBody b;
        std::memset(&b, 0, sizeof b);
        b.kind = 1;
        b.scene = s;
        b.mat = mat;
        b.q[0] = 1.0;
        const int32_t gid = (int32_t)bodies.size();
        w.mat = mat;
        w.id = gid;
        // keep the wall table grouped by scene
        int at = 0;
        while (at < (int)walls.size() && wall_scene[at] <= s) ++at;
        walls.insert(walls.begin() + at, w);
        wall_scene.insert(wall_scene.begin() + at, s);
        b.wall = -1;
        const int64_t local = (int64_t)S.gids.size();
        S.gids.push_back(gid);
        bodies.push_back(b);
        for (int i = 0; i < (int)walls.size(); ++i) bodies[walls[i].id].wall = i;
        S.n_walls += 1;
        kinds_checked = false;
        host_dirty = true;
        need_rebuild = true;
        return local;
    }

    double pwave_dt(int s) const
    {
        // radii and materials never change after insertion: the host copy is current for them
        double best = INFINITY;
        for (int32_t g : scenes[s].gids) {
            const HostBody& b = bodies[g];
            if (b.kind != 0) continue;
            const HostMaterial& m = mats[b.mat];
            const double dt = b.r / std::sqrt(m.young / m.density);
            if (dt < best) best = dt;
        }
        return best;
    }

    // ------------------------------------------------------- uploading
    void upload_bodies()
    {
        // sphere slots in gid order; the first broad-phase run sorts them
        std::vector<int32_t> sph;
        for (int32_t g = 0; g < (int32_t)bodies.size(); ++g)
            if (bodies[g].kind == 0) sph.push_back(g);
        nslots = (int)sph.size();
        const size_t n = std::max<size_t>(nslots, 1);
        for (auto& b : bs) b.ensure(n);
        BodySet& B = bs[active];
        std::vector<double> col(4 * n);
        // packed 4-vectors: component c of slot i goes to col[4 i + c]
        auto push = [&](DBuf& d, auto get) {
            for (int i = 0; i < nslots; ++i) {
                const HostBody& b = bodies[sph[i]];
                for (int c = 0; c < 4; ++c) col[4 * (size_t)i + c] = get(b, c);
            }
            HIPC(hipMemcpyAsync(d.p, col.data(), 32 * (size_t)nslots, hipMemcpyHostToDevice, stream));
            HIPC(hipStreamSynchronize(stream));
        };
        push(B.xr, [](const HostBody& b, int c) { return c < 3 ? b.x[c] : b.r; });
        push(B.vm, [](const HostBody& b, int c) { return c < 3 ? b.v[c] : 0.0; });  // fresh Verlet account
        push(B.w, [](const HostBody& b, int c) { return c < 3 ? b.w[c] : 0.0; });
        push(B.q, [](const HostBody& b, int c) { return b.q[c]; });
        std::vector<uint8_t> u8(n);
        std::vector<int32_t> i32(n);
        std::vector<uint16_t> u16(n);
        std::vector<uint16_t> m16(n);
        for (int i = 0; i < nslots; ++i) m16[i] = (uint16_t)bodies[sph[i]].mat;
        HIPC(hipMemcpyAsync(B.mat.p, m16.data(), 2 * (size_t)nslots, hipMemcpyHostToDevice, stream));
        HIPC(hipStreamSynchronize(stream));
        for (int i = 0; i < nslots; ++i) u8[i] = bodies[sph[i]].blocked;
        HIPC(hipMemcpyAsync(B.blocked.p, u8.data(), (size_t)nslots, hipMemcpyHostToDevice, stream));
        HIPC(hipStreamSynchronize(stream));
        for (int i = 0; i < nslots; ++i) i32[i] = sph[i];
        HIPC(hipMemcpyAsync(B.id.p, i32.data(), 4 * (size_t)nslots, hipMemcpyHostToDevice, stream));
        for (int i = 0; i < nslots; ++i) u16[i] = (uint16_t)bodies[sph[i]].scene;
        HIPC(hipMemcpyAsync(B.scene.p, u16.data(), 2 * (size_t)nslots, hipMemcpyHostToDevice, stream));
        HIPC(hipStreamSynchronize(stream));
        // gid -> slot
        const int ng = (int)bodies.size();
        slot_of_id.ensure(4 * (size_t)std::max(ng, 1));
        std::vector<int32_t> sl((size_t)std::max(ng, 1), -1);
        for (int i = 0; i < nslots; ++i) sl[sph[i]] = i;
        HIPC(hipMemcpyAsync(slot_of_id.p, sl.data(), 4 * (size_t)ng, hipMemcpyHostToDevice, stream));
        // walls, scene table wall ranges
        d_walls.ensure(sizeof(Wall) * std::max<size_t>(walls.size(), 1));
        if (!walls.empty())
            HIPC(hipMemcpyAsync(d_walls.p, walls.data(), sizeof(Wall) * walls.size(), hipMemcpyHostToDevice, stream));
        HIPC(hipStreamSynchronize(stream));
        // wall ranges live in the device scene table (which the device also
        // updates for a periodic cell): read, modify, write back
        pull_scene_table();
        for (size_t s = 0; s < scenes.size(); ++s) {
            int b = 0, c = 0;
            for (int i = 0; i < (int)walls.size(); ++i)
                if (wall_scene[i] == (int)s) {
                    if (!c) b = i;
                    ++c;
                }
            sp[s].wall_begin = b;
            sp[s].wall_count = c;
        }
        push_scene_table();
        // the own arrays of the active pair set must cover every gid
        for (auto& P : ps) {
            P.own_begin.ensure_keep(4 * (size_t)std::max(ng, 1), 4 * (size_t)ngids_dev, stream);
            P.own_count.ensure_keep(4 * (size_t)std::max(ng, 1), 4 * (size_t)ngids_dev, stream);
        }
        ngids_dev = ng;
        host_dirty = false;
        on_device = true;
        need_rebuild = true;
        invalidate_graphs();
    }

    void pull_scene_table()
    {
        HIPC(hipMemcpyAsync(sp.data(), d_scenes.p, sizeof(SceneParams) * sp.size(), hipMemcpyDeviceToHost, stream));
        HIPC(hipStreamSynchronize(stream));
    }
    void push_scene_table()
    {
        HIPC(hipMemcpyAsync(d_scenes.p, sp.data(), sizeof(SceneParams) * sp.size(), hipMemcpyHostToDevice, stream));
        HIPC(hipStreamSynchronize(stream));
    }

    // The step kernels read their arguments from device memory.
    void upload_args()
    {
        // the descriptor carries a copy of scene 0's parameters, which the
        // device advances for a periodic cell: start from the current ones
        if (periodic && d_scenes.p) pull_scene_table();
        d_acc_ctrl.ensure(sizeof(double) * (size_t)kNetworkWords * std::max(grid_c, 1));
        d_acc_ctrl2.ensure(sizeof(double) * (size_t)(kNetworkWords + 2) * kCtrlReduceGrid);
        const StepArgs a = step_args();
        d_args.ensure(sizeof(StepArgs));
        HIPC(hipMemcpyAsync(d_args.p, &a, sizeof(StepArgs), hipMemcpyHostToDevice, stream));
        HIPC(hipStreamSynchronize(stream));
    }

    // ------------------------------------------------------- broad phase
    void rebuild()
    {
        const auto rb_t0 = std::chrono::steady_clock::now();
        if (host_dirty) upload_bodies();
        // only a periodic cell is advanced on the device; otherwise the host
        // table is the current one
        if (periodic) pull_scene_table();
        const int nsc = (int)scenes.size();
        // Delta L per scene (InsertionSortCollider.verletDist, negative = times the smallest radius)
        std::vector<double> rmin(nsc, INFINITY), rmax(nsc, 0.0);
        for (int s = 0; s < nsc; ++s) {
            rmin[s] = scenes[s].r_lo;
            rmax[s] = scenes[s].r_hi;
        }
        double limit = INFINITY;
        for (int s = 0; s < nsc; ++s) {
            const double vd = scenes[s].p.verlet_dist;
            const double dl = vd < 0.0 ? (std::isfinite(rmin[s]) ? -vd * rmin[s] : 0.0) : vd;
            scenes[s].verlet = dl;
            sp[s].verlet = dl;
            if (std::isfinite(rmin[s])) limit = std::min(limit, dl);
        }
        // grid per scene
        std::vector<double> bnd(6 * (size_t)nsc, 0.0);
        // bounds: the grid of an aperiodic scene; in both cases the check
        // that no position went non-finite before it is binned
        if (nslots > 0) {
            d_bounds.ensure(sizeof(double) * 6 * nsc);
            radix_tmp.ensure(std::max(radix_temp_bytes(nslots), bounds_temp_bytes(nslots)));
            launch_bounds(bs[active].view(), nslots, nsc, d_bounds.as<double>(), radix_tmp.p, stream);
            HIPC(hipGetLastError());
            HIPC(hipMemcpyAsync(bnd.data(), d_bounds.p, sizeof(double) * 6 * nsc, hipMemcpyDeviceToHost, stream));
            HIPC(hipStreamSynchronize(stream));
            for (int s = 0; s < nsc; ++s)
                if (scenes[s].n_spheres > 0)
                    for (int k = 0; k < 6; ++k)
                        if (!std::isfinite(bnd[6 * s + k])) fail(DEM_ENONFINITE, "non-finite sphere position");
        }
        int cells = 0, maxdim = 1;
        for (int s = 0; s < nsc; ++s) {
            SceneParams& P = sp[s];
            const double dl2 = 2.0 * P.verlet;
            // the plain cell: 2 r_max + 2 Delta L; every body searches +-1 cell
            const double hmax = std::max(2.0 * rmax[s] + dl2, 1e-300) * (1.0 + 1e-9);
            double rs = scenes[s].r_split;
            double Hinv[9];
            if (periodic) {
                if (!invert(P.H, Hinv)) fail(DEM_EPERIODIC, "singular periodic cell");
                std::memcpy(P.Hinv, Hinv, sizeof Hinv);
            }
            // Periodic level: cells of at least h across each period; the
            // largest body of the scene reaches `far` (its largest candidate
            // distance on this level), which must stay within 2 k + 1 distinct
            // cells so that no image is visited twice.
            auto periodic_level = [&](double h, double far, int32_t* dims, double* inv_h, double* origin,
                                      double* cellw) -> bool {
                for (int k = 0; k < 3; ++k) {
                    const double rn = std::sqrt(Hinv[3 * k] * Hinv[3 * k] + Hinv[3 * k + 1] * Hinv[3 * k + 1] +
                                                Hinv[3 * k + 2] * Hinv[3 * k + 2]);
                    const double width = 1.0 / rn;  // distance between opposite faces
                    int n = (int)std::min(std::floor(width / h), (double)(1 << 20));
                    if (n < 3) return false;
                    const int kk = std::max(1, (int)std::ceil(far / (width / (double)n)));
                    if (n < 2 * kk + 1) return false;
                    dims[k] = n;
                    inv_h[k] = (double)n;
                    origin[k] = 0.0;
                    cellw[k] = width / (double)n;
                }
                return true;
            };
            // Aperiodic level: the bounding box in cells of at least h, the
            // cell grown until the level's table holds at most 4 cells per body
            auto box_level = [&](double h, int64_t nbodies, int32_t* dims, double* inv_h, double* origin,
                                 double* cellw) {
                const double lo[3] = {bnd[6 * s + 0], bnd[6 * s + 1], bnd[6 * s + 2]};
                const double hi[3] = {bnd[6 * s + 3], bnd[6 * s + 4], bnd[6 * s + 5]};
                for (;;) {
                    int64_t tot = 1;
                    for (int k = 0; k < 3; ++k) {
                        const double ext = hi[k] > lo[k] ? hi[k] - lo[k] : 0.0;
                        int64_t n = (int64_t)std::floor(ext / h) + 1;
                        dims[k] = (int)std::min<int64_t>(n, 1 << 20);
                        tot *= dims[k];
                    }
                    const int64_t nb = std::max<int64_t>(nbodies, 1);
                    if (tot <= 4 * nb + 4096 && dims[0] < (1 << 20) && dims[1] < (1 << 20) && dims[2] < (1 << 20)) break;
                    h *= 1.25;
                }
                for (int k = 0; k < 3; ++k) {
                    origin[k] = lo[k] - 1e-12 * std::fabs(lo[k]) - 1e-300;
                    inv_h[k] = 1.0 / h;
                    cellw[k] = h;
                }
            };
            for (int k = 0; k < 3; ++k) {
                P.dims2[k] = 1;
                P.inv_h2[k] = 1.0;
                P.origin2[k] = 0.0;
                P.cellw2[k] = hmax;
            }
            if (rs > 0.0) {
                // level 0 (radii <= r_split) and level 1 (the others)
                const double h0 = (2.0 * rs + dl2) * (1.0 + 1e-9);
                bool ok;
                if (periodic) {
                    ok = periodic_level(h0, (rmax[s] + rs) + dl2, P.dims, P.inv_h, P.origin, P.cellw) &&
                         periodic_level(hmax, 2.0 * rmax[s] + dl2, P.dims2, P.inv_h2, P.origin2, P.cellw2);
                } else {
                    box_level(h0, scenes[s].n_spheres - scenes[s].n_large, P.dims, P.inv_h, P.origin, P.cellw);
                    box_level(hmax, scenes[s].n_large, P.dims2, P.inv_h2, P.origin2, P.cellw2);
                    ok = true;
                }
                if (!ok) rs = 0.0;  // the cell is too small for the fine level: one level
            }
            if (rs == 0.0) {
                if (periodic) {
                    if (!periodic_level(hmax, 2.0 * rmax[s] + dl2, P.dims, P.inv_h, P.origin, P.cellw))
                        fail(DEM_EPERIODIC, "periodic cell narrower than 3 x (2 r_max + 2 Delta L) along an axis");
                } else {
                    box_level(hmax, scenes[s].n_spheres, P.dims, P.inv_h, P.origin, P.cellw);
                }
            }
            P.r_split = rs;
            P.cell_offset = cells;
            cells += P.dims[0] * P.dims[1] * P.dims[2];
            P.cell_offset2 = cells;
            if (rs > 0.0) cells += P.dims2[0] * P.dims2[1] * P.dims2[2];
            for (int k = 0; k < 3; ++k) maxdim = std::max({maxdim, P.dims[k], rs > 0.0 ? P.dims2[k] : 1});
            // mean-field share of the Verlet budget (periodic)
            double lf = 0.0;
            for (int k = 0; k < 9; ++k) lf += P.L[k] * P.L[k];
            P.verlet_cell_rate = 0.5 * std::sqrt(lf) * (2.0 * rmax[s] + 4.0 * P.verlet);
            scenes[s].rmax = rmax[s];
            P.rmax = rmax[s];
        }
        ncells = std::max(cells, 1);
        morton_bits = 1;
        while ((1 << morton_bits) < maxdim) ++morton_bits;
        scene_bits = 0;
        if (nsc > 1)
            while ((1 << scene_bits) < nsc) ++scene_bits;
        // key: scene bits | 3 x morton_bits (either level's cell)
        if (3 * morton_bits + scene_bits > 64) fail(DEM_EINVAL, "grid too large for 64-bit cell keys");
        int64_t nlarge = 0;
        for (int s = 0; s < nsc; ++s)
            if (sp[s].r_split > 0.0) nlarge += scenes[s].n_large;
        push_scene_table();

        Counters& C = *h_ctr;
        int npairs_new = 0;
        if (nslots > 0) {
            GridArgs g;
            g.bod = bs[active].view();
            g.scenes = d_scenes.as<SceneParams>();
            g.scene0 = sp[0];
            g.nscenes = nsc;
            g.nslots = nslots;
            g.scene_bits = scene_bits;
            g.morton_bits = morton_bits;
            // keys, sort, permute into the other body set
            keys.ensure(8 * (size_t)nslots);
            vals.ensure(4 * (size_t)nslots);
            keys_alt.ensure(8 * (size_t)nslots);
            vals_alt.ensure(4 * (size_t)nslots);
            radix_tmp.ensure(std::max(radix_temp_bytes(nslots), bounds_temp_bytes(nslots)));
            d_flag.ensure(4);
            g.period_range = d_flag.as<int32_t>();
            HIPC(hipMemsetAsync(d_flag.p, 0, 4, stream));
            launch_keys(g, keys.as<uint64_t>(), vals.as<uint32_t>(), stream);
            if (periodic) {
                int32_t far = 0;
                HIPC(hipMemcpyAsync(&far, d_flag.p, 4, hipMemcpyDeviceToHost, stream));
                HIPC(hipStreamSynchronize(stream));
                if (far)
                    fail(DEM_EPERIODIC, "a sphere is more than 511 periods from the periodic cell's origin; "
                                        "bring the positions back into the cell (dem_set_state)");
            }
            bool in_alt = false;
            radix_sort_pairs(keys.as<uint64_t>(), vals.as<uint32_t>(), keys_alt.as<uint64_t>(), vals_alt.as<uint32_t>(),
                             nslots, 3 * morton_bits + scene_bits, radix_tmp.p, stream, &in_alt);
            const uint64_t* skeys = in_alt ? keys_alt.as<uint64_t>() : keys.as<uint64_t>();
            const uint32_t* order = in_alt ? vals_alt.as<uint32_t>() : vals.as<uint32_t>();
            launch_permute(bs[active].view(), bs[1 - active].view(), order, nslots, batched(), periodic,
                           slot_of_id.as<int32_t>(), stream);
            active = 1 - active;
            g.bod = bs[active].view();
            // cells
            cell_start.ensure(4 * (size_t)ncells);
            cell_end.ensure(4 * (size_t)ncells);
            launch_cells(g, skeys, cell_start.as<uint32_t>(), cell_end.as<uint32_t>(), ncells, stream);
            g.large_slot = nullptr;
            if (nlarge > 0) {
                // level 1: the spheres above r_split, their slots sorted by
                // coarse cell (the bodies stay in level-0 order)
                lflag.ensure(4 * ((size_t)nslots + 1));
                lscan.ensure(4 * ((size_t)nslots + 1));
                keys2.ensure(8 * (size_t)nlarge);
                vals2.ensure(4 * (size_t)nlarge);
                keys2_alt.ensure(8 * (size_t)nlarge);
                vals2_alt.ensure(4 * (size_t)nlarge);
                scan_tmp.ensure(scan_temp_bytes(nslots + 1));
                d_total.ensure(16);
                launch_large_flags(g, lflag.as<uint32_t>(), stream);
                HIPC(hipMemsetAsync(lflag.as<uint32_t>() + nslots, 0, 4, stream));
                exclusive_scan_u32(lflag.as<uint32_t>(), lscan.as<uint32_t>(), nslots + 1, scan_tmp.p,
                                   d_total.as<uint32_t>(), stream);
                launch_large_keys(g, lscan.as<uint32_t>(), keys2.as<uint64_t>(), vals2.as<uint32_t>(), stream);
                bool alt2 = false;
                radix_sort_pairs(keys2.as<uint64_t>(), vals2.as<uint32_t>(), keys2_alt.as<uint64_t>(),
                                 vals2_alt.as<uint32_t>(), (int)nlarge, 3 * morton_bits + scene_bits, radix_tmp.p,
                                 stream, &alt2);
                const uint64_t* sk2 = alt2 ? keys2_alt.as<uint64_t>() : keys2.as<uint64_t>();
                launch_cells_large(g, sk2, (int)nlarge, cell_start.as<uint32_t>(), cell_end.as<uint32_t>(), ncells,
                                   stream);
                g.large_slot = alt2 ? vals2_alt.as<uint32_t>() : vals2.as<uint32_t>();
            }
            // sweep: count, scan, fill
            SweepArgs sw{};
            sw.g = g;
            sw.nlarge = (int)nlarge;
            sw.cell_start = cell_start.as<uint32_t>();
            sw.cell_end = cell_end.as<uint32_t>();
            sw.walls = d_walls.as<Wall>();
            counts.ensure(4 * ((size_t)nslots + 1));
            row_start.ensure(4 * ((size_t)nslots + 1));
            HIPC(hipMemsetAsync(counts.as<uint32_t>() + nslots, 0, 4, stream));
            sw.count = counts.as<uint32_t>();
            launch_sweep_count(sw, stream);
            d_total.ensure(16);
            scan_tmp.ensure(scan_temp_bytes(nslots + 1));
            exclusive_scan_u32(counts.as<uint32_t>(), row_start.as<uint32_t>(), nslots + 1, scan_tmp.p,
                               d_total.as<uint32_t>(), stream);
            uint32_t nent = 0;
            HIPC(hipMemcpyAsync(&nent, d_total.p, 4, hipMemcpyDeviceToHost, stream));
            HIPC(hipStreamSynchronize(stream));
            HIPC(hipGetLastError());
            if (nent > 0x7ffffff0u) fail(DEM_ENOMEM, "too many candidate entries");
            ent_slot.ensure(4 * ((size_t)nent + 1));
            ent_pid.ensure(4 * ((size_t)nent + 1));
            ent_cell.ensure(4 * ((size_t)nent + 1));
            ent_own.ensure(4 * ((size_t)nent + 1));
            own_scan.ensure(4 * ((size_t)nent + 1));
            rows_ent.ensure(4 * ((size_t)nent + 1));
            raw_slot.ensure(4 * ((size_t)nent + 1));
            raw_pid.ensure(4 * ((size_t)nent + 1));
            raw_cell.ensure(4 * ((size_t)nent + 1));
            ent_body.ensure(4 * ((size_t)nent + 1));
            sw.row_start = row_start.as<int32_t>();
            sw.raw_slot = raw_slot.as<int32_t>();
            sw.raw_pid = raw_pid.as<int32_t>();
            sw.raw_cell = raw_cell.as<int32_t>();
            sw.ent_body = ent_body.as<int32_t>();
            sw.nent = (int)nent;
            sw.ent_slot = ent_slot.as<int32_t>();
            sw.ent_pid = ent_pid.as<int32_t>();
            sw.ent_cell = ent_cell.as<int32_t>();
            sw.ent_own = ent_own.as<uint32_t>();
            sw.max_row = 0;
            launch_sweep_fill(sw, stream);
            HIPC(hipMemsetAsync(ent_own.as<uint32_t>() + nent, 0, 4, stream));
            scan_tmp.ensure(scan_temp_bytes((int)nent + 1));
            exclusive_scan_u32(ent_own.as<uint32_t>(), own_scan.as<uint32_t>(), (int)nent + 1, scan_tmp.p,
                               d_total.as<uint32_t>(), stream);
            uint32_t np = 0;
            HIPC(hipMemcpyAsync(&np, d_total.p, 4, hipMemcpyDeviceToHost, stream));
            HIPC(hipStreamSynchronize(stream));
            HIPC(hipGetLastError());
            if (np >= kPairMask) fail(DEM_ENOMEM, "too many candidate pairs");
            npairs_new = (int)np;
            n_candidates = np;
            // new pair set
            PairSet& NP = ps[1 - pactive];
            PairSet& OP = ps[pactive];
            NP.ensure(np, precision == DEM_FP32_MIXED);
            const int ng = (int)bodies.size();
            NP.own_begin.ensure(4 * (size_t)std::max(ng, 1));
            NP.own_count.ensure(4 * (size_t)std::max(ng, 1));
            HIPC(hipMemsetAsync(NP.own_begin.p, 0, 4 * (size_t)std::max(ng, 1), stream));
            HIPC(hipMemsetAsync(NP.own_count.p, 0, 4 * (size_t)std::max(ng, 1), stream));
            PairBuildArgs pb;
            pb.bod = g.bod;
            pb.row_start = row_start.as<int32_t>();
            pb.ent_slot = ent_slot.as<int32_t>();
            pb.ent_pid = ent_pid.as<int32_t>();
            pb.ent_cell = ent_cell.as<int32_t>();
            pb.own_scan = own_scan.as<uint32_t>();
            pb.ent_own = ent_own.as<uint32_t>();
            pb.ent_body = ent_body.as<int32_t>();
            pb.rows.start = row_start.as<int32_t>();
            pb.rows.ent = rows_ent.as<uint32_t>();
            pb.pr = NP.view();
            pb.hist_new = NP.history();
            pb.hist_old = OP.history();
            pb_ca.ensure(4 * ((size_t)np + 1));
            pb_cb.ensure(4 * ((size_t)np + 1));
            pb_found.ensure(4 * ((size_t)np + 1));
            pb_flag.ensure(4 * ((size_t)np + 1));
            pb_scan.ensure(4 * ((size_t)np + 1));
            pb.ca = pb_ca.as<int32_t>();
            pb.cb = pb_cb.as<int32_t>();
            pb.found = pb_found.as<int32_t>();
            pb.flag = pb_flag.as<uint32_t>();
            pb.flag_scan = pb_scan.as<uint32_t>();
            pb.nslots = nslots;
            pb.nent = (int)nent;
            pb.npairs = (int)np;
            pb.has_old = (OP.cap > 0 && OP.own_begin.p && old_ngids > 0) ? 1 : 0;
            pb.hist_f32 = precision == DEM_FP32_MIXED ? 1 : 0;
            launch_pair_build(pb, stream);
            launch_carry_find(pb, stream, std::min(old_ngids, ng));
            // touching pairs first: ranks from a scan of the carried flags
            scan_tmp.ensure(scan_temp_bytes((int)np + 1));
            exclusive_scan_u32(pb.flag, pb.flag_scan, (int)np + 1, scan_tmp.p, d_total.as<uint32_t>(), stream);
            launch_partition(pb, stream);
            HIPC(hipGetLastError());
            pactive = 1 - pactive;
            old_ngids = ng;
            // The previous list is not read again once this run's kernels
            // are done: size it for the new list's pairs now, so that the next
            // run (which fills it) allocates nothing.  A buffer it outgrows
            // is freed by hipFree, which waits for the device first.
            PairSet& spare = ps[1 - pactive];
            spare.ensure(np, precision == DEM_FP32_MIXED);
            spare.own_begin.ensure(4 * (size_t)std::max(ng, 1));
            spare.own_count.ensure(4 * (size_t)std::max(ng, 1));
        } else {
            npairs_new = 0;
            n_candidates = 0;
            row_start.ensure(8);
            HIPC(hipMemsetAsync(row_start.p, 0, 8, stream));
            old_ngids = (int)bodies.size();
        }
        npairs = npairs_new;
        // fold the per-block slots before the grids change, then size them
        fold_slots();
        // the contact kernel gives each of the 8 XCDs one eighth of the
        // pairs: at least ceil(ceil(npairs / 8) / block) blocks per XCD
        const int per_xcd = (int)((((int64_t)npairs + 7) / 8 + block_contact - 1) / block_contact);
        if ((int64_t)grid_c * block_contact < npairs || grid_c < 8 * per_xcd || grid_c < 1)
            grid_c = std::max({(int)(((int64_t)npairs * 5 / 4 + block_contact - 1) / block_contact), 8 * per_xcd, 1});
        grid_i = std::max((nslots + block_integrate - 1) / block_integrate, 1);
        d_part_c.ensure(sizeof(ContactAcc) * (size_t)grid_c);
        d_part_i.ensure(sizeof(IntAcc) * (size_t)grid_i);
        HIPC(hipMemsetAsync(d_part_c.p, 0, sizeof(ContactAcc) * (size_t)grid_c, stream));
        HIPC(hipMemsetAsync(d_part_i.p, 0, sizeof(IntAcc) * (size_t)grid_i, stream));
        acc_c_n = grid_c;
        acc_i_n = grid_i;
        // counters: fresh Verlet budget, flags clear, parity 0 (every field
        // is rewritten, so the device copy is not read back first)
        C.verlet_limit = 0.98 * (std::isfinite(limit) ? limit : 0.0);
        double cell_step = 0.0;
        for (int s = 0; s < nsc; ++s) cell_step = std::max(cell_step, sp[s].verlet_cell_rate * sp[s].dt);
        C.verlet_cell_step = cell_step;
        C.stall[0] = C.stall[1] = 0;
        C.steps_done = 0;
        C.halt = 0;
        C.iter0 = scenes[0].iter;
        C.nonfinite = 0;  // positions are finite (checked above); an earlier
        C.unstable = 0;   // failure was repaired with dem_set_state
        next_parity = 0;
        HIPC(hipMemcpyAsync(d_ctr.p, h_ctr, sizeof(Counters), hipMemcpyHostToDevice, stream));
        HIPC(hipStreamSynchronize(stream));
        upload_args();
        need_rebuild = false;
        ++rebuilds;
        iter_at_rebuild = scenes[0].iter;
        // the run ends with a synchronisation: its wall time is its cost
        last_rebuild_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - rb_t0).count();
        rebuild_ms_total += last_rebuild_ms;
    }

    // Largest Verlet account over the bodies (device reduction).
    double max_account()
    {
        if (nslots <= 0) return 0.0;
        d_acct.ensure(8);
        HIPC(hipMemsetAsync(d_acct.p, 0, 8, stream));
        launch_max_account(bs[active].view(), nslots, d_acct.as<unsigned long long>(), stream);
        unsigned long long bits = 0;
        HIPC(hipMemcpyAsync(&bits, d_acct.p, 8, hipMemcpyDeviceToHost, stream));
        HIPC(hipStreamSynchronize(stream));
        double v;
        std::memcpy(&v, &bits, 8);
        return v;
    }

    // Per-step mean-field share of the Verlet budget (periodic), written
    // into the device counters between steps.
    void update_cell_step()
    {
        if (need_rebuild || !d_ctr.p) return;  // the next run sets it
        double cell_step = 0.0;
        for (size_t s = 0; s < sp.size(); ++s) cell_step = std::max(cell_step, sp[s].verlet_cell_rate * sp[s].dt);
        h_ctr->verlet_cell_step = cell_step;
        HIPC(hipMemcpyAsync(reinterpret_cast<char*>(d_ctr.p) + offsetof(Counters, verlet_cell_step),
                            &h_ctr->verlet_cell_step, sizeof(double), hipMemcpyHostToDevice, stream));
        HIPC(hipStreamSynchronize(stream));
    }

    // Sum the per-block slots in block order.  cum = true: add the running
    // sums to the bases and clear the slots (before the grids change).
    struct SlotSums {
        double el = 0, plast = 0, kin = 0, rot = 0, grav = 0, damp = 0, visc = 0;
        unsigned long long ss = 0, sw = 0, cum = 0;
    };
    SlotSums read_slots()
    {
        SlotSums t;
        h_slots_c.ensure(sizeof(ContactAcc) * (size_t)std::max(acc_c_n, 1));
        h_slots_i.ensure(sizeof(IntAcc) * (size_t)std::max(acc_i_n, 1));
        const ContactAcc* c = h_slots_c.as<ContactAcc>();
        const IntAcc* i = h_slots_i.as<IntAcc>();
        if (acc_c_n)
            HIPC(hipMemcpyAsync(h_slots_c.p, d_part_c.p, sizeof(ContactAcc) * (size_t)acc_c_n, hipMemcpyDeviceToHost,
                                stream));
        if (acc_i_n)
            HIPC(hipMemcpyAsync(h_slots_i.p, d_part_i.p, sizeof(IntAcc) * (size_t)acc_i_n, hipMemcpyDeviceToHost,
                                stream));
        HIPC(hipStreamSynchronize(stream));
        for (int k = 0; k < acc_c_n; ++k) {
            const ContactAcc& a = c[k];
            t.el += a.el;
            t.plast += a.plast;
            t.visc += a.visc;
            t.ss += a.ss;
            t.sw += a.sw;
            t.cum += a.ss_cum + a.sw_cum;
        }
        for (int k = 0; k < acc_i_n; ++k) {
            const IntAcc& a = i[k];
            t.kin += a.kin;
            t.rot += a.rot;
            t.grav += a.grav;
            t.damp += a.damp;
        }
        return t;
    }
    void fold_slots()
    {
        if (!acc_c_n && !acc_i_n) return;
        const SlotSums t = read_slots();
        base_plast += t.plast;
        base_visc += t.visc;
        base_grav += t.grav;
        base_damp += t.damp;
        base_contact_steps += t.cum;
        if (!slots_fresh) {
            last_el = t.el;
            last_kin = t.kin;
            last_rot = t.rot;
            last_ss = t.ss;
            last_sw = t.sw;
        }
        slots_fresh = true;
    }
    // Largest overlap / smaller radius over the pairs that touched at the
    // last step (0 before the first step), from their history records.
    double max_overlap()
    {
        if (npairs <= 0 || !contacts_valid) return 0.0;
        d_acct.ensure(8);
        HIPC(hipMemsetAsync(d_acct.p, 0, 8, stream));
        StepArgs a = step_args();
        launch_max_overlap(a, precision, d_acct.as<unsigned long long>(), stream);
        HIPC(hipGetLastError());
        unsigned long long bits = 0;
        HIPC(hipMemcpyAsync(&bits, d_acct.p, 8, hipMemcpyDeviceToHost, stream));
        HIPC(hipStreamSynchronize(stream));
        double v;
        std::memcpy(&v, &bits, sizeof v);
        return v;
    }
    // Energies and contact counts as reported: bases + current slots.
    void totals(dem_energy* e, unsigned long long* ss, unsigned long long* sw, unsigned long long* csteps)
    {
        const SlotSums t = read_slots();
        const bool fresh = slots_fresh;
        const double el = fresh ? last_el : t.el, kin = fresh ? last_kin : t.kin, rot = fresh ? last_rot : t.rot;
        if (e) {
            e->kinetic = kin;
            e->kin_rot = rot;
            e->elastic = el;
            e->grav_work = base_grav + t.grav;
            e->damp_dissip = base_damp + t.damp;
            e->plastic_dissip = base_plast + t.plast;
            e->visc_dissip = base_visc + t.visc;
            e->total = (((((e->kinetic + e->kin_rot) + e->elastic) + e->grav_work) + e->damp_dissip) + e->plastic_dissip) +
                       e->visc_dissip;
        }
        if (ss) *ss = fresh ? last_ss : t.ss;
        if (sw) *sw = fresh ? last_sw : t.sw;
        if (csteps) *csteps = base_contact_steps + t.cum;
    }

    // ------------------------------------------------------------ tuning
    // Performance knobs that leave every result unchanged: the launch shape
    // of the two step kernels, the number of steps per captured graph, and
    // the Verlet distance (it changes which non-touching pairs are carried
    // as candidates and how often the broad phase runs, never the real
    // contacts or the order of a body's force sum).
    dem_tuning tuning() const
    {
        dem_tuning t;
        std::memset(&t, 0, sizeof t);
        t.block_contact = block_contact;
        t.block_integrate = block_integrate;
        t.chunk = chunk;
        const double vd = scenes.empty() ? -0.5 : scenes[0].p.verlet_dist;
        t.verlet_factor = vd < 0.0 ? -vd : 0.0;
        t.ms_per_step = tuned_ms;
        return t;
    }
    void set_tuning(const dem_tuning& t)
    {
        auto ok_block = [](int b) { return b >= 64 && b <= 1024 && b % 64 == 0; };
        if (!ok_block(t.block_contact) || !ok_block(t.block_integrate))
            fail(DEM_EINVAL, "tuning: block sizes must be multiples of 64 in [64, 1024]");
        if (t.chunk < 2 || t.chunk > 4096 || t.chunk % 2) fail(DEM_EINVAL, "tuning: chunk must be even, 2..4096");
        if (!(t.verlet_factor >= 0.0) || !(t.verlet_factor <= 4.0))
            fail(DEM_EINVAL, "tuning: verlet_factor must be in [0, 4] (0 keeps each scene's own verlet_dist)");
        block_contact = t.block_contact;
        block_integrate = t.block_integrate;
        chunk = t.chunk;
        if (t.verlet_factor > 0.0) {
            for (auto& S : scenes) S.p.verlet_dist = -t.verlet_factor;
            need_rebuild = true;
        }
        // the contact grid follows the block size at the next run
        grid_c = 0;
        need_rebuild = true;
        invalidate_graphs();
    }
    // Milliseconds per step over `steps` ordinary steps, with the broad phase
    // charged at its rate rather than by the runs that happen to fall in the
    // window: the window's wall time less its broad-phase runs, plus the last
    // run's cost divided by the number of steps between runs, which is
    // estimated from how fast the largest Verlet account grew (the run comes
    // when it reaches the budget) and, when runs did fall in the window, no
    // longer than their observed spacing.
    double probe(int64_t steps)
    {
        HIPC(hipStreamSynchronize(stream));
        const int64_t rb0 = rebuilds;
        const double rbt0 = rebuild_ms_total;
        const auto t0 = std::chrono::steady_clock::now();
        step(steps);
        HIPC(hipStreamSynchronize(stream));
        const auto t1 = std::chrono::steady_clock::now();
        const double wall = std::chrono::duration<double, std::milli>(t1 - t0).count();
        const int64_t n = std::max<int64_t>(steps, 1);
        const double steady = std::max(wall - (rebuild_ms_total - rbt0), 0.0) / (double)n;
        double interval = INFINITY;
        const int64_t since = scenes[0].iter - iter_at_rebuild;
        const double acct = max_account();
        if (since > 0 && acct > 0.0) interval = (double)since * h_ctr->verlet_limit / acct;
        if (rebuilds > rb0) interval = std::min(interval, (double)n / (double)(rebuilds - rb0));
        return steady + (std::isfinite(interval) ? last_rebuild_ms / std::max(interval, 1.0) : 0.0);
    }
    std::string tuning_key()
    {
        hipDeviceProp_t prop;
        HIPC(hipGetDeviceProperties(&prop, device));
        auto lg = [](int64_t v) {
            int b = 0;
            while ((int64_t)1 << b < v + 1) ++b;
            return b;
        };
        std::ostringstream k;
        k << prop.gcnArchName << "|p" << precision << "|b" << (batched() ? 1 : 0) << "|c" << (periodic ? 1 : 0) << "|n"
          << lg(nslots) << "|k" << lg(n_candidates) << "|s" << scenes.size();
        std::string key = k.str();
        for (char& c : key)
            if (c == ' ' || c == ':') c = '_';
        return key;
    }
    // The autotuner: with a cache file that already holds this workload's
    // key, apply its entry; otherwise try each knob in turn (coordinate
    // descent from the current setting), each candidate timed over
    // `probe_steps` ordinary steps, keep the fastest, and append it to the
    // cache.  The probe steps advance the simulation like any others.
    dem_tuning autotune(int64_t probe_steps, const char* cache_path)
    {
        if (probe_steps < 2) fail(DEM_EINVAL, "dem_autotune: probe_steps must be >= 2");
        if (need_rebuild || host_dirty) step(1);  // build the candidate list the key refers to
        const std::string key = tuning_key();
        if (cache_path && *cache_path) {
            std::ifstream in(cache_path);
            std::string line;
            while (std::getline(in, line)) {
                std::istringstream ls(line);
                std::string k;
                dem_tuning t;
                std::memset(&t, 0, sizeof t);
                if (ls >> k >> t.block_contact >> t.block_integrate >> t.chunk >> t.verlet_factor >> t.ms_per_step &&
                    k == key) {
                    set_tuning(t);
                    tuned_ms = t.ms_per_step;
                    return tuning();
                }
            }
        }
        dem_tuning best = tuning();
        probe(probe_steps);  // warm the current setting (graph capture, first broad phase)
        best.ms_per_step = probe(probe_steps);
        const int blocks[] = {64, 128, 256, 512, 1024};
        const int chunks[] = {16, 32, 64};
        const double vfs[] = {0.05, 0.1, 0.25, 0.5, 1.0};
        auto trial = [&](dem_tuning t) {
            set_tuning(t);
            probe(2);  // first run of the new setting: capture and broad phase
            t.ms_per_step = probe(probe_steps);
            if (t.ms_per_step < best.ms_per_step) best = t;
        };
        for (double v : vfs)
            if (v != best.verlet_factor) {
                dem_tuning t = best;
                t.verlet_factor = v;
                trial(t);
            }
        for (int b : blocks)
            if (b != best.block_contact) {
                dem_tuning t = best;
                t.block_contact = b;
                trial(t);
            }
        for (int b : blocks)
            if (b != best.block_integrate) {
                dem_tuning t = best;
                t.block_integrate = b;
                trial(t);
            }
        for (int c : chunks)
            if (c != best.chunk) {
                dem_tuning t = best;
                t.chunk = c;
                trial(t);
            }
        set_tuning(best);
        tuned_ms = best.ms_per_step;
        if (cache_path && *cache_path) {
            std::ofstream out(cache_path, std::ios::app);
            if (!out) fail(DEM_EINVAL, std::string("dem_autotune: cannot write ") + cache_path);
            out.precision(9);
            out << key << ' ' << best.block_contact << ' ' << best.block_integrate << ' ' << best.chunk << ' '
                << best.verlet_factor << ' ' << best.ms_per_step << '\n';
        }
        return tuning();
    }

    // ------------------------------------------------------------ step
    StepArgs step_args() const
    {
        StepArgs a;
        a.bod = bs[active].view();
        a.pr = ps[pactive].view();
        a.rows.start = row_start.as<int32_t>();
        a.rows.ent = rows_ent.as<uint32_t>();
        a.walls = d_walls.as<Wall>();
        a.mats = d_mats.as<Material>();
        a.tanphi = d_tanphi.as<double>();
        a.ve = d_ve.as<ViscElPair>();
        a.nmat = (int)mats.size();
        a.scenes = d_scenes.as<SceneParams>();
        a.scene0 = sp[0];
        a.nscenes = (int)scenes.size();
        a.nslots = nslots;
        a.npairs = npairs;
        a.ctr = d_ctr.as<Counters>();
        a.acc_contact = d_part_c.as<ContactAcc>();
        a.acc_integrate = d_part_i.as<IntAcc>();
        a.track_energy = track_energy ? 1 : 0;
        a.ctrl = d_ctrl_cfg.as<CtrlConfig>();
        a.ctrl_state = d_ctrl_state.as<CtrlState>();
        a.acc_ctrl = d_acc_ctrl.as<double>();
        a.acc_ctrl2 = d_acc_ctrl2.as<double>();
        a.nblocks_contact = grid_c;
        a.nblocks_integrate = grid_i;
        a.use_frec = uses_force_records(precision, has_viscel()) ? 1 : 0;
        a.pad_ = 0;
        return a;
    }

    // ev (timing mode): 4 events, stamped at the start and end of the
    // contact and the integrate kernels by the dispatch packets themselves
    // measure: the step ends an update period of the controlled cell (its
    // contact sums kernel runs after integrate)
    void launch_step(int parity, hipEvent_t* ev, bool measure)
    {
        const StepArgs* a = d_args.as<StepArgs>();
        launch_contact(a, parity, grid_c, precision, batched(), periodic, block_contact, stream, ev ? ev[0] : nullptr,
                       ev ? ev[1] : nullptr, periodic && pt_active && measure, has_prims(), has_viscel());
        launch_integrate(a, parity, grid_i, precision, batched(), periodic, uses_force_records(precision, has_viscel()),
                         block_integrate, stream, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
        if (periodic && pt_active && measure) launch_ctrl_reduce(a, parity, stream);
        if (periodic) launch_cell_update(a, parity, stream);
    }
    // phase of the controlled cell's update period at a launch chain's first
    // step; step i of the chain ends a period when (phase + i + 1) % period == 0
    int ctrl_period() const { return pt_active ? std::max(pt_glob_update, 1) : 1; }
    int ctrl_phase() const { return pt_active ? (int)(scenes[0].iter % ctrl_period()) : 0; }
    bool measure_step(int phase, int i) const { return pt_active && (phase + i + 1) % ctrl_period() == 0; }

    std::string graph_key(int n, int phase) const
    {
        char buf[256];
        std::snprintf(buf, sizeof buf, "%p/%d/%d/%d/%d/%d/%d/%d/%d/%d/%d/%d", d_args.p, grid_c, grid_i, n,
                      timing ? 1 : 0, block_contact, block_integrate, pt_active ? 1 : 0, ctrl_period(), phase,
                      has_prims() ? 1 : 0, has_viscel() ? 1 : 0);
        return buf;
    }

    GraphEntry& get_graph(int n, int phase)
    {
        const std::string key = graph_key(n, phase);
        auto it = graphs.find(key);
        if (it != graphs.end()) return it->second;
        if (graphs.size() > 16) invalidate_graphs();
        GraphEntry ge;
        hipGraph_t g;
        HIPC(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < n; ++i) launch_step(i & 1, nullptr, measure_step(phase, i));
        HIPC(hipStreamEndCapture(stream, &g));
        HIPC(hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0));
        HIPC(hipGraphDestroy(g));
        return graphs.emplace(key, std::move(ge)).first->second;
    }

    void read_counters()
    {
        HIPC(hipMemcpyAsync(h_ctr, d_ctr.p, sizeof(Counters), hipMemcpyDeviceToHost, stream));
        HIPC(hipStreamSynchronize(stream));
    }

    void add_time(const char* name, hipEvent_t a, hipEvent_t b)
    {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, a, b) == hipSuccess) {
            timers[name].total_ms += ms;
            timers[name].launches += 1;
        } else {
            (void)hipGetLastError();  // do not leave the failed query as a sticky error
        }
    }

    // O.step x nsteps.  With the stiffness timestepper active the steps run
    // in segments, and the timestepper sets dt before each step whose
    // iteration count is a multiple of its interval.  The controlled cell
    // runs on the device inside the steps; when it reaches its goal with
    // stop_when_done the call returns early.
    void step(int64_t nsteps)
    {
        if (nsteps < 0) fail(DEM_EINVAL, "dem_step: nsteps < 0");
        HIPC(hipSetDevice(device));
        check_material_kinds();
        if ((pt_active || ts_interval > 0) && has_viscel())
            fail(DEM_EINVAL, "dem_step: the stiffness timestepper and the controlled cell are not available with "
                             "visco-elastic materials");
        if (timing) timers.clear();
        if (ts_interval <= 0) {
            run_steps(nsteps);
            return;
        }
        HostScene& S = scenes[0];
        int64_t left = nsteps;
        while (left > 0) {
            if (S.iter % ts_interval == 0) set_dt(0, stiffness_dt(0, ts_safety));
            const int64_t seg = std::min(left, ts_interval - S.iter % ts_interval);
            const int64_t before = S.iter;
            const bool halted = run_steps(seg);
            left -= S.iter - before;
            if (halted) break;
        }
    }

    // Returns true when the controlled cell halted the steps.
    bool run_steps(int64_t nsteps)
    {
        if (host_dirty) upload_bodies();
        // no step: only bring the pair list up to date (a pending broad-phase run)
        if (nsteps == 0) {
            if ((nslots > 0 || !walls.empty()) && (need_rebuild || h_ctr->stall[next_parity ^ 1])) {
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (timing) {
                    HIPC(hipEventCreate(&e0));
                    HIPC(hipEventCreate(&e1));
                    HIPC(hipEventRecord(e0, stream));
                }
                try {
                    rebuild();
                    if (timing) {
                        HIPC(hipEventRecord(e1, stream));
                        HIPC(hipEventSynchronize(e1));
                        add_time("rebuild", e0, e1);
                    }
                } catch (...) {
                    if (e0) (void)hipEventDestroy(e0);
                    if (e1) (void)hipEventDestroy(e1);
                    throw;
                }
                if (e0) (void)hipEventDestroy(e0);
                if (e1) (void)hipEventDestroy(e1);
            }
            return false;
        }
        if (nslots == 0 && walls.empty()) {
            for (auto& S : scenes) {
                S.iter += nsteps;
                S.time += nsteps * S.p.dt;
            }
            return false;
        }
        bool halted = false;
        int64_t remaining = nsteps;
        std::vector<hipEvent_t> direct_ev;
        hipEvent_t rb0 = nullptr, rb1 = nullptr;
        if (timing) {
            HIPC(hipEventCreate(&rb0));
            HIPC(hipEventCreate(&rb1));
        }
        try {
            while (remaining > 0) {
                if (need_rebuild || h_ctr->stall[next_parity ^ 1]) {
                    if (timing) HIPC(hipEventRecord(rb0, stream));
                    rebuild();
                    if (timing) {
                        HIPC(hipEventRecord(rb1, stream));
                        HIPC(hipEventSynchronize(rb1));
                        add_time("rebuild", rb0, rb1);
                    }
                }
                h_ctr->steps_done = 0;
                h_chunk->steps_done = 0;
                h_chunk->halt = 0;
                h_chunk->iter0 = scenes[0].iter;
                HIPC(hipMemcpyAsync(reinterpret_cast<char*>(d_ctr.p) + offsetof(Counters, steps_done), h_chunk,
                                    sizeof(ChunkStart), hipMemcpyHostToDevice, stream));
                // graphs hold an even number of steps starting at parity 0
                const int n = (int)std::min<int64_t>(remaining, chunk);
                GraphEntry* ge = nullptr;
                const int par0 = next_parity;
                // timing mode launches directly: kernel events come from the
                // dispatch packets, which graph nodes do not expose here
                if (use_graph && !timing && n == chunk && chunk % 2 == 0 && par0 == 0) {
                    ge = &get_graph(n, ctrl_phase());
                    HIPC(hipGraphLaunch(ge->exec, stream));
                } else {
                    if (timing && direct_ev.size() < 4 * (size_t)n) {
                        const size_t old = direct_ev.size();
                        direct_ev.resize(4 * (size_t)n);
                        for (size_t q = old; q < direct_ev.size(); ++q) HIPC(hipEventCreate(&direct_ev[q]));
                    }
                    for (int i = 0; i < n; ++i)
                        launch_step((par0 + i) & 1, timing ? &direct_ev[4 * (size_t)i] : nullptr,
                                    measure_step(ctrl_phase(), i));
                }
                next_parity = (par0 + n) & 1;
                HIPC(hipGetLastError());
                read_counters();
                const int done = h_ctr->steps_done;
                if (done > 0) slots_fresh = false;
                if (timing)
                    for (int i = 0; i < done; ++i) {
                        add_time("contact", direct_ev[4 * (size_t)i], direct_ev[4 * (size_t)i + 1]);
                        add_time("integrate", direct_ev[4 * (size_t)i + 2], direct_ev[4 * (size_t)i + 3]);
                    }
                for (auto& S : scenes) {
                    S.iter += done;
                    S.time += done * S.p.dt;
                }
                remaining -= done;
                contacts_valid = done > 0 || contacts_valid;
                if (h_ctr->nonfinite) fail(DEM_ENONFINITE, "non-finite position or velocity after a step");
                if (h_ctr->unstable) fail(DEM_EUNSTABLE, "an overlap exceeded a sphere radius (numerically exploding)");
                const bool stalled = h_ctr->stall[next_parity ^ 1] != 0;
                if (done == 0 && !stalled) fail(DEM_EDEVICE, "no step completed");
                if (done < n && !stalled) fail(DEM_EDEVICE, "steps stopped without a broad-phase request");
                if (h_ctr->halt) {
                    // the controlled cell reached its goal; the stall flags it
                    // raised (with any broad-phase request of the same step)
                    // are cleared by the broad-phase run the next call starts with
                    halted = true;
                    need_rebuild = true;
                    break;
                }
            }
        } catch (...) {
            for (auto e : direct_ev) (void)hipEventDestroy(e);
            if (rb0) (void)hipEventDestroy(rb0);
            if (rb1) (void)hipEventDestroy(rb1);
            throw;
        }
        for (auto e : direct_ev) (void)hipEventDestroy(e);
        if (rb0) (void)hipEventDestroy(rb0);
        if (rb1) (void)hipEventDestroy(rb1);
        return halted;
    }

    // ------------------------------------------------------- read-back
    struct Snapshot {
        std::vector<double> x, y, z, vx, vy, vz, wx, wy, wz, qw, qx, qy, qz;
        std::vector<int32_t> id;
        std::vector<int32_t> slot_of;  // gid -> slot
    };

    Snapshot snapshot()
    {
        Snapshot s;
        const BodySet& B = bs[active];
        const size_t n = (size_t)nslots;
        std::vector<double> buf(4 * n);
        // packed 4-vectors: split the components into the snapshot's columns
        auto get = [&](const DBuf& d, std::vector<double>* cols[4]) {
            for (int c = 0; c < 4; ++c)
                if (cols[c]) cols[c]->resize(n);
            if (!n) return;
            HIPC(hipMemcpyAsync(buf.data(), d.p, 32 * n, hipMemcpyDeviceToHost, stream));
            HIPC(hipStreamSynchronize(stream));
            for (size_t i = 0; i < n; ++i)
                for (int c = 0; c < 4; ++c)
                    if (cols[c]) (*cols[c])[i] = buf[4 * i + c];
        };
        std::vector<double>* cx[4] = {&s.x, &s.y, &s.z, nullptr};
        std::vector<double>* cv[4] = {&s.vx, &s.vy, &s.vz, nullptr};
        std::vector<double>* cw[4] = {&s.wx, &s.wy, &s.wz, nullptr};
        std::vector<double>* cq[4] = {&s.qw, &s.qx, &s.qy, &s.qz};
        get(B.xr, cx);
        get(B.vm, cv);
        get(B.w, cw);
        get(B.q, cq);
        s.id.resize(n);
        if (n) HIPC(hipMemcpyAsync(s.id.data(), B.id.p, 4 * n, hipMemcpyDeviceToHost, stream));
        HIPC(hipStreamSynchronize(stream));
        s.slot_of.assign(bodies.size(), -1);
        for (size_t i = 0; i < n; ++i) s.slot_of[s.id[i]] = (int32_t)i;
        return s;
    }

    struct PairSnapshot {
        std::vector<int32_t> a, b, cell;
        std::vector<double> fsx, fsy, fsz, nx, ny, nz, fx, fy, fz;
        std::vector<double> pen, fn;   // overlap and normal force of the last evaluation
    };

    PairSnapshot pair_snapshot()
    {
        PairSnapshot p;
        const PairSet& P = ps[pactive];
        const size_t n = (size_t)npairs;
        auto gi = [&](const DBuf& d, std::vector<int32_t>& v) {
            v.resize(n);
            if (n) HIPC(hipMemcpyAsync(v.data(), d.p, 4 * n, hipMemcpyDeviceToHost, stream));
        };
        auto gd = [&](const DBuf& d, std::vector<double>& v) {
            v.resize(n);
            if (n) HIPC(hipMemcpyAsync(v.data(), d.p, 8 * n, hipMemcpyDeviceToHost, stream));
        };
        gi(P.a, p.a);
        gi(P.b, p.b);
        gi(P.cell, p.cell);
        {
            std::vector<HistRec> h(n);
            if (precision == DEM_FP32_MIXED) {
                std::vector<HistRec32> h32(n);
                if (n) HIPC(hipMemcpyAsync(h32.data(), P.hist.p, sizeof(HistRec32) * n, hipMemcpyDeviceToHost, stream));
                HIPC(hipStreamSynchronize(stream));
                for (size_t k = 0; k < n; ++k) h[k] = widen(h32[k]);
            } else {
                if (n) HIPC(hipMemcpyAsync(h.data(), P.hist.p, sizeof(HistRec) * n, hipMemcpyDeviceToHost, stream));
                HIPC(hipStreamSynchronize(stream));
            }
            for (auto* v : {&p.fsx, &p.fsy, &p.fsz, &p.nx, &p.ny, &p.nz, &p.pen, &p.fn}) v->resize(n);
            for (size_t k = 0; k < n; ++k) {
                p.pen[k] = h[k].pen;
                p.fn[k] = h[k].fn;
                p.fsx[k] = h[k].fsx;
                p.fsy[k] = h[k].fsy;
                p.fsz[k] = h[k].fsz;
                p.nx[k] = h[k].nx;
                p.ny[k] = h[k].ny;
                p.nz[k] = h[k].nz;
            }
        }
        // force on #2 of every pair
        p.fx.assign(n, 0.0);
        p.fy.assign(n, 0.0);
        p.fz.assign(n, 0.0);
        if (n) {
            d_tmp3.ensure(sizeof(double) * 3 * n);
            StepArgs a = step_args();
            launch_pair_forces(a, precision, d_tmp3.as<double>(), stream);
            HIPC(hipGetLastError());
            std::vector<double> f(3 * n);
            HIPC(hipMemcpyAsync(f.data(), d_tmp3.p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, stream));
            HIPC(hipStreamSynchronize(stream));
            for (size_t k = 0; k < n; ++k) {
                p.fx[k] = f[3 * k];
                p.fy[k] = f[3 * k + 1];
                p.fz[k] = f[3 * k + 2];
            }
        }
        HIPC(hipStreamSynchronize(stream));
        return p;
    }

    void check_scene_id(int s, int64_t first, int64_t count) const
    {
        if (first < 0 || count < 0 || first + count > (int64_t)scenes[s].gids.size())
            fail(DEM_ERANGE, "Body id out of range");
    }

    // Reported position of a boundary: a plane's coordinate on its axis (0
    // elsewhere), a box's centre, a facet's centroid.
    static double boundary_position(const Wall& W, int k)
    {
        if (W.kind == kPlane) return k == W.axis ? W.pos : 0.0;
        if (W.kind == kBox) return 0.5 * (W.g[k] + W.g[3 + k]);
        return (W.g[k] + W.g[3 + k] + W.g[6 + k]) / 3.0;
    }

    void get_state(int s, int64_t first, int64_t count, double* pos3, double* vel3, double* angvel3, double* ori4,
                   double* force3, double* torque3)
    {
        check_scene_id(s, first, count);
        const HostScene& S = scenes[s];
        if (host_dirty || !on_device) {
            for (int64_t i = 0; i < count; ++i) {
                const HostBody& b = bodies[S.gids[first + i]];
                for (int k = 0; k < 3; ++k) {
                    if (pos3) pos3[3 * i + k] = b.kind ? boundary_position(walls[b.wall], k) : b.x[k];
                    if (vel3) vel3[3 * i + k] = b.v[k];
                    if (angvel3) angvel3[3 * i + k] = b.w[k];
                    if (force3) force3[3 * i + k] = 0.0;
                    if (torque3) torque3[3 * i + k] = 0.0;
                }
                if (ori4)
                    for (int k = 0; k < 4; ++k) ori4[4 * i + k] = b.q[k];
            }
            return;
        }
        Snapshot sn = snapshot();
        std::vector<double> f, t;
        std::vector<double> wallF(3 * walls.size(), 0.0);
        if (force3 || torque3) {
            f.assign(3 * (size_t)nslots, 0.0);
            t.assign(3 * (size_t)nslots, 0.0);
            if (nslots > 0 && contacts_valid) {
                d_tmp3.ensure(sizeof(double) * 6 * (size_t)nslots);
                StepArgs a = step_args();
                launch_body_forces(a, precision, d_tmp3.as<double>(), d_tmp3.as<double>() + 3 * (size_t)nslots, stream);
                HIPC(hipGetLastError());
                HIPC(hipMemcpyAsync(f.data(), d_tmp3.p, 8 * 3 * (size_t)nslots, hipMemcpyDeviceToHost, stream));
                HIPC(hipMemcpyAsync(t.data(), d_tmp3.as<double>() + 3 * (size_t)nslots, 8 * 3 * (size_t)nslots,
                                    hipMemcpyDeviceToHost, stream));
                HIPC(hipStreamSynchronize(stream));
                // reaction on walls: minus the force on the sphere, in pair order
                PairSnapshot p = pair_snapshot();
                for (int k = 0; k < npairs; ++k)
                    if (p.a[k] < 0 && (p.nx[k] != 0.0 || p.ny[k] != 0.0 || p.nz[k] != 0.0)) {
                        const int w = -1 - p.a[k];
                        wallF[3 * w + 0] += -p.fx[k];
                        wallF[3 * w + 1] += -p.fy[k];
                        wallF[3 * w + 2] += -p.fz[k];
                    }
            }
        }
        for (int64_t i = 0; i < count; ++i) {
            const int32_t g = S.gids[first + i];
            const HostBody& b = bodies[g];
            if (b.kind == 1) {
                const Wall& W = walls[b.wall];
                for (int k = 0; k < 3; ++k) {
                    if (pos3) pos3[3 * i + k] = boundary_position(W, k);
                    if (vel3) vel3[3 * i + k] = 0.0;
                    if (angvel3) angvel3[3 * i + k] = 0.0;
                    if (force3) force3[3 * i + k] = wallF[3 * b.wall + k];
                    if (torque3) torque3[3 * i + k] = 0.0;
                }
                if (ori4) {
                    ori4[4 * i] = 1.0;
                    ori4[4 * i + 1] = ori4[4 * i + 2] = ori4[4 * i + 3] = 0.0;
                }
                continue;
            }
            const int sl = sn.slot_of[g];
            if (pos3) {
                pos3[3 * i] = sn.x[sl];
                pos3[3 * i + 1] = sn.y[sl];
                pos3[3 * i + 2] = sn.z[sl];
            }
            if (vel3) {
                vel3[3 * i] = sn.vx[sl];
                vel3[3 * i + 1] = sn.vy[sl];
                vel3[3 * i + 2] = sn.vz[sl];
            }
            if (angvel3) {
                angvel3[3 * i] = sn.wx[sl];
                angvel3[3 * i + 1] = sn.wy[sl];
                angvel3[3 * i + 2] = sn.wz[sl];
            }
            if (ori4) {
                ori4[4 * i] = sn.qw[sl];
                ori4[4 * i + 1] = sn.qx[sl];
                ori4[4 * i + 2] = sn.qy[sl];
                ori4[4 * i + 3] = sn.qz[sl];
            }
            for (int k = 0; k < 3; ++k) {
                if (force3) force3[3 * i + k] = f[3 * (size_t)sl + k];
                if (torque3) torque3[3 * i + k] = t[3 * (size_t)sl + k];
            }
        }
    }

    void set_state(int s, const double* pos3, const double* vel3, const double* angvel3, const double* ori4)
    {
        const HostScene& S = scenes[s];
        for (size_t i = 0; i < 3 * S.gids.size(); ++i)
            if ((pos3 && !std::isfinite(pos3[i])) || (vel3 && !std::isfinite(vel3[i])) ||
                (angvel3 && !std::isfinite(angvel3[i])))
                fail(DEM_EINVAL, "dem_set_state: non-finite value");
        pull_bodies();
        for (size_t i = 0; i < S.gids.size(); ++i) {
            HostBody& b = bodies[S.gids[i]];
            if (b.kind != 0) continue;
            for (int k = 0; k < 3; ++k) {
                if (pos3) b.x[k] = pos3[3 * i + k];
                if (vel3) b.v[k] = vel3[3 * i + k];
                if (angvel3) b.w[k] = angvel3[3 * i + k];
            }
            if (ori4)
                for (int k = 0; k < 4; ++k) b.q[k] = ori4[4 * i + k];
        }
        host_dirty = true;
        need_rebuild = true;
    }

    // local id of a gid within its scene
    std::vector<int64_t> local_ids() const
    {
        std::vector<int64_t> loc(bodies.size(), -1);
        for (const HostScene& S : scenes)
            for (size_t i = 0; i < S.gids.size(); ++i) loc[S.gids[i]] = (int64_t)i;
        return loc;
    }

    static void unpack_cell(int32_t p, int32_t* c)
    {
        const uint32_t u = (uint32_t)p;
        c[0] = (int32_t)((u >> 20) & 1023u) - 512;
        c[1] = (int32_t)((u >> 10) & 1023u) - 512;
        c[2] = (int32_t)(u & 1023u) - 512;
    }

    // Love-Weber stress of scene s: partial sums per block on the device,
    // combined here in block order, divided by the volume (periodic: the
    // cell's, else the caller's).
    // O.dt between steps
    void set_dt(int s, double dt)
    {
        pull_scene_table();
        scenes[s].p.dt = dt;
        sp[s].dt = dt;
        push_scene_table();
        if (d_args.p) upload_args();
        update_cell_step();
    }
    // Cell.velGrad between steps: the next step sees it, and the last
    // step's one as the previous gradient
    void set_velgrad(int s, const double* L9)
    {
        pull_scene_table();
        for (int k = 0; k < 9; ++k) {
            scenes[s].p.velgrad[k] = L9[k];
            sp[s].L[k] = L9[k];
        }
        // the mean field's share of the Verlet budget changes from the next
        // step on; what the bodies' accounts hold stays valid
        double lf = 0.0;
        for (int k = 0; k < 9; ++k) lf += L9[k] * L9[k];
        sp[s].verlet_cell_rate = 0.5 * std::sqrt(lf) * (2.0 * scenes[s].rmax + 4.0 * sp[s].verlet);
        push_scene_table();
        if (d_args.p) upload_args();
        update_cell_step();
    }

    // Device sums over the last step's contacts and bodies of scene s, in a
    // fixed block order (the kernels reduce waves in a fixed order too).
    struct Measures {
        double sigma[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // times the volume
        double modulus[3] = {0, 0, 0};                   // times the volume
        double contact_force_sum = 0.0, contacts = 0.0;
        double body_force_sum = 0.0, body_force_max = 0.0, bodies_dyn = 0.0;
        double min_dt = INFINITY;
    };
    Measures measures(int s)
    {
        Measures m;
        if (host_dirty) upload_bodies();
        if (!contacts_valid || nslots == 0) return m;
        const int np = npairs > 0 ? stress_blocks(npairs) : 0;
        const int nb = body_blocks(nslots);
        d_tmp3.ensure(sizeof(double) * ((size_t)kNetworkWords * np + (size_t)kBodyWords * nb));
        double* part_p = d_tmp3.as<double>();
        double* part_b = part_p + (size_t)kNetworkWords * np;
        const StepArgs a = step_args();
        const bool batched = scenes.size() > 1;
        if (np > 0) launch_network(a, precision, batched, s, part_p, stream);
        launch_body_measures(a, precision, batched, s, part_b, stream);
        HIPC(hipGetLastError());
        std::vector<double> hp((size_t)kNetworkWords * np), hb((size_t)kBodyWords * nb);
        if (np > 0)
            HIPC(hipMemcpyAsync(hp.data(), part_p, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, stream));
        HIPC(hipMemcpyAsync(hb.data(), part_b, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, stream));
        HIPC(hipStreamSynchronize(stream));
        for (int b = 0; b < np; ++b) {
            const double* q = &hp[(size_t)kNetworkWords * b];
            for (int k = 0; k < 9; ++k) m.sigma[k] += q[k];
            for (int k = 0; k < 3; ++k) m.modulus[k] += q[9 + k];
            m.contact_force_sum += q[12];
            m.contacts += q[13];
        }
        for (int b = 0; b < nb; ++b) {
            const double* q = &hb[(size_t)kBodyWords * b];
            m.body_force_sum += q[0];
            m.body_force_max = std::max(m.body_force_max, q[1]);
            m.bodies_dyn += q[2];
            m.min_dt = std::min(m.min_dt, q[3]);
        }
        return m;
    }
    static double unbalanced_of(const Measures& m, bool use_max)
    {
        if (!(m.contacts > 0.0) || !(m.bodies_dyn > 0.0)) return NAN;
        const double mean_contact = m.contact_force_sum / m.contacts;
        const double top = use_max ? m.body_force_max : m.body_force_sum / m.bodies_dyn;
        return top / mean_contact;
    }
    double stiffness_dt(int s, double safety)
    {
        if (has_viscel()) fail(DEM_EINVAL, "dem_stiffness_dt: not available with visco-elastic materials");
        const Measures m = measures(s);
        if (std::isinf(m.min_dt)) return safety * pwave_dt(s);
        return safety * m.min_dt;
    }

    // ---- GlobalStiffnessTimeStepper and the stress-controlled cell, run
    // between steps by step() (scene 0 of an unbatched world)
    double ts_safety = 0.8;
    int64_t ts_interval = 0;
    bool pt_active = false;
    bool pt_iso = false;        // the active controller is the isotropic compressor
    int pt_glob_update = 1;

    void set_peri_triax(const dem_peri_triax* c)
    {
        CtrlConfig k;
        std::memset(&k, 0, sizeof k);
        if (c) {
            for (int i = 0; i < 3; ++i) {
                k.goal[i] = c->goal[i];
                k.max_rate[i] = c->max_strain_rate[i];
            }
            k.stress_mask = c->stress_mask;
            k.glob_update = c->glob_update;
            k.grow_damping = c->grow_damping;
            k.max_unbalanced = c->max_unbalanced;
            k.abs_tol = c->abs_stress_tol;
            k.rel_tol = c->rel_stress_tol;
            k.stop_when_done = c->stop_when_done;
            k.active = 1;
        } else {
            k.glob_update = 1;
        }
        HIPC(hipMemcpyAsync(d_ctrl_cfg.p, &k, sizeof k, hipMemcpyHostToDevice, stream));
        if (c) {
            CtrlState st;
            std::memset(&st, 0, sizeof st);
            st.unbalanced = NAN;
            HIPC(hipMemcpyAsync(d_ctrl_state.p, &st, sizeof st, hipMemcpyHostToDevice, stream));
        }
        HIPC(hipStreamSynchronize(stream));
        pt_active = c != nullptr;
        pt_iso = false;
        pt_glob_update = c ? c->glob_update : 1;
        if (d_args.p) upload_args();
    }
    // The isotropic compressor through a stress series: the same device
    // controller in its iso mode.
    void set_peri_iso(const dem_peri_iso* c)
    {
        CtrlConfig k;
        std::memset(&k, 0, sizeof k);
        k.iso = 1;
        k.stress_mask = 7;
        k.n_series = c->n_stresses;
        for (int j = 0; j < c->n_stresses; ++j) k.series[j] = c->stresses[j];
        for (int i = 0; i < 3; ++i) {
            k.goal[i] = c->stresses[0];
            k.max_rate[i] = c->max_strain_rate;
        }
        k.glob_update = c->global_update;
        k.grow_damping = c->grow_damping;
        k.max_unbalanced = c->max_unbalanced;
        k.abs_tol = c->abs_stress_tol;
        k.rel_tol = c->rel_stress_tol;
        k.stop_when_done = c->stop_when_done;
        k.active = 1;
        HIPC(hipMemcpyAsync(d_ctrl_cfg.p, &k, sizeof k, hipMemcpyHostToDevice, stream));
        CtrlState st;
        std::memset(&st, 0, sizeof st);
        st.unbalanced = NAN;
        HIPC(hipMemcpyAsync(d_ctrl_state.p, &st, sizeof st, hipMemcpyHostToDevice, stream));
        HIPC(hipStreamSynchronize(stream));
        pt_active = true;
        pt_iso = true;
        pt_glob_update = c->global_update;
        if (d_args.p) upload_args();
    }
    dem_peri_iso_state peri_iso_state()
    {
        CtrlState st;
        HIPC(hipMemcpyAsync(&st, d_ctrl_state.p, sizeof st, hipMemcpyDeviceToHost, stream));
        HIPC(hipStreamSynchronize(stream));
        dem_peri_iso_state o;
        std::memset(&o, 0, sizeof o);
        o.state = st.series_index;
        o.done = st.done;
        o.sigma = (st.stress[0] + st.stress[1] + st.stress[2]) / 3.0;
        o.stiff = (st.stiff[0] + st.stiff[1] + st.stiff[2]) / 3.0;
        o.strain_rate = st.rate[0];
        o.unbalanced = st.unbalanced;
        o.updates = st.updates;
        o.active = (pt_active && pt_iso) ? 1 : 0;
        return o;
    }

    dem_peri_triax_state peri_triax_state()
    {
        CtrlState st;
        HIPC(hipMemcpyAsync(&st, d_ctrl_state.p, sizeof st, hipMemcpyDeviceToHost, stream));
        HIPC(hipStreamSynchronize(stream));
        dem_peri_triax_state o;
        std::memset(&o, 0, sizeof o);
        for (int i = 0; i < 3; ++i) {
            o.stress[i] = st.stress[i];
            o.strain[i] = st.strain[i];
            o.strain_rate[i] = st.rate[i];
            o.stiff[i] = st.stiff[i];
        }
        o.unbalanced = st.unbalanced;
        o.updates = st.updates;
        o.done = st.done;
        o.active = (pt_active && !pt_iso) ? 1 : 0;
        return o;
    }

    void stress(int s, double volume, double* out9)
    {
        double V = volume;
        if (!(V > 0.0)) {
            if (!scenes[s].p.periodic) fail(DEM_EINVAL, "dem_get_stress: give the volume of an aperiodic scene");
            pull_scene_table();
            const double* H = sp[s].H;
            V = std::fabs(H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                          H[2] * (H[3] * H[7] - H[4] * H[6]));
        }
        if (!std::isfinite(V) || !(V > 0.0)) fail(DEM_EINVAL, "dem_get_stress: volume must be > 0");
        double sum[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (host_dirty) upload_bodies();
        const int nb = (contacts_valid && npairs > 0) ? stress_blocks(npairs) : 0;
        if (nb > 0) {
            d_tmp3.ensure(sizeof(double) * kNetworkWords * (size_t)nb);
            StepArgs a = step_args();
            launch_network(a, precision, scenes.size() > 1, s, d_tmp3.as<double>(), stream);
            HIPC(hipGetLastError());
            std::vector<double> part(kNetworkWords * (size_t)nb);
            HIPC(hipMemcpyAsync(part.data(), d_tmp3.p, sizeof(double) * part.size(), hipMemcpyDeviceToHost, stream));
            HIPC(hipStreamSynchronize(stream));
            for (int b = 0; b < nb; ++b)
                for (int q = 0; q < 9; ++q) sum[q] += part[kNetworkWords * (size_t)b + q];
        }
        for (int q = 0; q < 9; ++q) out9[q] = sum[q] / V;
    }

    // The same sums in the library's fixed device scratch: no device or host
    // allocation (the device state must already be current, so bodies added
    // or a state set since the last step are refused rather than uploaded).
    void stress_noalloc(int s, double volume, double* out9)
    {
        if (host_dirty)
            fail(DEM_EINVAL, "dem_get_stress_noalloc: bodies or state changed since the last step; step first");
        double V = volume;
        if (!(V > 0.0)) {
            if (!scenes[s].p.periodic) fail(DEM_EINVAL, "dem_get_stress_noalloc: give the volume of an aperiodic scene");
            pull_scene_table();
            const double* H = sp[s].H;
            V = std::fabs(H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                          H[2] * (H[3] * H[7] - H[4] * H[6]));
        }
        if (!std::isfinite(V) || !(V > 0.0)) fail(DEM_EINVAL, "dem_get_stress_noalloc: volume must be > 0");
        double sum[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (contacts_valid && npairs > 0) {
            if ((int64_t)npairs > stress_noalloc_max_pairs())
                fail(DEM_EINVAL, "dem_get_stress_noalloc: " + std::to_string(npairs) +
                                     " candidate pairs exceed the fixed scratch's limit of " +
                                     std::to_string(stress_noalloc_max_pairs()));
            const double* d = launch_stress_noalloc(step_args(), precision, scenes.size() > 1, s, stream);
            if (!d) fail(DEM_EDEVICE, "dem_get_stress_noalloc: the device scratch's address is not available");
            HIPC(hipGetLastError());
            HIPC(hipMemcpyAsync(sum, d, sizeof sum, hipMemcpyDeviceToHost, stream));
            HIPC(hipStreamSynchronize(stream));
        }
        for (int q = 0; q < 9; ++q) out9[q] = sum[q] / V;
    }

    std::vector<dem_contact> contacts(int s)
    {
        std::vector<dem_contact> out;
        if (!contacts_valid || host_dirty || npairs == 0) return out;
        Snapshot sn = snapshot();
        PairSnapshot p = pair_snapshot();
        const std::vector<int64_t> loc = local_ids();
        for (int k = 0; k < npairs; ++k) {
            const double nn = p.nx[k] * p.nx[k] + p.ny[k] * p.ny[k] + p.nz[k] * p.nz[k];
            if (!(nn > 0.0)) continue;
            const int sb = p.b[k];
            const int32_t g2 = sn.id[sb];
            const HostBody& B2 = bodies[g2];
            if (B2.scene != s) continue;
            dem_contact c;
            std::memset(&c, 0, sizeof c);
            const bool wall = p.a[k] < 0;
            const HostBody* B1 = nullptr;
            int32_t g1;
            if (wall) {
                g1 = walls[-1 - p.a[k]].id;
            } else {
                g1 = sn.id[p.a[k]];
                B1 = &bodies[g1];
            }
            c.id1 = loc[g1];
            c.id2 = loc[g2];
            c.is_wall = wall ? 1 : 0;
            unpack_cell(p.cell[k], c.cell);
            c.normal[0] = p.nx[k];
            c.normal[1] = p.ny[k];
            c.normal[2] = p.nz[k];
            // the kernel's own overlap and normal force (history record); the
            // shear force is the stored spring (linear law) or the total less
            // the normal force (visco-elastic law, whose dashpot is not stored)
            c.pen = p.pen[k];
            for (int q = 0; q < 3; ++q) c.fn[q] = p.fn[k] * c.normal[q];
            c.fs[0] = p.fsx[k];
            c.fs[1] = p.fsy[k];
            c.fs[2] = p.fsz[k];
            const HostMaterial& M2 = mats[B2.mat];
            const HostMaterial& M1 = wall ? mats[walls[-1 - p.a[k]].mat] : mats[B1->mat];
            const double R1 = wall ? (walls[-1 - p.a[k]].kind == kFacet ? 2.0 * B2.r : B2.r) : B1->r, R2 = B2.r;
            if (M2.kind == 1) {
                // visco-elastic law: the kernel left the overlap and the signed
                // normal force in the history record; the shear force reported
                // is the total (spring and dashpot) less the normal force
                const bool fixed1 = wall || B1->blocked == 63u, fixed2 = B2.blocked == 63u;
                const double m1 = wall ? 0.0 : B1->m;
                double mr = m1 * B2.m / (m1 + B2.m);
                if (fixed1 && !fixed2) mr = B2.m;
                if (fixed2 && !fixed1) mr = m1;
                const double tc = 0.5 * (M1.tc + M2.tc);
                const double len = std::log(0.5 * (M1.en + M2.en)), let = std::log(0.5 * (M1.et + M2.et));
                const double pi2 = 3.14159265358979323846 * 3.14159265358979323846;
                c.kn = mr * (pi2 + len * len) / (tc * tc);
                c.ks = 2.0 / 7.0 * mr * (pi2 + let * let) / (tc * tc);
                c.fs[0] = p.fx[k] - c.fn[0];
                c.fs[1] = p.fy[k] - c.fn[1];
                c.fs[2] = p.fz[k] - c.fn[2];
            } else {
                const double k1 = M1.young * (2.0 * R1), k2 = M2.young * (2.0 * R2);
                c.kn = k1 * k2 / (k1 + k2);
                const double q1 = (M1.young * M1.poisson) * (2.0 * R1), q2 = (M2.young * M2.poisson) * (2.0 * R2);
                c.ks = q1 * q2 / (q1 + q2);
            }
            const double dt = scenes[s].p.dt;
            // positions of the step the contact was evaluated at: x - v dt
            const double x2[3] = {sn.x[sb] - sn.vx[sb] * dt, sn.y[sb] - sn.vy[sb] * dt, sn.z[sb] - sn.vz[sb] * dt};
            if (wall) {
                for (int q = 0; q < 3; ++q) c.point[q] = x2[q] - (R2 - 0.5 * c.pen) * c.normal[q];
            } else {
                const int sa = p.a[k];
                const double x1[3] = {sn.x[sa] - sn.vx[sa] * dt, sn.y[sa] - sn.vy[sa] * dt, sn.z[sa] - sn.vz[sa] * dt};
                for (int q = 0; q < 3; ++q) c.point[q] = x1[q] + (R1 - 0.5 * c.pen) * c.normal[q];
            }
            out.push_back(c);
        }
        std::sort(out.begin(), out.end(), [](const dem_contact& a, const dem_contact& b) {
            const int64_t alo = std::min(a.id1, a.id2), ahi = std::max(a.id1, a.id2);
            const int64_t blo = std::min(b.id1, b.id2), bhi = std::max(b.id1, b.id2);
            if (alo != blo) return alo < blo;
            if (ahi != bhi) return ahi < bhi;
            for (int q = 0; q < 3; ++q)
                if (a.cell[q] != b.cell[q]) return a.cell[q] < b.cell[q];
            return false;
        });
        return out;
    }

    void set_history(int s, int64_t n, const dem_history* in)
    {
        if (n < 0 || (n > 0 && !in)) fail(DEM_EINVAL, "dem_set_history: bad arguments");
        if (host_dirty) upload_bodies();
        const HostScene& S = scenes[s];
        struct Rec {
            int32_t owner, partner, cell;
            double fs[3], n[3];
        };
        std::vector<Rec> recs;
        recs.reserve((size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            const dem_history& h = in[i];
            if (h.id1 < 0 || h.id2 < 0 || h.id1 >= (int64_t)S.gids.size() || h.id2 >= (int64_t)S.gids.size() ||
                h.id1 == h.id2)
                fail(DEM_ERANGE, "dem_set_history: body id out of range");
            int32_t g1 = S.gids[h.id1], g2 = S.gids[h.id2];
            int32_t c[3] = {h.cell[0], h.cell[1], h.cell[2]};
            const bool w1 = bodies[g1].kind == 1, w2 = bodies[g2].kind == 1;
            if (w1 && w2) fail(DEM_EINVAL, "dem_set_history: wall-wall record");
            Rec r;
            if (w1 || w2) {
                r.owner = w1 ? g2 : g1;
                r.partner = w1 ? g1 : g2;
                c[0] = c[1] = c[2] = 0;
            } else if (g1 < g2) {
                r.owner = g1;
                r.partner = g2;
            } else {
                r.owner = g2;
                r.partner = g1;
                for (int q = 0; q < 3; ++q) c[q] = -c[q];
            }
            for (int q = 0; q < 3; ++q)
                if (c[q] < -512 || c[q] > 511) fail(DEM_EINVAL, "dem_set_history: cell shift out of range");
            r.cell = (int32_t)(((uint32_t)(c[0] + 512) << 20) | ((uint32_t)(c[1] + 512) << 10) | (uint32_t)(c[2] + 512));
            for (int q = 0; q < 3; ++q) {
                r.fs[q] = h.fs[q];
                r.n[q] = h.nprev[q];
            }
            recs.push_back(r);
        }
        std::sort(recs.begin(), recs.end(), [](const Rec& a, const Rec& b) {
            if (a.owner != b.owner) return a.owner < b.owner;
            if (a.partner != b.partner) return a.partner < b.partner;
            return (uint32_t)a.cell < (uint32_t)b.cell;
        });
        // keep the history of other scenes: merge with the current real contacts
        std::vector<Rec> keep;
        if (scenes.size() > 1 && contacts_valid && npairs > 0) {
            Snapshot sn = snapshot();
            PairSnapshot p = pair_snapshot();
            for (int k = 0; k < npairs; ++k) {
                const double nn = p.nx[k] * p.nx[k] + p.ny[k] * p.ny[k] + p.nz[k] * p.nz[k];
                if (!(nn > 0.0)) continue;
                const int32_t g2 = sn.id[p.b[k]];
                if (bodies[g2].scene == s) continue;
                Rec r;
                if (p.a[k] < 0) {
                    r.owner = g2;
                    r.partner = walls[-1 - p.a[k]].id;
                } else {
                    r.owner = sn.id[p.a[k]];
                    r.partner = g2;
                }
                r.cell = p.cell[k];
                r.fs[0] = p.fsx[k];
                r.fs[1] = p.fsy[k];
                r.fs[2] = p.fsz[k];
                r.n[0] = p.nx[k];
                r.n[1] = p.ny[k];
                r.n[2] = p.nz[k];
                keep.push_back(r);
            }
        }
        recs.insert(recs.end(), keep.begin(), keep.end());
        std::sort(recs.begin(), recs.end(), [](const Rec& a, const Rec& b) {
            if (a.owner != b.owner) return a.owner < b.owner;
            if (a.partner != b.partner) return a.partner < b.partner;
            return (uint32_t)a.cell < (uint32_t)b.cell;
        });
        const int ng = (int)bodies.size();
        std::vector<int32_t> ob((size_t)std::max(ng, 1), 0), oc((size_t)std::max(ng, 1), 0);
        for (size_t i = 0; i < recs.size(); ++i) {
            if (oc[recs[i].owner] == 0) ob[recs[i].owner] = (int32_t)i;
            oc[recs[i].owner] += 1;
        }
        const size_t m = recs.size();
        PairSet& P = ps[pactive];
        P.ensure(std::max<size_t>(m, (size_t)npairs), precision == DEM_FP32_MIXED);
        P.own_begin.ensure(4 * (size_t)std::max(ng, 1));
        P.own_count.ensure(4 * (size_t)std::max(ng, 1));
        std::vector<int32_t> pid(m), cell(m);
        std::vector<HistRec> h(m);
        std::vector<HistRec32> h32(precision == DEM_FP32_MIXED ? m : 0);
        for (size_t i = 0; i < m; ++i) {
            pid[i] = recs[i].partner;
            cell[i] = recs[i].cell;
            h[i] = HistRec{recs[i].fs[0], recs[i].fs[1], recs[i].fs[2], 0.0, recs[i].n[0], recs[i].n[1], recs[i].n[2], 0.0};
            if (!h32.empty())
                h32[i] = HistRec32{recs[i].fs[0], recs[i].fs[1], recs[i].fs[2], 0.0, (float)recs[i].n[0],
                                   (float)recs[i].n[1], (float)recs[i].n[2], 0.0f};
        }
        HIPC(hipMemcpyAsync(P.own_begin.p, ob.data(), 4 * (size_t)ng, hipMemcpyHostToDevice, stream));
        HIPC(hipMemcpyAsync(P.own_count.p, oc.data(), 4 * (size_t)ng, hipMemcpyHostToDevice, stream));
        std::vector<int32_t> ident(m);
        for (size_t i = 0; i < m; ++i) ident[i] = (int32_t)i;
        if (m) {
            HIPC(hipMemcpyAsync(P.hpid.p, pid.data(), 4 * m, hipMemcpyHostToDevice, stream));
            HIPC(hipMemcpyAsync(P.hcell.p, cell.data(), 4 * m, hipMemcpyHostToDevice, stream));
            HIPC(hipMemcpyAsync(P.hmap.p, ident.data(), 4 * m, hipMemcpyHostToDevice, stream));
            if (h32.empty())
                HIPC(hipMemcpyAsync(P.hist.p, h.data(), sizeof(HistRec) * m, hipMemcpyHostToDevice, stream));
            else
                HIPC(hipMemcpyAsync(P.hist.p, h32.data(), sizeof(HistRec32) * m, hipMemcpyHostToDevice, stream));
        }
        HIPC(hipStreamSynchronize(stream));
        old_ngids = ng;
        npairs = 0;  // the active set now only holds history: nothing to report until the next step
        contacts_valid = false;
        need_rebuild = true;
        invalidate_graphs();
    }
};

}  // namespace
}  // namespace dem

// ======================================================================
//                                C ABI
// ======================================================================

struct dem_scene {
    dem::World* w;
    int s;
    bool owner;
};
struct dem_batch {
    dem::World* w;
    std::vector<dem_scene> views;
};

namespace {

template <typename F>
dem_status guarded(F&& f)
{
    try {
        f();
        dem::g_err.clear();
        return DEM_OK;
    } catch (const dem::Error& e) {
        dem::g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        dem::g_err = "host allocation failed";
        return DEM_ENOMEM;
    } catch (const std::exception& e) {
        dem::g_err = e.what();
        return DEM_EINVAL;
    }
}

void check_params(const dem_params* p)
{
    if (!p) dem::fail(DEM_EINVAL, "null params");
    if (!(p->dt >= 0.0) || !std::isfinite(p->dt)) dem::fail(DEM_EINVAL, "dt must be >= 0 and finite");
    if (!(p->damping >= 0.0 && p->damping < 1.0)) dem::fail(DEM_EINVAL, "damping must be in [0, 1)");
    if (p->precision != DEM_FP64 && p->precision != DEM_FP32_MIXED) dem::fail(DEM_EINVAL, "unknown precision");
    if (p->homo_deform < 0 || p->homo_deform > 2) dem::fail(DEM_EINVAL, "homo_deform must be 0, 1 or 2");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(p->gravity[k])) dem::fail(DEM_EINVAL, "gravity must be finite");
    if (p->periodic) {
        double inv[9];
        if (!dem::World::invert(p->hsize, inv)) dem::fail(DEM_EINVAL, "singular cell matrix");
    }
}

dem::World* world_of(dem_scene* s)
{
    if (!s || !s->w) dem::fail(DEM_EINVAL, "null scene");
    if (s->w->busy.load()) dem::fail(DEM_EBUSY, "an asynchronous step is in flight: call dem_wait first");
    HIPC(hipSetDevice(s->w->device));
    return s->w;
}

void check_steppable(dem_scene* s, dem::World* w)
{
    if (!s->owner) dem::fail(DEM_EINVAL, "dem_step: step the batch, not one of its scenes");
    for (const auto& S : w->scenes)
        if (!(S.p.dt > 0.0)) dem::fail(DEM_EINVAL, "dem_step: dt is not set");
}

}  // namespace

extern "C" {

int32_t dem_abi_version(void) { return DEM_ABI_VERSION; }

const char* dem_last_error(void) { return dem::g_err.c_str(); }

void dem_params_default(dem_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->damping = 0.2;
    p->damp_rot = 1;
    p->verlet_dist = -0.5;
    p->precision = DEM_FP64;
    p->homo_deform = 2;
    for (int k = 0; k < 9; ++k) p->hsize[k] = (k % 4 == 0) ? 1.0 : 0.0;
}

dem_status dem_create(const dem_params* p, dem_scene** out)
{
    return guarded([&] {
        check_params(p);
        if (!out) dem::fail(DEM_EINVAL, "null out");
        std::unique_ptr<dem::World> w(new dem::World());
        w->init(1, p);
        *out = new dem_scene{w.release(), 0, true};
    });
}

dem_status dem_destroy(dem_scene* s)
{
    return guarded([&] {
        if (!s) dem::fail(DEM_EINVAL, "null scene");
        if (!s->owner) dem::fail(DEM_EINVAL, "dem_destroy: batch views are owned by the batch");
        if (s->w->worker.joinable()) s->w->worker.join();
        (void)hipSetDevice(s->w->device);
        delete s->w;
        delete s;
    });
}

dem_status dem_add_material(dem_scene* s, double density, double young, double poisson, double friction_angle,
                            int32_t* out_mat)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        const int m = w->add_material(density, young, poisson, friction_angle);
        if (out_mat) *out_mat = m;
    });
}

dem_status dem_add_viscel_material(dem_scene* s, double density, double tc, double en, double et,
                                   double friction_angle, int32_t* out_mat)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        const int m = w->add_viscel_material(density, tc, en, et, friction_angle);
        if (out_mat) *out_mat = m;
    });
}

dem_status dem_add_spheres(dem_scene* s, int64_t n, const double* pos3, const double* radius, const double* vel3,
                           const double* angvel3, const int32_t* mat, int32_t default_mat, const uint8_t* blocked,
                           int64_t* out_first_id)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        const int64_t first = w->add_spheres(s->s, n, pos3, radius, vel3, angvel3, mat, default_mat, blocked);
        if (out_first_id) *out_first_id = first;
    });
}

dem_status dem_add_wall(dem_scene* s, int32_t axis, double position, int32_t sense, int32_t mat, int64_t* out_id)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        const int64_t id = w->add_wall(s->s, axis, position, sense, mat);
        if (out_id) *out_id = id;
    });
}

dem_status dem_add_box(dem_scene* s, const double* center3, const double* half3, int32_t mat, int64_t* out_id)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        const int64_t id = w->add_box(s->s, center3, half3, mat);
        if (out_id) *out_id = id;
    });
}

dem_status dem_add_facet(dem_scene* s, const double* v0, const double* v1, const double* v2, int32_t mat,
                         int64_t* out_id)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        const int64_t id = w->add_facet(s->s, v0, v1, v2, mat);
        if (out_id) *out_id = id;
    });
}

dem_status dem_pwave_dt(dem_scene* s, double* out)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!out) dem::fail(DEM_EINVAL, "null out");
        *out = w->pwave_dt(s->s);
    });
}

dem_status dem_set_dt(dem_scene* s, double dt)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!(dt > 0.0) || !std::isfinite(dt)) dem::fail(DEM_EINVAL, "dt must be > 0");
        w->set_dt(s->s, dt);
    });
}

dem_status dem_set_velgrad(dem_scene* s, const double* velgrad9)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!velgrad9) dem::fail(DEM_EINVAL, "null velgrad");
        if (!w->scenes[s->s].p.periodic) dem::fail(DEM_EINVAL, "dem_set_velgrad: scene is not periodic");
        for (int k = 0; k < 9; ++k)
            if (!std::isfinite(velgrad9[k])) dem::fail(DEM_EINVAL, "dem_set_velgrad: non-finite entry");
        w->set_velgrad(s->s, velgrad9);
    });
}

dem_status dem_get_cell(dem_scene* s, double* hsize9, double* trsf9)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        w->pull_scene_table();
        for (int k = 0; k < 9; ++k) {
            if (hsize9) hsize9[k] = w->sp[s->s].H[k];
            if (trsf9) trsf9[k] = w->sp[s->s].trsf[k];
        }
    });
}

dem_status dem_step(dem_scene* s, int64_t nsteps)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        check_steppable(s, w);
        w->step(nsteps);
    });
}

dem_status dem_step_async(dem_scene* s, int64_t nsteps)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        check_steppable(s, w);
        if (nsteps < 0) dem::fail(DEM_EINVAL, "nsteps < 0");
        if (w->worker.joinable()) w->worker.join();
        w->async_rc = DEM_OK;
        w->async_msg.clear();
        w->busy.store(1);
        w->worker = std::thread([w, nsteps] {
            // the same guard as the synchronous call, on the worker thread;
            // its message is moved to the thread that calls dem_wait
            w->async_rc = guarded([&] {
                HIPC(hipSetDevice(w->device));
                w->step(nsteps);
            });
            w->async_msg = dem::g_err;
        });
    });
}

dem_status dem_wait(dem_scene* s)
{
    if (!s || !s->w) {
        dem::g_err = "null scene";
        return DEM_EINVAL;
    }
    dem::World* w = s->w;
    if (w->worker.joinable()) w->worker.join();
    const bool was_busy = w->busy.exchange(0) != 0;
    if (!was_busy) {
        dem::g_err.clear();
        return DEM_OK;
    }
    dem::g_err = w->async_msg;
    return w->async_rc;
}

dem_status dem_get_interaction(dem_scene* s, int64_t id1, int64_t id2, const int32_t* cell3, dem_contact* out)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!out) dem::fail(DEM_EINVAL, "null out");
        const int64_t nb = (int64_t)w->scenes[s->s].gids.size();
        if (id1 < 0 || id2 < 0 || id1 >= nb || id2 >= nb) dem::fail(DEM_ERANGE, "body id out of range");
        int32_t c[3] = {0, 0, 0};
        if (cell3)
            for (int q = 0; q < 3; ++q) c[q] = cell3[q];
        // symmetric lookup: the record keeps #1 = lower id (wall first), and
        // the image is that of #2 seen from #1
        const std::vector<dem_contact> all = w->contacts(s->s);
        for (const dem_contact& k : all) {
            if (k.id1 == id1 && k.id2 == id2 && k.cell[0] == c[0] && k.cell[1] == c[1] && k.cell[2] == c[2]) {
                *out = k;
                return;
            }
            if (k.id1 == id2 && k.id2 == id1 && k.cell[0] == -c[0] && k.cell[1] == -c[1] && k.cell[2] == -c[2]) {
                *out = k;
                return;
            }
        }
        dem::fail(DEM_ENOENT, "no real interaction between these bodies");
    });
}

dem_status dem_get_state(dem_scene* s, int64_t first_id, int64_t count, double* pos3, double* vel3, double* angvel3,
                         double* ori4, double* force3, double* torque3)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        w->get_state(s->s, first_id, count, pos3, vel3, angvel3, ori4, force3, torque3);
    });
}

dem_status dem_get_state_device(dem_scene* s, int64_t first_id, int64_t count, double* pos3, double* vel3,
                                double* angvel3, double* ori4)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        w->check_scene_id(s->s, first_id, count);
        std::vector<double> p(pos3 ? 3 * count : 0), v(vel3 ? 3 * count : 0), a(angvel3 ? 3 * count : 0),
            q(ori4 ? 4 * count : 0);
        w->get_state(s->s, first_id, count, pos3 ? p.data() : nullptr, vel3 ? v.data() : nullptr,
                     angvel3 ? a.data() : nullptr, ori4 ? q.data() : nullptr, nullptr, nullptr);
        auto put = [&](double* dst, const std::vector<double>& src) {
            if (dst && !src.empty())
                HIPC(hipMemcpyAsync(dst, src.data(), 8 * src.size(), hipMemcpyHostToDevice, w->stream));
        };
        put(pos3, p);
        put(vel3, v);
        put(angvel3, a);
        put(ori4, q);
        HIPC(hipStreamSynchronize(w->stream));
    });
}

dem_status dem_set_state(dem_scene* s, const double* pos3, const double* vel3, const double* angvel3,
                         const double* ori4)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        w->set_state(s->s, pos3, vel3, angvel3, ori4);
    });
}

dem_status dem_get_mass(dem_scene* s, double* mass, double* inertia)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        const auto& S = w->scenes[s->s];
        for (size_t i = 0; i < S.gids.size(); ++i) {
            const auto& b = w->bodies[S.gids[i]];
            if (mass) mass[i] = b.kind ? 0.0 : b.m;
            if (inertia) inertia[i] = b.kind ? 0.0 : 2.0 * b.m * b.r * b.r / 5.0;
        }
    });
}

dem_status dem_get_contacts(dem_scene* s, int64_t capacity, dem_contact* out, int64_t* out_count)
{
    dem_status rc = DEM_OK;
    dem_status g = guarded([&] {
        dem::World* w = world_of(s);
        if (!out_count) dem::fail(DEM_EINVAL, "null out_count");
        std::vector<dem_contact> c = w->contacts(s->s);
        *out_count = (int64_t)c.size();
        if (capacity < (int64_t)c.size()) {
            rc = DEM_ECAPACITY;
            return;
        }
        if (!c.empty()) {
            if (!out) dem::fail(DEM_EINVAL, "null out");
            std::memcpy(out, c.data(), sizeof(dem_contact) * c.size());
        }
    });
    if (g == DEM_OK && rc != DEM_OK) dem::g_err = "dem_get_contacts: buffer too small";
    return g != DEM_OK ? g : rc;
}

dem_status dem_get_history(dem_scene* s, int64_t capacity, dem_history* out, int64_t* out_count)
{
    dem_status rc = DEM_OK;
    dem_status g = guarded([&] {
        dem::World* w = world_of(s);
        if (!out_count) dem::fail(DEM_EINVAL, "null out_count");
        std::vector<dem_contact> c = w->contacts(s->s);
        *out_count = (int64_t)c.size();
        if (capacity < (int64_t)c.size()) {
            rc = DEM_ECAPACITY;
            return;
        }
        for (size_t i = 0; i < c.size(); ++i) {
            dem_history h;
            std::memset(&h, 0, sizeof h);
            h.id1 = c[i].id1;
            h.id2 = c[i].id2;
            for (int q = 0; q < 3; ++q) {
                h.cell[q] = c[i].cell[q];
                h.fs[q] = c[i].fs[q];
                h.nprev[q] = c[i].normal[q];
            }
            out[i] = h;
        }
    });
    if (g == DEM_OK && rc != DEM_OK) dem::g_err = "dem_get_history: buffer too small";
    return g != DEM_OK ? g : rc;
}

dem_status dem_set_history(dem_scene* s, int64_t n, const dem_history* in)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        w->set_history(s->s, n, in);
    });
}

dem_status dem_get_stress(dem_scene* s, double volume, double* sigma9)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!sigma9) dem::fail(DEM_EINVAL, "null out");
        w->stress(s->s, volume, sigma9);
    });
}

dem_status dem_get_stress_noalloc(dem_scene* s, double volume, double* sigma9)
{
    return guarded([&] {
        if (!sigma9) dem::fail(DEM_EINVAL, "null output");
        dem::World* w = world_of(s);
        w->stress_noalloc(s->s, volume, sigma9);
    });
}

dem_status dem_get_energy(dem_scene* s, dem_energy* out)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!out) dem::fail(DEM_EINVAL, "null out");
        if (w->scenes.size() > 1) dem::fail(DEM_EINVAL, "dem_get_energy: energies are tracked per world, not per batch scene");
        w->totals(out, nullptr, nullptr, nullptr);
    });
}

// Per-scene fields come from scene s (s < 0: totals over the batch); the
// contact counters are kept per world.
static void fill_stats(dem::World* w, int s, dem_stats* out)
{
    unsigned long long ss = 0, sw = 0, csteps = 0;
    w->totals(nullptr, &ss, &sw, &csteps);
    std::memset(out, 0, sizeof *out);
    int64_t nsph = 0, nw = 0;
    const int s0 = s < 0 ? 0 : s;
    out->iter = w->scenes[s0].iter;
    out->time = w->scenes[s0].time;
    out->verlet_dist = w->scenes[s0].verlet;
    for (int i = 0; i < (int)w->scenes.size(); ++i)
        if (s < 0 || i == s) {
            nsph += w->scenes[i].n_spheres;
            nw += w->scenes[i].n_walls;
        }
    int64_t all = 0;
    for (const auto& S : w->scenes) all += S.n_spheres;
    out->n_spheres = nsph;
    out->n_walls = nw;
    out->n_contacts_ss = (int64_t)ss;
    out->n_contacts_sw = (int64_t)sw;
    out->n_candidates = w->n_candidates;
    out->rebuilds = w->rebuilds;
    out->contact_steps = (int64_t)csteps;
    out->coordination = all ? 2.0 * (double)ss / (double)all : 0.0;
    out->max_overlap_ratio = w->max_overlap();
}

dem_status dem_get_unbalanced_force(dem_scene* s, int32_t use_max, double* out)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!out) dem::fail(DEM_EINVAL, "null output");
        *out = dem::World::unbalanced_of(w->measures(s->s), use_max != 0);
    });
}

dem_status dem_stiffness_dt(dem_scene* s, double safety, double* out)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!out) dem::fail(DEM_EINVAL, "null output");
        if (!(safety > 0.0) || !(safety <= 1.0)) dem::fail(DEM_EINVAL, "dem_stiffness_dt: safety in (0, 1]");
        *out = w->stiffness_dt(s->s, safety);
    });
}

dem_status dem_set_stiffness_timestepper(dem_scene* s, double safety, int64_t interval)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (w->scenes.size() > 1) dem::fail(DEM_EINVAL, "dem_set_stiffness_timestepper: not available for batch scenes");
        if (interval < 0) dem::fail(DEM_EINVAL, "dem_set_stiffness_timestepper: interval >= 0");
        if (interval > 0 && (!(safety > 0.0) || !(safety <= 1.0)))
            dem::fail(DEM_EINVAL, "dem_set_stiffness_timestepper: safety in (0, 1]");
        if (interval > 0 && w->has_viscel())
            dem::fail(DEM_EINVAL, "dem_set_stiffness_timestepper: not available with visco-elastic materials");
        w->ts_safety = safety;
        w->ts_interval = interval;
    });
}

void dem_peri_triax_default(dem_peri_triax* c)
{
    if (!c) return;
    std::memset(c, 0, sizeof *c);
    c->stress_mask = 7;
    c->glob_update = 5;
    for (int i = 0; i < 3; ++i) c->max_strain_rate[i] = 1.0;
    c->grow_damping = 0.25;
    c->max_unbalanced = 1e-4;
    c->abs_stress_tol = 1e3;
    c->rel_stress_tol = 3e-5;
}

void dem_peri_iso_default(dem_peri_iso* c)
{
    if (!c) return;
    std::memset(c, 0, sizeof *c);
    c->global_update = 20;
    c->max_strain_rate = 1.0;
    c->grow_damping = 0.25;
    c->max_unbalanced = 1e-4;
    c->abs_stress_tol = 1e3;
    c->rel_stress_tol = 3e-5;
}

dem_status dem_set_peri_iso(dem_scene* s, const dem_peri_iso* c)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!c) {
            w->set_peri_triax(nullptr);
            return;
        }
        if (w->has_viscel()) dem::fail(DEM_EINVAL, "dem_set_peri_iso: not available with visco-elastic materials");
        if (!w->scenes[s->s].p.periodic || w->scenes.size() > 1)
            dem::fail(DEM_EINVAL, "dem_set_peri_iso: needs an unbatched periodic scene");
        if (c->n_stresses < 1 || c->n_stresses > DEM_MAX_STRESS_SERIES)
            dem::fail(DEM_EINVAL, "dem_set_peri_iso: 1 to 8 stresses");
        for (int j = 0; j < c->n_stresses; ++j)
            if (!std::isfinite(c->stresses[j])) dem::fail(DEM_EINVAL, "dem_set_peri_iso: non-finite stress");
        if (c->global_update < 1) dem::fail(DEM_EINVAL, "dem_set_peri_iso: global_update >= 1");
        if (!(c->grow_damping >= 0.0 && c->grow_damping < 1.0)) dem::fail(DEM_EINVAL, "dem_set_peri_iso: grow_damping in [0, 1)");
        if (!(c->max_strain_rate > 0.0) || !std::isfinite(c->max_strain_rate))
            dem::fail(DEM_EINVAL, "dem_set_peri_iso: max_strain_rate > 0");
        if (!(c->abs_stress_tol >= 0.0) || !(c->rel_stress_tol >= 0.0) || std::isnan(c->max_unbalanced))
            dem::fail(DEM_EINVAL, "dem_set_peri_iso: tolerances >= 0");
        w->set_peri_iso(c);
    });
}

dem_status dem_get_peri_iso(dem_scene* s, dem_peri_iso_state* out)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!out) dem::fail(DEM_EINVAL, "null output");
        *out = w->peri_iso_state();
    });
}

dem_status dem_set_peri_triax(dem_scene* s, const dem_peri_triax* c)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!c) {
            w->set_peri_triax(nullptr);
            return;
        }
        if (w->has_viscel()) dem::fail(DEM_EINVAL, "dem_set_peri_triax: not available with visco-elastic materials");
        if (!w->scenes[s->s].p.periodic || w->scenes.size() > 1)
            dem::fail(DEM_EINVAL, "dem_set_peri_triax: needs an unbatched periodic scene");
        if (c->glob_update < 1) dem::fail(DEM_EINVAL, "dem_set_peri_triax: glob_update >= 1");
        if (c->stress_mask < 0 || c->stress_mask > 7) dem::fail(DEM_EINVAL, "dem_set_peri_triax: stress_mask in 0..7");
        if (!(c->grow_damping >= 0.0 && c->grow_damping < 1.0)) dem::fail(DEM_EINVAL, "dem_set_peri_triax: grow_damping in [0, 1)");
        for (int i = 0; i < 3; ++i) {
            if (!(c->max_strain_rate[i] > 0.0) || !std::isfinite(c->max_strain_rate[i]))
                dem::fail(DEM_EINVAL, "dem_set_peri_triax: max_strain_rate > 0");
            if (!std::isfinite(c->goal[i])) dem::fail(DEM_EINVAL, "dem_set_peri_triax: non-finite goal");
        }
        if (!(c->abs_stress_tol >= 0.0) || !(c->rel_stress_tol >= 0.0) || std::isnan(c->max_unbalanced))
            dem::fail(DEM_EINVAL, "dem_set_peri_triax: tolerances >= 0");
        w->set_peri_triax(c);
    });
}

dem_status dem_get_peri_triax(dem_scene* s, dem_peri_triax_state* out)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!out) dem::fail(DEM_EINVAL, "null output");
        *out = w->peri_triax_state();
    });
}

dem_status dem_get_stats(dem_scene* s, dem_stats* out)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!out) dem::fail(DEM_EINVAL, "null out");
        fill_stats(w, s->s, out);
    });
}

dem_status dem_set_timing(dem_scene* s, int32_t on)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        w->timing = on != 0;
        w->invalidate_graphs();
    });
}

dem_status dem_get_timing(dem_scene* s, const char* name, double* avg_ms, int64_t* launches)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!name) dem::fail(DEM_EINVAL, "null name");
        auto it = w->timers.find(name);
        const double tot = it == w->timers.end() ? 0.0 : it->second.total_ms;
        const int64_t n = it == w->timers.end() ? 0 : it->second.launches;
        if (avg_ms) *avg_ms = n ? tot / (double)n : 0.0;
        if (launches) *launches = n;
    });
}

dem_status dem_get_tuning(dem_scene* s, dem_tuning* out)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!out) dem::fail(DEM_EINVAL, "null out");
        *out = w->tuning();
    });
}

dem_status dem_set_tuning(dem_scene* s, const dem_tuning* t)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        if (!t) dem::fail(DEM_EINVAL, "null tuning");
        if (!s->owner) dem::fail(DEM_EINVAL, "dem_set_tuning: tune the batch, not one of its scenes");
        w->set_tuning(*t);
    });
}

dem_status dem_autotune(dem_scene* s, int64_t probe_steps, const char* cache_path, dem_tuning* out)
{
    return guarded([&] {
        dem::World* w = world_of(s);
        check_steppable(s, w);
        const dem_tuning t = w->autotune(probe_steps, cache_path);
        if (out) *out = t;
    });
}

dem_status dem_batch_create(int32_t n_scenes, const dem_params* per_scene, dem_batch** out)
{
    return guarded([&] {
        if (n_scenes < 1 || n_scenes > 65535 || !per_scene || !out) dem::fail(DEM_EINVAL, "dem_batch_create: bad arguments");
        for (int i = 0; i < n_scenes; ++i) {
            check_params(&per_scene[i]);
            if (per_scene[i].periodic) dem::fail(DEM_EINVAL, "dem_batch_create: periodic scenes cannot be batched");
        }
        std::unique_ptr<dem::World> w(new dem::World());
        w->init(n_scenes, per_scene);
        dem_batch* b = new dem_batch;
        b->w = w.release();
        b->views.resize(n_scenes);
        for (int i = 0; i < n_scenes; ++i) b->views[i] = dem_scene{b->w, i, false};
        *out = b;
    });
}

dem_status dem_batch_scene(dem_batch* b, int32_t i, dem_scene** view)
{
    return guarded([&] {
        if (!b || !view) dem::fail(DEM_EINVAL, "null argument");
        if (i < 0 || i >= (int32_t)b->views.size()) dem::fail(DEM_ERANGE, "scene index out of range");
        *view = &b->views[i];
    });
}

dem_status dem_batch_step(dem_batch* b, int64_t nsteps)
{
    return guarded([&] {
        if (!b) dem::fail(DEM_EINVAL, "null batch");
        HIPC(hipSetDevice(b->w->device));
        for (const auto& S : b->w->scenes)
            if (!(S.p.dt > 0.0)) dem::fail(DEM_EINVAL, "dem_batch_step: dt is not set");
        b->w->step(nsteps);
    });
}

dem_status dem_batch_stats(dem_batch* b, dem_stats* out)
{
    return guarded([&] {
        if (!b || !out) dem::fail(DEM_EINVAL, "null argument");
        HIPC(hipSetDevice(b->w->device));
        fill_stats(b->w, -1, out);
    });
}

dem_status dem_batch_set_tuning(dem_batch* b, const dem_tuning* t)
{
    return guarded([&] {
        if (!b || !t) dem::fail(DEM_EINVAL, "null argument");
        HIPC(hipSetDevice(b->w->device));
        b->w->set_tuning(*t);
    });
}

dem_status dem_batch_autotune(dem_batch* b, int64_t probe_steps, const char* cache_path, dem_tuning* out)
{
    return guarded([&] {
        if (!b) dem::fail(DEM_EINVAL, "null batch");
        HIPC(hipSetDevice(b->w->device));
        for (const auto& S : b->w->scenes)
            if (!(S.p.dt > 0.0)) dem::fail(DEM_EINVAL, "dem_batch_autotune: dt is not set");
        const dem_tuning t = b->w->autotune(probe_steps, cache_path);
        if (out) *out = t;
    });
}

dem_status dem_batch_destroy(dem_batch* b)
{
    return guarded([&] {
        if (!b) dem::fail(DEM_EINVAL, "null batch");
        (void)hipSetDevice(b->w->device);
        delete b->w;
        delete b;
    });
}

}  // extern "C"
