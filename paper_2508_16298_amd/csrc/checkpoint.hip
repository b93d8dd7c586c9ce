// Checkpoint and resume of one Markov chain.  The heat bath and the
// Metropolis uniform of trajectory k are drawn from counter-based streams
// (Philox4x32-10 keyed by the seed, the trajectory index in the counter;
// Methods, HQMC steps (i) and (iii)), so the lattice parameters, theta and the
// index of the next trajectory fix the rest of the chain: a chain resumed from
// a checkpoint repeats, bit for bit, the trajectories it would have run.
//
// File layout (little endian, 8-byte fields after the magic):
//   "QEDHMCK1"                       magic (8 bytes)
//   uint64 version = 1
//   int64  L, Nt
//   double dtau, t, J, K
//   uint64 seed
//   int64  action                    (qedhmc_action)
//   uint64 next_traj
//   uint64 n = 2 Nt L^2              number of angles
//   double theta[n]                  [d][tau][y][x]
//   uint64 FNV-1a 64 hash of every byte before it
// Written to "<path>.tmp" and renamed over <path>, so a crash never leaves a
// half-written checkpoint under the final name.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qedhmc_internal.h"

using namespace qh;

namespace {

constexpr char kMagic[8] = {'Q', 'E', 'D', 'H', 'M', 'C', 'K', '1'};
constexpr uint64_t kVersion = 1;
constexpr size_t kHeader = 8 + 8 * 11;  // magic + eleven 8-byte fields

uint64_t fnv1a(const unsigned char* p, size_t n) {
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; i++) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

template <typename T>
void put(std::vector<unsigned char>& b, T v) {
    unsigned char tmp[sizeof(T)];
    std::memcpy(tmp, &v, sizeof(T));
    b.insert(b.end(), tmp, tmp + sizeof(T));
}

template <typename T>
T get(const unsigned char* p) {
    T v;
    std::memcpy(&v, p, sizeof(T));
    return v;
}

qedhmc_status fail(qedhmc_status st, const std::string& msg) {
    set_error("checkpoint: " + msg);
    return st;
}

// read and verify a whole checkpoint file; params and next_traj from its header
qedhmc_status read_file(const char* path, std::vector<unsigned char>& buf, qedhmc_params& p, uint64_t& next,
                        uint64_t& n) {
    if (!path) return fail(QEDHMC_EINVAL, "null path");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(QEDHMC_EINVAL, std::string("cannot open ") + path);
    std::fseek(f, 0, SEEK_END);
    const long len = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    if (len < (long)(kHeader + 8)) {
        std::fclose(f);
        return fail(QEDHMC_EINVAL, "file too short");
    }
    buf.resize((size_t)len);
    const size_t got = std::fread(buf.data(), 1, buf.size(), f);
    std::fclose(f);
    if (got != buf.size()) return fail(QEDHMC_EINVAL, "short read");
    const unsigned char* b = buf.data();
    if (std::memcmp(b, kMagic, 8) != 0) return fail(QEDHMC_EINVAL, "not a checkpoint (magic)");
    if (get<uint64_t>(b + 8) != kVersion) return fail(QEDHMC_EINVAL, "unknown version");
    const int64_t L = get<int64_t>(b + 16), Nt = get<int64_t>(b + 24);
    if (L < 2 || L > 2048 || L % 2 || Nt < 1 || (uint64_t)L * L * Nt >= (1ull << 31))
        return fail(QEDHMC_EINVAL, "bad lattice in header");
    p.L = (int32_t)L;
    p.Nt = (int32_t)Nt;
    p.dtau = get<double>(b + 32);
    p.t = get<double>(b + 40);
    p.J = get<double>(b + 48);
    p.K = get<double>(b + 56);
    p.seed = get<uint64_t>(b + 64);
    const int64_t act = get<int64_t>(b + 72);
    if (act != QEDHMC_COMPACT && act != QEDHMC_NONCOMPACT) return fail(QEDHMC_EINVAL, "bad gauge action in header");
    p.action = (int32_t)act;
    p.reserved = 0;
    next = get<uint64_t>(b + 80);
    n = get<uint64_t>(b + 88);
    if (n != 2ull * L * L * Nt) return fail(QEDHMC_EINVAL, "angle count does not match the lattice");
    if (buf.size() != kHeader + 8 * n + 8) return fail(QEDHMC_EINVAL, "file length does not match the lattice");
    if (fnv1a(b, buf.size() - 8) != get<uint64_t>(b + buf.size() - 8))
        return fail(QEDHMC_EINVAL, "checksum mismatch (corrupt file)");
    return QEDHMC_OK;
}

bool same_params(const qedhmc_params& a, const qedhmc_params& b) {
    return a.L == b.L && a.Nt == b.Nt && std::memcmp(&a.dtau, &b.dtau, 8) == 0 && std::memcmp(&a.t, &b.t, 8) == 0 &&
           std::memcmp(&a.J, &b.J, 8) == 0 && std::memcmp(&a.K, &b.K, 8) == 0 && a.seed == b.seed &&
           a.action == b.action;
}

}  // namespace

extern "C" {

qedhmc_status qedhmc_checkpoint_save(qedhmc_t h, const double* theta, uint64_t next_traj, const char* path) {
    if (!h || !theta || !path) return fail(QEDHMC_EINVAL, "null argument");
    const uint64_t n = 2ull * h->lat.Nt * h->lat.Vs;
    std::vector<unsigned char> buf;
    buf.reserve(kHeader + 8 * n + 8);
    buf.insert(buf.end(), kMagic, kMagic + 8);
    put<uint64_t>(buf, kVersion);
    put<int64_t>(buf, h->p.L);
    put<int64_t>(buf, h->p.Nt);
    put<double>(buf, h->p.dtau);
    put<double>(buf, h->p.t);
    put<double>(buf, h->p.J);
    put<double>(buf, h->p.K);
    put<uint64_t>(buf, h->p.seed);
    put<int64_t>(buf, h->p.action);
    put<uint64_t>(buf, next_traj);
    put<uint64_t>(buf, n);
    const size_t at = buf.size();
    buf.resize(at + 8 * n);
    QH_HIP(hipMemcpyAsync(buf.data() + at, theta, 8 * n, hipMemcpyDeviceToHost, h->stream));
    QH_HIP(hipStreamSynchronize(h->stream));
    put<uint64_t>(buf, fnv1a(buf.data(), buf.size()));
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(QEDHMC_EINVAL, "cannot create " + tmp);
    const size_t wrote = std::fwrite(buf.data(), 1, buf.size(), f);
    const bool ok = wrote == buf.size() && std::fflush(f) == 0;
    if (std::fclose(f) != 0 || !ok) {
        std::remove(tmp.c_str());
        return fail(QEDHMC_EINVAL, "write failed: " + tmp);
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(QEDHMC_EINVAL, std::string("cannot rename onto ") + path);
    }
    return QEDHMC_OK;
}

qedhmc_status qedhmc_checkpoint_info(const char* path, qedhmc_params* params, uint64_t* next_traj) {
    if (!params || !next_traj) return fail(QEDHMC_EINVAL, "null argument");
    std::vector<unsigned char> buf;
    qedhmc_params p{};
    uint64_t next = 0, n = 0;
    QH_TRY(read_file(path, buf, p, next, n));
    *params = p;
    *next_traj = next;
    return QEDHMC_OK;
}

qedhmc_status qedhmc_checkpoint_load(qedhmc_t h, const char* path, double* theta, uint64_t* next_traj) {
    if (!h || !theta || !next_traj) return fail(QEDHMC_EINVAL, "null argument");
    std::vector<unsigned char> buf;
    qedhmc_params p{};
    uint64_t next = 0, n = 0;
    QH_TRY(read_file(path, buf, p, next, n));
    if (!same_params(p, h->p)) return fail(QEDHMC_EINVAL, "lattice parameters differ from the handle's");
    QH_HIP(hipMemcpyAsync(theta, buf.data() + kHeader, 8 * n, hipMemcpyHostToDevice, h->stream));
    QH_HIP(hipStreamSynchronize(h->stream));
    *next_traj = next;
    return QEDHMC_OK;
}

}  // extern "C"
