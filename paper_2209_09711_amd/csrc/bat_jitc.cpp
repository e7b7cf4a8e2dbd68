// bat_jitc: compiles one graph-specialised kernel source with hiprtc and
// writes the code object to a file.
//
//     bat_jitc <hiprtc library> <source file> <output file> <hiprtc option>...
//
// The library starts several of these as child processes when it compiles
// many kernels at once (the autotuner's candidates): hiprtc serialises the
// compilations of one process, separate processes run them side by side.
// The hiprtc library (the very file the calling process has loaded: a
// process may hold another ROCm's copy than the system's) and the options
// come from the command line, so that the code object is byte for byte the
// one an in-process compile makes.  Exit status 0 on success, 1 on a
// compile error (the log on stderr), 2 on a usage, library or file error.
#include <hip/hiprtc.h>

#include <dlfcn.h>

#include <cstdio>
#include <string>
#include <vector>

int main(int argc, char **argv)
{
    if (argc < 4) {
        fprintf(stderr, "usage: bat_jitc <hiprtc library> <source> <output> <option>...\n");
        return 2;
    }
    void *lib = dlopen(argv[1], RTLD_NOW | RTLD_LOCAL);
    if (!lib) {
        fprintf(stderr, "bat_jitc: %s\n", dlerror());
        return 2;
    }
    auto sym = [&](const char *name) { return dlsym(lib, name); };
    auto create = (decltype(&hiprtcCreateProgram))sym("hiprtcCreateProgram");
    auto compile = (decltype(&hiprtcCompileProgram))sym("hiprtcCompileProgram");
    auto log_size = (decltype(&hiprtcGetProgramLogSize))sym("hiprtcGetProgramLogSize");
    auto get_log = (decltype(&hiprtcGetProgramLog))sym("hiprtcGetProgramLog");
    auto code_size = (decltype(&hiprtcGetCodeSize))sym("hiprtcGetCodeSize");
    auto get_code = (decltype(&hiprtcGetCode))sym("hiprtcGetCode");
    auto destroy = (decltype(&hiprtcDestroyProgram))sym("hiprtcDestroyProgram");
    auto err_str = (decltype(&hiprtcGetErrorString))sym("hiprtcGetErrorString");
    if (!create || !compile || !log_size || !get_log || !code_size || !get_code || !destroy || !err_str) {
        fprintf(stderr, "bat_jitc: %s lacks the hiprtc entry points\n", argv[1]);
        return 2;
    }
    const char *out_path = argv[3];
    std::string src;
    {
        FILE *f = fopen(argv[2], "rb");
        if (!f) return 2;
        char buf[1 << 16];
        size_t k;
        while ((k = fread(buf, 1, sizeof buf, f)) > 0) src.append(buf, k);
        fclose(f);
    }
    hiprtcProgram prog;
    if (create(&prog, src.c_str(), "bat_jit.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) return 1;
    const hiprtcResult rc = compile(prog, argc - 4, (const char **)(argv + 4));
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        log_size(prog, &ls);
        std::string log(ls + 1, '\0');
        get_log(prog, &log[0]);
        fprintf(stderr, "%s: %s\n", err_str(rc), log.c_str());
        destroy(&prog);
        return 1;
    }
    size_t sz = 0;
    if (code_size(prog, &sz) != HIPRTC_SUCCESS || sz == 0) return 1;
    std::vector<char> code(sz);
    if (get_code(prog, code.data()) != HIPRTC_SUCCESS) return 1;
    destroy(&prog);
    // write beside the target, then rename: a reader never sees a partial file
    const std::string tmp = std::string(out_path) + ".part";
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return 2;
    const bool ok = fwrite(code.data(), 1, sz, f) == sz;
    if (fclose(f) != 0 || !ok || rename(tmp.c_str(), out_path) != 0) {
        remove(tmp.c_str());
        return 2;
    }
    return 0;
}
